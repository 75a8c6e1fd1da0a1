// Create-time kernels: friction table, road quantisation, triangle records,
// per-world bounding boxes and the per-world uniform road grid (counting
// sort: count -> exclusive scan -> scatter -> per-cell order by index).
#include "sf_dev.h"

// ---------------------------------------------------------------- friction
// Effective static mu against water film depth at 13.89 m/s for the three
// pavements (AC, SMA, OGFC), the paper's curves of Sec. "Weather-to-Friction
// Model Details" sampled at 0.1 mm from 0 to 0.8 mm.
__constant__ float c_mu_curve[3][9] = {
    {1.1048f, 1.0657f, 1.0161f, 0.9593f, 0.9039f, 0.8595f, 0.8302f, 0.8134f, 0.8044f},
    {1.2043f, 1.1618f, 1.1078f, 1.0461f, 0.9857f, 0.9374f, 0.9056f, 0.8874f, 0.8776f},
    {1.3368f, 1.2898f, 1.2301f, 1.1617f, 1.0948f, 1.0413f, 1.0061f, 0.9860f, 0.9753f}};

// Friction after rain: the class mu scaled by the pavement curve relative
// to its dry value; linear between samples, falling linearly to zero
// between 0.8 mm and full hydroplaning at 1 mm; floor 1e-3 (Sec. "Weather-
// to-Friction Module").  Computed in double: a create-time table.
__device__ double curve_ratio(int pav, double h) {
    const float *c = c_mu_curve[(pav >= 0 && pav < 3) ? pav : 0];
    double v;
    if (!(h > 0.0)) v = c[0];
    else if (h >= 1.0) v = 0.0;
    else if (h > 0.8) v = (double)c[8] * (1.0 - h) * 5.0;
    else {
        double x = h * 10.0;
        int i = (int)floor(x);
        if (i > 7) i = 7;
        double a = x - i;
        v = (double)c[i] + ((double)c[i + 1] - (double)c[i]) * a;
    }
    return v / (double)c[0];
}

__global__ void k_weather_mu(const float *mu_class, const float *film, const uint8_t *pav, int W,
                             int S, float *mu) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= W * S) return;
    int w = k / S;
    double h = film ? (double)film[w] : 0.0;
    double m = mu_class[k];
    if (h > 0.0) {
        m *= curve_ratio(pav ? pav[w] : 0, h);
        if (m < 1e-3) m = 1e-3;
    }
    mu[k] = (float)m;
}

void launch_weather_mu(const float *mu_class, const float *film, const uint8_t *pav, int W, int S,
                       float *mu_out, hipStream_t st) {
    int n = W * S;
    if (n == 0) return;
    k_weather_mu<<<(n + 255) / 256, 256, 0, st>>>(mu_class, film, pav, W, S, mu_out);
}

// ------------------------------------------------------------ road points
__global__ void k_quantise_roads(const float2 *xy, int2 *q, int P) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    float2 p = xy[k];
    q[k] = make_int2(qpos(p.x), qpos(p.y));
}

void launch_quantise_roads(const float2 *xy, int2 *q, int P, hipStream_t st) {
    if (P == 0) return;
    k_quantise_roads<<<(P + 255) / 256, 256, 0, st>>>(xy, q, P);
}

// -------------------------------------------------------------- triangles
// (v0, surface) (e1) (e2) (unit normal of e1 x e2) for Moller-Trumbore
__global__ void k_prep_tris(const float *v, const uint8_t *surf, float4 *tri, int T) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= T) return;
    const float *p = v + 9 * (size_t)k;
    f3 a = mk3(p[0], p[1], p[2]);
    f3 e1 = sub3(mk3(p[3], p[4], p[5]), a);
    f3 e2 = sub3(mk3(p[6], p[7], p[8]), a);
    f3 n = cross3(e1, e2);
    float L = sqrtf(dot3(n, n));
    n = L > 0.f ? mul3(n, 1.f / L) : mk3(0.f, 0.f, 1.f);
    tri[4 * (size_t)k + 0] = make_float4(a.x, a.y, a.z, (float)surf[k]);
    tri[4 * (size_t)k + 1] = make_float4(e1.x, e1.y, e1.z, 0.f);
    tri[4 * (size_t)k + 2] = make_float4(e2.x, e2.y, e2.z, 1.f);   // friction factor (1: the class value)
    tri[4 * (size_t)k + 3] = make_float4(n.x, n.y, n.z, 0.f);
}

// per-triangle friction factors into the triangles' fourth e2 component
// (null: every factor back to 1)
__global__ void k_tri_friction(const float *scale, float4 *tri, int T) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < T) tri[4 * (size_t)k + 2].w = scale ? scale[k] : 1.f;
}

void launch_tri_friction(const float *scale, float4 *tri, int T, hipStream_t st) {
    if (T > 0) k_tri_friction<<<(T + 255) / 256, 256, 0, st>>>(scale, tri, T);
}

void launch_prep_tris(const float *verts, const uint8_t *surf, float4 *tri, int T, hipStream_t st) {
    if (T == 0) return;
    k_prep_tris<<<(T + 255) / 256, 256, 0, st>>>(verts, surf, tri, T);
}

// ------------------------------------------------------------ world bbox
__global__ __launch_bounds__(256) void k_world_bbox(const int *roff, const float2 *xy,
                                                    const int *toff, const float *verts,
                                                    float4 *bbox) {
    int w = blockIdx.x;
    float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int k = roff[w] + threadIdx.x; k < roff[w + 1]; k += blockDim.x) {
        float2 p = xy[k];
        x0 = fminf(x0, p.x); x1 = fmaxf(x1, p.x);
        y0 = fminf(y0, p.y); y1 = fmaxf(y1, p.y);
    }
    for (int k = toff[w] + threadIdx.x; k < toff[w + 1]; k += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            float px = verts[9 * (size_t)k + 3 * c], py = verts[9 * (size_t)k + 3 * c + 1];
            x0 = fminf(x0, px); x1 = fmaxf(x1, px);
            y0 = fminf(y0, py); y1 = fmaxf(y1, py);
        }
    __shared__ float s[4][256];
    s[0][threadIdx.x] = x0; s[1][threadIdx.x] = y0; s[2][threadIdx.x] = x1; s[3][threadIdx.x] = y1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[0][threadIdx.x] = fminf(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fminf(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmaxf(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmaxf(s[3][threadIdx.x], s[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) bbox[w] = make_float4(s[0][0], s[1][0], s[2][0], s[3][0]);
}

void launch_world_bbox(const int *roff, const float2 *xy, const int *toff, const float *verts, int W,
                       float4 *bbox, hipStream_t st) {
    if (W == 0) return;
    k_world_bbox<<<W, 256, 0, st>>>(roff, xy, toff, verts, bbox);
}

// ------------------------------------------------------------------- grid
__device__ __forceinline__ int cell_x(const GridHdr &g, float x) {
    int c = (int)floorf((x - g.x0) * g.inv_cell);
    return c < 0 ? 0 : (c >= g.nx ? g.nx - 1 : c);
}
__device__ __forceinline__ int cell_y(const GridHdr &g, float y) {
    int c = (int)floorf((y - g.y0) * g.inv_cell);
    return c < 0 ? 0 : (c >= g.ny ? g.ny - 1 : c);
}

// Whether triangle (a, b, c), projected on the ground plane, may meet the
// cell [x0, x1] x [y0, y1]: false only when one of its edges separates the
// two, with the cell widened by 1 mm (far above the rounding of these
// coordinates), so no cell that a point of the triangle lies in is ever
// left out.  A degenerate projection keeps its whole bounding box.
__device__ __forceinline__ bool tri_meets_cell(const float *p, float x0, float y0, float x1, float y1) {
    const float ax = p[0], ay = p[1], bx = p[3], by = p[4], cx = p[6], cy = p[7];
    const float area2 = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
    if (fabsf(area2) < 1e-6f) return true;
    const float s = area2 > 0.f ? 1.f : -1.f;
    const float m = 1e-3f;
    x0 -= m; y0 -= m; x1 += m; y1 += m;
    const float vx[3] = {ax, bx, cx}, vy[3] = {ay, by, cy};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const float px = vx[e], py = vy[e];
        const float ex = vx[(e + 1) % 3] - px, ey = vy[(e + 1) % 3] - py;
        // s * cross(edge, q - p) >= 0 inside; the cell's corner that
        // maximises it
        const float nx = -s * ey, ny = s * ex;
        const float qx = nx > 0.f ? x1 : x0, qy = ny > 0.f ? y1 : y0;
        if (nx * (qx - px) + ny * (qy - py) < 0.f) return false;
    }
    return true;
}

// mode 0: count, mode 1: scatter through cursors (both take the same cells:
// those of the triangle's bounding box that the triangle itself meets)
template <int MODE>
__global__ void k_grid_tris(DevWorld Wd, const float *verts, int T, int *cnt_or_cursor, int *items) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= T) return;
    // world of triangle k: binary search over tri offsets
    int lo = 0, hi = Wd.W - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (Wd.toff[mid] <= k) lo = mid; else hi = mid - 1;
    }
    int w = lo;
    GridHdr g = Wd.tgrid[w];
    const float *p = verts + 9 * (size_t)k;
    float xa = fminf(p[0], fminf(p[3], p[6])), xb = fmaxf(p[0], fmaxf(p[3], p[6]));
    float ya = fminf(p[1], fminf(p[4], p[7])), yb = fmaxf(p[1], fmaxf(p[4], p[7]));
    int cx0 = cell_x(g, xa), cx1 = cell_x(g, xb), cy0 = cell_y(g, ya), cy1 = cell_y(g, yb);
    const bool one = cx0 == cx1 && cy0 == cy1;
    for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
            // cells at the grid's clamped border reach to infinity
            const float x0 = cx == 0 ? -INFINITY : g.x0 + (float)cx * g.cell;
            const float x1 = cx == g.nx - 1 ? INFINITY : g.x0 + (float)(cx + 1) * g.cell;
            const float y0 = cy == 0 ? -INFINITY : g.y0 + (float)cy * g.cell;
            const float y1 = cy == g.ny - 1 ? INFINITY : g.y0 + (float)(cy + 1) * g.cell;
            if (!one && !tri_meets_cell(p, x0, y0, x1, y1)) continue;
            int c = g.cbase + cy * g.nx + cx;
            if (MODE == 0) atomicAdd(&cnt_or_cursor[c], 1);
            else items[atomicAdd(&cnt_or_cursor[c], 1)] = k - Wd.toff[w];
        }
}

template <int MODE>
__global__ void k_grid_pts(DevWorld Wd, int P, int *cnt_or_cursor, int *items) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    int lo = 0, hi = Wd.W - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (Wd.roff[mid] <= k) lo = mid; else hi = mid - 1;
    }
    int w = lo;
    GridHdr g = Wd.grid[w];
    float2 p = Wd.road_xy[k];
    int c = g.cbase + cell_y(g, p.y) * g.nx + cell_x(g, p.x);
    if (MODE == 0) atomicAdd(&cnt_or_cursor[c], 1);
    else items[atomicAdd(&cnt_or_cursor[c], 1)] = k - Wd.roff[w];
}

void launch_grid_count(const DevWorld &Wd, const float *verts, int T, int P, int *tri_cnt,
                       int *pt_cnt, hipStream_t st) {
    if (T) k_grid_tris<0><<<(T + 255) / 256, 256, 0, st>>>(Wd, verts, T, tri_cnt, nullptr);
    if (P) k_grid_pts<0><<<(P + 255) / 256, 256, 0, st>>>(Wd, P, pt_cnt, nullptr);
}

void launch_grid_fill(const DevWorld &Wd, const float *verts, int T, int P, int *tri_cursor,
                      int *pt_cursor, int *tri_items, int *pt_items, hipStream_t st) {
    if (T) k_grid_tris<1><<<(T + 255) / 256, 256, 0, st>>>(Wd, verts, T, tri_cursor, tri_items);
    if (P) k_grid_pts<1><<<(P + 255) / 256, 256, 0, st>>>(Wd, P, pt_cursor, pt_items);
}

// order each cell's items by index (the scatter order is not
// deterministic).  Small cells (most of them, many empty) are sorted by one
// thread each in place; a cell with more than CELL_SORT_SMALL items goes to
// a list that persistent waves then take one cell at a time: a bitonic sort
// across the lanes up to 64 items, ranks counted against a copy in LDS up to
// CELL_SORT_LDS (items of a cell are distinct), an insertion sort on one
// lane beyond
#define CELL_SORT_SMALL 16
#define CELL_SORT_LDS 2048
__global__ void k_cell_sort_small(const int *start, int C, int *items, int *big_count, int *big) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int a = start[c], n = start[c + 1] - a;
    if (n > CELL_SORT_SMALL) {
        big[atomicAdd(big_count, 1)] = c;
        return;
    }
    for (int i = a + 1; i < a + n; ++i) {
        int v = items[i], j = i - 1;
        while (j >= a && items[j] > v) { items[j + 1] = items[j]; --j; }
        items[j + 1] = v;
    }
}

__global__ __launch_bounds__(256) void k_cell_sort_big(const int *start, int *items, const int *big_count,
                                                       const int *big) {
    __shared__ int buf[4][CELL_SORT_LDS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nb = *big_count;
    for (int q = blockIdx.x * 4 + wv; q < nb; q += gridDim.x * 4) {
        const int c = big[q];
        const int a = start[c], n = start[c + 1] - a;
        if (n <= 64) {
            unsigned v = lane < n ? (unsigned)items[a + lane] : 0xffffffffu;
            v = wave_sort_u32(v);
            if (lane < n) items[a + lane] = (int)v;
        } else if (n <= CELL_SORT_LDS) {
            int *b = buf[wv];
            for (int i = lane; i < n; i += 64) b[i] = items[a + i];
            wave_sync();
            for (int i = lane; i < n; i += 64) {
                const int v = b[i];
                int rank = 0;
                for (int j = 0; j < n; ++j) rank += b[j] < v;
                items[a + rank] = v;
            }
            wave_sync();   // the copy is reused by this wave's next cell
        } else if (lane == 0) {
            for (int i = a + 1; i < a + n; ++i) {
                int v = items[i], j = i - 1;
                while (j >= a && items[j] > v) { items[j + 1] = items[j]; --j; }
                items[j + 1] = v;
            }
        }
    }
}

static void cell_sort(const int *start, int C, int *items, int *work, hipStream_t st) {
    // work: [0] the count of large cells, [1..C] their list
    (void)hipMemsetAsync(work, 0, sizeof(int), st);
    k_cell_sort_small<<<(C + 255) / 256, 256, 0, st>>>(start, C, items, work, work + 1);
    k_cell_sort_big<<<1024, 256, 0, st>>>(start, items, work, work + 1);
}

__device__ __forceinline__ int world_of_cell(const GridHdr *grid, int W, int c) {
    int lo = 0, hi = W - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (grid[mid].cbase <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_pack_pts(DevWorld Wd, int C, const int *pt_items, int4 *pt_cell) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int r0 = Wd.roff[world_of_cell(Wd.grid, Wd.W, c)];
    for (int k = Wd.pt_cell_start[c]; k < Wd.pt_cell_start[c + 1]; ++k) {
        int idx = pt_items[k];
        int2 q = Wd.road_q[r0 + idx];
        pt_cell[k] = make_int4(q.x, q.y, idx, 0);
    }
}

// triangle records copied into cell order: a ray then reads contiguous
// candidates with no id -> record indirection
__global__ void k_pack_tris(DevWorld Wd, int C, const int *tri_items, float4 *rec) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int t0 = Wd.toff[world_of_cell(Wd.tgrid, Wd.W, c)];
    for (int k = Wd.tri_cell_start[c]; k < Wd.tri_cell_start[c + 1]; ++k) {
        const int id = tri_items[k];
        const float4 a = Wd.tri[4 * (size_t)(t0 + id)];
        const float4 b = Wd.tri[4 * (size_t)(t0 + id) + 1];
        const float4 e = Wd.tri[4 * (size_t)(t0 + id) + 2];
        rec[3 * (size_t)k] = make_float4(a.x, a.y, a.z, __int_as_float(id));
        rec[3 * (size_t)k + 1] = make_float4(b.x, b.y, b.z, a.w);
        rec[3 * (size_t)k + 2] = make_float4(e.x, e.y, e.z, e.w);
    }
}

// Chebyshev distance (in cells) from every point cell to the nearest cell
// holding road points: relaxation d = min(d, d(neighbour) + 1) until it
// settles (values only decrease and stay upper bounds, so in-place updates
// are safe).  The kNN search skips the rings closer than this distance.
__global__ __launch_bounds__(256) void k_occ(DevWorld Wd, int *occ) {
    const int w = blockIdx.x;
    const GridHdr g = Wd.grid[w];
    const int n = g.nx * g.ny;
    int *d = occ + g.cbase;
    for (int c = threadIdx.x; c < n; c += blockDim.x)
        d[c] = Wd.pt_cell_start[g.cbase + c + 1] > Wd.pt_cell_start[g.cbase + c] ? 0 : (1 << 20);
    __shared__ int changed;
    for (int it = 0; it < g.nx + g.ny + 2; ++it) {
        __syncthreads();
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const int x = c % g.nx, y = c / g.nx;
            int m = d[c];
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx, yy = y + dy;
                    if ((dx | dy) == 0 || xx < 0 || yy < 0 || xx >= g.nx || yy >= g.ny) continue;
                    m = min(m, __atomic_load_n(&d[yy * g.nx + xx], __ATOMIC_RELAXED) + 1);
                }
            if (m < d[c]) {
                __atomic_store_n(&d[c], m, __ATOMIC_RELAXED);
                changed = 1;
            }
        }
        __syncthreads();
        if (!changed) break;
    }
}

void launch_grid_finish(const DevWorld &Wd, int CT, int CP, int *tri_items, int *pt_items,
                        float4 *tri_rec, int4 *pt_cell, int *pt_occ, int *tri_work, int *pt_work,
                        hipStream_t st) {
    if (CT) {
        cell_sort(Wd.tri_cell_start, CT, tri_items, tri_work, st);
        k_pack_tris<<<(CT + 255) / 256, 256, 0, st>>>(Wd, CT, tri_items, tri_rec);
    }
    if (CP) {
        cell_sort(Wd.pt_cell_start, CP, pt_items, pt_work, st);
        k_pack_pts<<<(CP + 255) / 256, 256, 0, st>>>(Wd, CP, pt_items, pt_cell);
    }
    if (Wd.W) k_occ<<<Wd.W, 256, 0, st>>>(Wd, pt_occ);
}

// ------------------------------------------------------------------- scan
// exclusive prefix sum of n ints into out[0..n] (out[n] = total), three
// passes: per-block scan, scan of block totals, add block offsets
#define SCAN_BLOCK 256
#define SCAN_ITEMS 4

__device__ int block_scan_excl(int v, int *s, int &total) {
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s[wv] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        if (k < wv) base += s[k];
        tot += s[k];
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_local(const int *in, int *out, int n, int *bsum) {
    __shared__ int s[SCAN_BLOCK / 64];
    int base = blockIdx.x * SCAN_BLOCK * SCAN_ITEMS + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS], sum = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        sum += v[k];
    }
    int tot;
    int pre = block_scan_excl(sum, s, tot);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_blocks(int *bsum, int nb, int *total_out) {
    __shared__ int s[SCAN_BLOCK / 64];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
        int k = b0 + threadIdx.x;
        int v = k < nb ? bsum[k] : 0;
        int tot;
        int pre = block_scan_excl(v, s, tot);
        if (k < nb) bsum[k] = pre + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_add(int *out, int n, const int *bsum) {
    int base = blockIdx.x * SCAN_BLOCK * SCAN_ITEMS + threadIdx.x * SCAN_ITEMS;
    int add = bsum[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) out[base + k] += add;
}

void launch_scan(const int *in, int *out, int n, int *tmp, hipStream_t st) {
    int per = SCAN_BLOCK * SCAN_ITEMS;
    int nb = (n + per - 1) / per;
    if (nb == 0) {
        (void)hipMemsetAsync(out, 0, sizeof(int), st);
        return;
    }
    k_scan_local<<<nb, SCAN_BLOCK, 0, st>>>(in, out, n, tmp);
    k_scan_blocks<<<1, SCAN_BLOCK, 0, st>>>(tmp, nb, out + n);
    k_scan_add<<<nb, SCAN_BLOCK, 0, st>>>(out, n, tmp);
}

// ------------------------------------------------------------ world of agent
__global__ void k_world_of(const int *aoff, int W, int *world_of) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    for (int n = aoff[w]; n < aoff[w + 1]; ++n) world_of[n] = w;
}

void launch_world_of(const int *aoff, int W, int *world_of, hipStream_t st) {
    if (W == 0) return;
    k_world_of<<<(W + 255) / 256, 256, 0, st>>>(aoff, W, world_of);
}

// per agent, what the observation needs of its world (one read instead of
// world index then world arrays)
__global__ void k_agent_desc(const int *aoff, const int *roff, const GridHdr *grid, int W, int4 *agent_world,
                             GridHdr *agent_grid) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const int4 d = make_int4(aoff[w], aoff[w + 1] - aoff[w], roff[w], roff[w + 1] - roff[w]);
    const GridHdr g = grid[w];
    for (int n = aoff[w]; n < aoff[w + 1]; ++n) {
        agent_world[n] = d;
        agent_grid[n] = g;
    }
}

void launch_agent_desc(const int *aoff, const int *roff, const GridHdr *grid, int W, int4 *agent_world,
                       GridHdr *agent_grid, hipStream_t st) {
    if (W == 0) return;
    k_agent_desc<<<(W + 255) / 256, 256, 0, st>>>(aoff, roff, grid, W, agent_world, agent_grid);
}
