// The fused control-step kernel: one workgroup owns one world for all
// substeps of a control step (contacts never cross worlds, so no grid-wide
// synchronisation is needed).  World state lives in LDS across substeps;
// threads map to wheels for ray/suspension/tire work, to agents for the
// chassis, and to agent pairs for contact detection.
#include "sf_dev.h"

// ---------------------------------------------------------------- raycast
// body-frame mount point of wheel wh: selects between the four (uniform)
// parameter entries rather than an indexed read of the argument block,
// which would be a memory round trip on every substep
__device__ __forceinline__ f3 mount_of(const DevParams &P, int wh) {
    const float x = wh == 0 ? P.mount[0][0] : wh == 1 ? P.mount[1][0] : wh == 2 ? P.mount[2][0] : P.mount[3][0];
    const float y = wh == 0 ? P.mount[0][1] : wh == 1 ? P.mount[1][1] : wh == 2 ? P.mount[2][1] : P.mount[3][1];
    const float z = wh == 0 ? P.mount[0][2] : wh == 1 ? P.mount[1][2] : wh == 2 ? P.mount[2][2] : P.mount[3][2];
    return mk3(x, y, z);
}

// Ray-triangle test (Moller-Trumbore) on a packed record: v0, edges e1 and
// e2.  Every product-sum is an explicit fused multiply-add and the compiler
// may fuse nothing else, so a call rounds the same wherever it is inlined
// (the records of a ray sit at layout-dependent places in its batch).  The
// determinant's reciprocal is the hardware's (one ulp), and the barycentric
// and distance tests are taken together without branches: a wave runs the
// test for every record up to its lanes' longest list, so its cost is the
// instruction count.
__device__ __forceinline__ float mt_rec(const float4 &a, const float4 &b, const float4 &c, f3 m, f3 u,
                                        float ell) {
#pragma clang fp contract(off)
    const float pvx = fmaf(u.y, c.z, -(u.z * c.y));
    const float pvy = fmaf(u.z, c.x, -(u.x * c.z));
    const float pvz = fmaf(u.x, c.y, -(u.y * c.x));
    const float det = fmaf(b.x, pvx, fmaf(b.y, pvy, b.z * pvz));
    const float inv = __builtin_amdgcn_rcpf(det);
    const float tx = m.x - a.x, ty = m.y - a.y, tz = m.z - a.z;
    const float bu = fmaf(tx, pvx, fmaf(ty, pvy, tz * pvz)) * inv;
    const float qx = fmaf(ty, b.z, -(tz * b.y));
    const float qy = fmaf(tz, b.x, -(tx * b.z));
    const float qz = fmaf(tx, b.y, -(ty * b.x));
    const float bv = fmaf(u.x, qx, fmaf(u.y, qy, u.z * qz)) * inv;
    const float t = fmaf(c.x, qx, fmaf(c.y, qy, c.z * qz)) * inv;
    // NaN (a degenerate record) fails every comparison
    const bool ok = fabsf(det) >= 1e-12f && bu >= 0.f && bu <= 1.f && bv >= 0.f && bu + bv <= 1.f &&
                    t >= 0.f && t <= ell;
    return ok ? t : INFINITY;
}

struct RayHit {
    int hit, surf, tri;
    float t, mus;   // mus: the hit triangle's friction factor (1 on the ground)
    f3 n;
};

// record hit (t, id) of record k: the nearest distance so far and up to 4
// distinct triangle hits, in separate registers (an indexed array here
// would be placed in scratch memory), and the first hit's edge records
#define RAY_HIT(t_, id_, k_, b_, c_)                                                \
    do {                                                                            \
        const float th = (t_);                                                      \
        const int idh = (id_), kh = (k_);                                           \
        const bool nw = th < INFINITY && idh != i0 && idh != i1 && idh != i2 && idh != i3; \
        const bool s0 = nw && nh == 0, s1 = nw && nh == 1, s2 = nw && nh == 2,     \
                   s3 = nw && nh == 3;                                              \
        tmin = fminf(tmin, th);                                                     \
        t0 = s0 ? th : t0; i0 = s0 ? idh : i0; k0 = s0 ? kh : k0;                   \
        const float4 bh = (b_), ch = (c_);                                          \
        fb0 = s0 ? bh.x : fb0; fb1 = s0 ? bh.y : fb1; fb2 = s0 ? bh.z : fb2;        \
        fb3 = s0 ? bh.w : fb3; fc0 = s0 ? ch.x : fc0; fc1 = s0 ? ch.y : fc1;        \
        fc2 = s0 ? ch.z : fc2; fc3 = s0 ? ch.w : fc3;                               \
        t1 = s1 ? th : t1; i1 = s1 ? idh : i1; k1 = s1 ? kh : k1;                   \
        t2 = s2 ? th : t2; i2 = s2 ? idh : i2; k2 = s2 ? kh : k2;                   \
        t3 = s3 ? th : t3; i3 = s3 ? idh : i3; k3 = s3 ? kh : k3;                   \
        nh += nw ? 1 : 0;                                                           \
    } while (0)

// Nearest hit of the wheel ray against the ground plane z = 0 and the road
// triangles of the triangle-grid cells under the ray's footprint.  Hits
// within 0.1 mm of the nearest are one surface point: a road triangle wins
// over the ground, the lowest triangle index first.  One pass keeps up to 4
// distinct triangle hits in registers; more (stacked geometry) triggers a
// second pass that applies the same rule.  The record ranges of two cell
// rows are fetched together and their records tested in batches of 8 whose
// loads are all in flight at once (the rule does not depend on the order in
// which records are visited).
__device__ __forceinline__ RayHit raycast(const DevParams &P, const DevWorld &Wd, const GridHdr &g, bool any_tri,
                                        f3 m, f3 u) {
    const float ell = P.ell;
    float tg = INFINITY;
    if (u.z < 0.f) {
        const float t = m.z / (-u.z);
        if (t >= 0.f && t <= ell) tg = t;
    }
    RayHit H;
    H.tri = -1;
    H.surf = 0;
    H.t = tg;
    H.mus = 1.f;
    H.n = mk3(0.f, 0.f, 1.f);
    if (!any_tri) {
        H.hit = tg < INFINITY;
        return H;
    }
    const float ex = m.x + ell * u.x, ey = m.y + ell * u.y;
    int cx0 = (int)floorf((fminf(m.x, ex) - g.x0) * g.inv_cell);
    int cx1 = (int)floorf((fmaxf(m.x, ex) - g.x0) * g.inv_cell);
    int cy0 = (int)floorf((fminf(m.y, ey) - g.y0) * g.inv_cell);
    int cy1 = (int)floorf((fmaxf(m.y, ey) - g.y0) * g.inv_cell);
    cx0 = max(0, min(cx0, g.nx - 1)); cx1 = max(0, min(cx1, g.nx - 1));
    cy0 = max(0, min(cy0, g.ny - 1)); cy1 = max(0, min(cy1, g.ny - 1));
    float tmin = tg, t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f;
    int nh = 0, i0 = -1, i1 = -1, i2 = -1, i3 = -1, k0 = -1, k1 = -1, k2 = -1, k3 = -1;
    // edge records of the first hit (scalars: a selected float4 would be
    // placed in scratch memory)
    float fb0 = 0.f, fb1 = 0.f, fb2 = 0.f, fb3 = 0.f, fc0 = 0.f, fc1 = 0.f, fc2 = 0.f, fc3 = 0.f;
    // two cell rows at a time (the second empty unless the footprint spans it)
    for (int cy = cy0; cy <= cy1; cy += 2) {
        const int ca = g.cbase + cy * g.nx, cb = g.cbase + min(cy + 1, g.ny - 1) * g.nx;
        const int sA = Wd.tri_cell_start[ca + cx0], eA = Wd.tri_cell_start[ca + cx1 + 1];
        int sB = 0, eB = 0;
        if (cy < cy1) {
            sB = Wd.tri_cell_start[cb + cx0];
            eB = Wd.tri_cell_start[cb + cx1 + 1];
        }
        const int nA = eA - sA, nAB = nA + eB - sB;
        if (Wd.touch) {
            touch(Wd, SF_T_TRI_START, ca + cx0);
            touch(Wd, SF_T_TRI_START, ca + cx1 + 1);
            if (cy < cy1) {
                touch(Wd, SF_T_TRI_START, cb + cx0);
                touch(Wd, SF_T_TRI_START, cb + cx1 + 1);
            }
            for (int r = 0; r < nAB; ++r) touch(Wd, SF_T_TRI_REC, r < nA ? sA + r : sB + (r - nA));
        }
        for (int rb = 0; rb < nAB; rb += 8) {
            float4 ra[8], rbv[8], rc[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = rb + q;
                if (r < nAB) {
                    const size_t k = (size_t)(r < nA ? sA + r : sB + (r - nA));
                    ra[q] = Wd.tri_rec[3 * k];
                    rbv[q] = Wd.tri_rec[3 * k + 1];
                    rc[q] = Wd.tri_rec[3 * k + 2];
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = rb + q;
                if (r < nAB) {
                    const float t = mt_rec(ra[q], rbv[q], rc[q], m, u, ell);
                    RAY_HIT(t, __float_as_int(ra[q].w), r < nA ? sA + r : sB + (r - nA), rbv[q], rc[q]);
                }
            }
        }
    }
    H.hit = tmin < INFINITY;
    if (!H.hit || nh == 0) return H;
    int best = 0x7fffffff, bk = -1;
    float bt = 0.f;
    const float lim = tmin + 1e-4f;
    if (nh <= 4) {
        if (t0 <= lim && i0 < best) { best = i0; bt = t0; bk = k0; }
        if (nh > 1 && t1 <= lim && i1 < best) { best = i1; bt = t1; bk = k1; }
        if (nh > 2 && t2 <= lim && i2 < best) { best = i2; bt = t2; bk = k2; }
        if (nh > 3 && t3 <= lim && i3 < best) { best = i3; bt = t3; bk = k3; }
    } else {
        // more than 4 distinct triangles under one ray: apply the rule in a
        // second pass over the same cells
        for (int cy = cy0; cy <= cy1; ++cy) {
            const int c0 = g.cbase + cy * g.nx;
            const int s = Wd.tri_cell_start[c0 + cx0], e = Wd.tri_cell_start[c0 + cx1 + 1];
            for (int k = s; k < e; ++k) {
                const float4 a = Wd.tri_rec[3 * (size_t)k];
                const int id = __float_as_int(a.w);
                if (id >= best) continue;
                const float t = mt_rec(a, Wd.tri_rec[3 * (size_t)k + 1], Wd.tri_rec[3 * (size_t)k + 2], m, u, ell);
                if (t <= lim) { best = id; bt = t; bk = k; }
            }
        }
    }
    if (bk >= 0) {
        // the first hit wins in the common case: its records are at hand
        float4 b = make_float4(fb0, fb1, fb2, fb3), c = make_float4(fc0, fc1, fc2, fc3);
        if (bk != k0) {
            b = Wd.tri_rec[3 * (size_t)bk + 1];
            c = Wd.tri_rec[3 * (size_t)bk + 2];
        }
        f3 n = cross3(mk3(b.x, b.y, b.z), mk3(c.x, c.y, c.z));
        const float L = sqrtf(dot3(n, n));
        n = L > 0.f ? mul3(n, 1.f / L) : mk3(0.f, 0.f, 1.f);
        if (dot3(n, u) > 0.f) n = mul3(n, -1.f);
        H.t = bt;
        H.n = n;
        H.surf = (int)b.w;
        H.mus = c.w;
        H.tri = best;
    }
    return H;
}
#undef RAY_HIT

// ------------------------------------------------------------------ tire
// Linear-saturated tire in a friction circle with an implicit wheel-spin
// update and Coulomb brake (closed form).  K = c_kappa Fz / max(|vx|, v_eps)
// is the slip stiffness; the spin solve is implicit in it; forces outside
// the circle scale onto it and the spin then integrates the saturated force.
__device__ __forceinline__ void tire(const DevParams &P, float h, float Fz, float mu, float vx,
                                     float vy, float om, float td, float tb, float &Fx, float &Fy,
                                     float &om1) {
    float D = fmaxf(fabsf(vx), P.v_eps);
    float K = P.c_kappa * Fz / D;
    float Fy0 = -P.c_alpha * Fz * vy / D;
    float a = h / P.Iw;
    float B = om + a * (td + P.rw * K * vx);
    float Am = 1.f + a * P.rw * P.rw * K;
    float bb = a * tb;
    float os = B > bb ? (B - bb) / Am : (B < -bb ? (B + bb) / Am : 0.f);
    float Fx0 = K * (P.rw * os - vx);
    float lim = mu * Fz;
    float F2 = Fx0 * Fx0 + Fy0 * Fy0;
    if (F2 <= lim * lim) {
        Fx = Fx0;
        Fy = Fy0;
        om1 = os;
    } else {
        float sc = lim / sqrtf(F2);
        Fx = sc * Fx0;
        Fy = sc * Fy0;
        float Bs = om + a * (td - P.rw * Fx);
        float mag = fmaxf(fabsf(Bs) - bb, 0.f);
        om1 = Bs > 0.f ? mag : (Bs < 0.f ? -mag : 0.f);
    }
}

__device__ __forceinline__ f3 inv_inertia(const DevParams &P, const float R[9], f3 x) {
    f3 b = RTmul(R, x);
    b.x *= P.inv_inertia[0];
    b.y *= P.inv_inertia[1];
    b.z *= P.inv_inertia[2];
    return Rmul(R, b);
}

// ------------------------------------------------------ surrogate inference
#define SUR_LD 136    // row stride (bf16) of a wave's activation tile
#define SUR_ROWS 32   // rows per pass: half a wave's wheels
// LDS copy of the network: bf16 weights in padded rows (conflict-free
// fragment reads; W1's inputs 16..31 are zero so the first layer is one
// 32-deep product), then fp32 biases b1 b2 b3 b4
#define SURW_LD1 40
#define SURW_W2 (128 * SURW_LD1)
#define SURW_W3 (SURW_W2 + 128 * SUR_LD)
#define SURW_W4 (SURW_W3 + 128 * SUR_LD)
#define SURW_BF16 (SURW_W4 + 3 * SUR_LD)
#define SURW_NB (3 * 128 + 4)

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// One hidden layer for the tile's 16 RT rows (RT = 1 or 2), written back
// over its input.  The product is taken transposed, out^T = W in^T (weights
// as the row operand), so that each lane ends up with four consecutive
// outputs of one row: bias, ReLU, one packed bf16 conversion and one 8-byte
// store.
template <int KS, int RT>
__device__ __forceinline__ void sur_layer(uint16_t *buf, const uint16_t *W, int ldw, const float *bias) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[8][RT];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[n][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // every fragment of a 32-deep slice is read before its products are
    // issued, so that the LDS reads overlap one another
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 32 + kq * 8;
        bf16x8 x[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) x[t] = ld8(buf + (16 * t + r16) * SUR_LD + k0);
        bf16x8 w[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) w[n] = ld8(W + (n * 16 + r16) * ldw + k0);
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[n][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[n], x[t], acc[n][t], 0, 0, 0);
        // scheduling hint: the slice's LDS reads, then its products
        __builtin_amdgcn_sched_group_barrier(0x100, 8 + RT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 8 * RT, 0);
    }
    wave_sync();
    // lane holds out[row 16 t + lane % 16][16 n + 4 (lane / 16) + j]
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const float4 bb = *reinterpret_cast<const float4 *>(bias + n * 16 + kq * 4);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            bf16x4 o;
            o[0] = (__bf16)fmaxf(acc[n][t][0] + bb.x, 0.f);
            o[1] = (__bf16)fmaxf(acc[n][t][1] + bb.y, 0.f);
            o[2] = (__bf16)fmaxf(acc[n][t][2] + bb.z, 0.f);
            o[3] = (__bf16)fmaxf(acc[n][t][3] + bb.w, 0.f);
            *reinterpret_cast<bf16x4 *>(buf + (t * 16 + r16) * SUR_LD + n * 16 + kq * 4) = o;
        }
    }
    wave_sync();
}

// The three hidden layers and the 3-wide output layer for 16 RT rows of the
// tile.  The output is a product against W4 padded to 16 rows; its fp32
// results go to the row's padding columns, where the row's lane reads them.
template <int RT>
__device__ __forceinline__ void sur_pass(uint16_t *buf, const uint16_t *Wl, const float *bl) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
    sur_layer<1, RT>(buf, Wl, SURW_LD1, bl);
    sur_layer<4, RT>(buf, Wl + SURW_W2, SUR_LD, bl + 128);
    sur_layer<4, RT>(buf, Wl + SURW_W3, SUR_LD, bl + 256);
    f32x4 o[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) o[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int k0 = ks * 32 + kq * 8;
        const bf16x8 w = ld8(Wl + SURW_W4 + (r16 < 3 ? r16 : 0) * SUR_LD + k0);
        const bf16x8 wz = r16 < 3 ? w : zero8();
#pragma unroll
        for (int t = 0; t < RT; ++t)
            o[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(buf + (16 * t + r16) * SUR_LD + k0), wz, o[t], 0, 0, 0);
    }
    wave_sync();
    if (r16 < 3) {
        const float b4 = bl[384 + r16];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                reinterpret_cast<float *>(buf + (16 * t + kq * 4 + j) * SUR_LD + 128)[r16] = o[t][j] + b4;
    }
    wave_sync();
}

// The learned tire model on the wheels of one wave that are inside its
// domain, compacted: the k-th such wheel (in lane order) takes row k % 32 of
// pass k / 32, so that a wave runs one pass per 32 wheels that use the
// network (none when no wheel does; a pass of at most 16 rows runs one
// 16-row tile) and a row's result does not depend on the pass or tile it
// lands in; bf16 inputs and weights on the matrix cores, fp32 accumulation.
// Lanes outside the domain ignore y.
__device__ void sur_mlp_wave(uint16_t *buf, const float (&feat)[SF_SUR_IN], bool inside, const uint16_t *Wl,
                             const float *bl, float (&y)[3]) {
    const int lane = threadIdx.x & 63;
    const unsigned long long any = __ballot(inside);
    const int cnt = __popcll(any);
    const int pos = __popcll(any & ((1ull << lane) - 1ull));    // rank among the inside lanes
    y[0] = y[1] = y[2] = 0.f;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        const int rows = min(cnt - 32 * half, 32);
        if (rows <= 0) break;
        const int tile_rows = rows > 16 ? 32 : 16;
        if (inside && (pos >> 5) == half) {
            bf16x8 v0, v1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                v0[q] = (__bf16)feat[q];
                v1[q] = (__bf16)feat[8 + q];
            }
            bf16x8 *d = reinterpret_cast<bf16x8 *>(buf + (pos & 31) * SUR_LD);
            d[0] = v0;
            d[1] = v1;
            d[2] = zero8();
            d[3] = zero8();
        } else if (lane < tile_rows && lane >= rows) {
            // rows no wheel takes in this pass: zero inputs
            bf16x8 *d = reinterpret_cast<bf16x8 *>(buf + lane * SUR_LD);
            d[0] = d[1] = d[2] = d[3] = zero8();
        }
        wave_sync();
        if (tile_rows == 32) sur_pass<2>(buf, Wl, bl);
        else sur_pass<1>(buf, Wl, bl);
        if (inside && (pos >> 5) == half) {
            const float *yo = reinterpret_cast<const float *>(buf + (pos & 31) * SUR_LD + 128);
            y[0] = yo[0];
            y[1] = yo[1];
            y[2] = yo[2];
        }
        wave_sync();
    }
}

// Contact point of circle a of body i against circle b of body j (ab = 3a + b,
// the pair's mask bit): unit normal from i to j, midpoint of the two circle
// centres (height: mean of the bodies'), Baumgarte bias on the penetration
// past the slop.
struct CPoint {
    float nx, ny, px, py, pz, b;
};
__device__ __forceinline__ CPoint contact_point(const DevParams &P, float h, const float (*p)[SF_MAXA],
                                               const float *hx, const float *hy, int i, int j, int ab) {
    const int a = ab / 3, b = ab - 3 * a;
    const float cix = p[0][i] + (float)(a - 1) * P.cd * hx[i];
    const float ciy = p[1][i] + (float)(a - 1) * P.cd * hy[i];
    const float cjx = p[0][j] + (float)(b - 1) * P.cd * hx[j];
    const float cjy = p[1][j] + (float)(b - 1) * P.cd * hy[j];
    const float dx = cjx - cix, dy = cjy - ciy;
    const float L = sqrtf(dx * dx + dy * dy);
    CPoint c;
    c.nx = L > 0.f ? dx / L : 1.f;
    c.ny = L > 0.f ? dy / L : 0.f;
    c.px = 0.5f * (cix + cjx);
    c.py = 0.5f * (ciy + cjy);
    c.pz = 0.5f * (p[2][i] + p[2][j]);
    const float pen = 2.f * P.cr - L - P.slop;
    c.b = pen > 0.f ? (P.baumgarte / h) * pen : 0.f;
    return c;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    unsigned lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// (i, j), i < j, of the k-th pair in row-major order over A agents
__device__ __forceinline__ void pair_of(int k, int A, int &i, int &j) {
    float b = (float)(2 * A - 1);
    int ii = (int)((b - sqrtf(b * b - 8.f * (float)k)) * 0.5f);
    if (ii < 0) ii = 0;
    while (ii > 0 && ii * (2 * A - ii - 1) / 2 > k) --ii;
    while ((ii + 1) * (2 * A - ii - 2) / 2 <= k) ++ii;
    i = ii;
    j = k - ii * (2 * A - ii - 1) / 2 + ii + 1;
}

// Overlapping circle pairs (i < j, both active) of one world's A vehicles
// from their quantised centres, compacted by one wave with ballots into
// `pairs` in canonical (i, j) order, packed i | j << 8 | mask << 16 (mask
// bit 3a + b: circle a of i against circle b of j).  Every lane of the wave
// returns the number of pairs.
__device__ __forceinline__ int detect_pairs_wave(const DevParams &P, const int (*cq)[SF_MAXA], const int *act,
                                                 int A, uint32_t *pairs) {
    const int lane = threadIdx.x & 63;
    const int npc = A * (A - 1) / 2;
    const int pair_bound = (int)sqrtf((float)P.Qr2) + 2 + 2 * P.Qd;
    int np = 0;
    for (int base = 0; base < npc; base += 64) {
        const int k = base + lane;
        int flag = 0;
        uint32_t packed = 0;
        if (k < npc) {
            int i, j;
            pair_of(k, A, i, j);
            // centres farther apart than 2 (r + d) on either axis cannot
            // overlap; past that test every offset is below 2^13 units and
            // the squares fit 32-bit integers
            const int dX = cq[2][i] - cq[2][j], dY = cq[3][i] - cq[3][j];
            if (act[i] && act[j] && abs(dX) < pair_bound && abs(dY) < pair_bound) {
                uint32_t mask = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int dx = cq[2 * a][i] - cq[2 * b][j];
                        const int dy = cq[2 * a + 1][i] - cq[2 * b + 1][j];
                        if (dx * dx + dy * dy < P.Qr2) mask |= 1u << (3 * a + b);
                    }
                if (mask) {
                    flag = 1;
                    packed = (uint32_t)i | ((uint32_t)j << 8) | (mask << 16);
                }
            }
        }
        const unsigned long long bal = __ballot(flag);
        if (flag) pairs[np + __popcll(bal & lanemask_lt())] = packed;
        np += __popcll(bal);
    }
    return np;
}

// End of a control step for active agent n (slot i of world w): writes its
// new dynamic state dyn and friction seen, takes the sparse events on the
// quantised pose (Sec. "Reward Design Details": goal within 3 m, collision
// after the spawn warm-up, crash on falling, drifting or tilting), the
// time-out, reward and termination, then respawns or parks it
// (Sec. "Termination and time-out").
// Goal, start and step counters of an agent, read with its state at the
// start of the control step.
struct AgentTail {
    float gx, gy, sx, sy;
    int since, ep;
};
// A world's spawn entries [s0, s0 + M), read with its header.
struct SpawnRange {
    int s0, M;
};
__device__ __forceinline__ AgentTail load_tail(const float *st, const int *ist, int N, int n) {
    AgentTail a;
    a.gx = st[SF_F_GOAL_X * N + n];
    a.gy = st[SF_F_GOAL_Y * N + n];
    a.sx = st[SF_F_START_X * N + n];
    a.sy = st[SF_F_START_Y * N + n];
    a.since = ist[SF_I_SINCE_SPAWN * N + n];
    a.ep = ist[SF_I_EP_STEP * N + n];
    return a;
}

__device__ __forceinline__ void finish_agent(const DevParams &P, const DevWorld &Wd, float *st, int *ist, int N,
                                             int n, int w, int i, const float (&dyn)[SF_F_MU], float mu_seen,
                                             bool coll, bool nan_act, bool ovf, bool forbid, float2 p0,
                                             const AgentTail &tl, SpawnRange sr, float *reward,
                                             uint8_t *done, uint8_t *events) {
    bool finite = true;
    for (int c = 0; c < SF_F_MU; ++c) {
        st[c * N + n] = dyn[c];
        finite = finite && isfinite(dyn[c]);
    }
    st[SF_F_MU * N + n] = mu_seen;
    uint32_t ev = 0;
    if (!finite) {
        ev = SF_EV_CRASH | SF_EV_NUMERIC;
    } else {
        const long long X = qpos(dyn[SF_F_PX]), Y = qpos(dyn[SF_F_PY]), Z = qpos(dyn[SF_F_PZ]);
        const long long gx = X - qpos(tl.gx), gy = Y - qpos(tl.gy);
        if (gx * gx + gy * gy <= 3072ll * 3072ll) ev |= SF_EV_GOAL;
        if (coll && tl.since >= P.warmup) ev |= SF_EV_COLLISION;
        const long long sx = X - qpos(tl.sx), sy = Y - qpos(tl.sy);
        bool crash = sx * sx + sy * sy > 102400ll * 102400ll || Z < 0;
        const long long qx = qquat(dyn[SF_F_QX]), qy = qquat(dyn[SF_F_QY]);
        crash = crash || ((1ll << 28) - 2 * (qx * qx + qy * qy) < 40265318ll);
        if (crash) ev |= SF_EV_CRASH;
    }
    // road edge touched at the start of the step (shaping on)
    if (forbid && !(ev & SF_EV_NUMERIC)) ev |= SF_EV_LANE_FORBIDDEN;
    if (nan_act) ev |= SF_EV_NAN_ACTION;
    if (ovf) ev |= SF_EV_CONTACT_OVERFLOW;
    if (Wd.disp) Wd.disp[n] = make_float2(dyn[SF_F_PX] - p0.x, dyn[SF_F_PY] - p0.y);
    const int ep = tl.ep + 1;
    ist[SF_I_EP_STEP * N + n] = ep;
    ist[SF_I_SINCE_SPAWN * N + n] = tl.since + 1;
    if (ep >= P.max_ep) ev |= SF_EV_TIMEOUT;
    const float r = (ev & SF_EV_GOAL) ? 45.f : (ev & SF_EV_COLLISION) ? -6.f : (ev & SF_EV_CRASH) ? -10.f
                  : (ev & SF_EV_LANE_FORBIDDEN) ? -20.f : 0.f;
    const bool term = (ev & (SF_EV_GOAL | SF_EV_COLLISION | SF_EV_CRASH | SF_EV_LANE_FORBIDDEN)) != 0;
    const bool dn = (term && !(P.flags & SF_INVINCIBLE)) || (ev & (SF_EV_TIMEOUT | SF_EV_NUMERIC));
    reward[n] = r;
    done[n] = dn;
    events[n] = (uint8_t)ev;
    if (dn) {
        if (P.flags & SF_AUTO_RESET) {
            ist[SF_I_EPISODE * N + n] += 1;
            spawn_agent(P, Wd, st, ist, N, n, w, i, sr.s0, sr.M);
        } else {
            // parked off-stage at x = 1000 m at rest (Sec. "Termination and time-out")
            st[SF_F_PX * N + n] = 1000.f;
            st[SF_F_PY * N + n] = 0.f;
            st[SF_F_PZ * N + n] = P.z_ride;
            st[SF_F_QW * N + n] = 1.f;
            st[SF_F_QX * N + n] = 0.f;
            st[SF_F_QY * N + n] = 0.f;
            st[SF_F_QZ * N + n] = 0.f;
            for (int c = SF_F_VX; c <= SF_F_MU; ++c) st[c * N + n] = 0.f;
            ist[SF_I_ACTIVE * N + n] = 0;
        }
    }
}

// ---- A: steering PD (Eq. steer PD, implicit in the rate), rotation, planar
//      heading and the quantised three-circle centres of active agent i
//      (run for the first substep after the load, and for each later one
//      right after the previous substep's integration, by the same thread)
#define SF_PHASE_A(i)                                                                \
    do {                                                                             \
        float th = s_th[i], thd = s_thd[i], tgt = s_tgt[i];                          \
        float g = h / P.Is;                                                          \
        float thd1 = (thd + g * P.kp * (tgt - th)) / (1.f + g * (P.kd + h * P.kp));  \
        float tau = P.kp * (tgt - th - h * thd1) - P.kd * thd1;                      \
        if (fabsf(tau) > P.tau_max) {                                                \
            tau = tau > 0.f ? P.tau_max : -P.tau_max;                                \
            thd1 = thd + g * tau;                                                    \
        }                                                                            \
        s_th[i] = th + h * thd1;                                                     \
        s_thd[i] = thd1;                                                             \
        float R[9];                                                                  \
        quat_R(s_q[0][i], s_q[1][i], s_q[2][i], s_q[3][i], R);                       \
        for (int c = 0; c < 9; ++c) s_R[c][i] = R[c];                                \
        float L = sqrtf(R[0] * R[0] + R[3] * R[3]);                                  \
        s_hx[i] = L < 1e-12f ? 1.f : R[0] / L;                                       \
        s_hy[i] = L < 1e-12f ? 0.f : R[3] / L;                                       \
        int cq_[6];                                                                  \
        circle_centres_q(P, s_p[0][i], s_p[1][i], s_q[0][i], s_q[1][i], s_q[2][i],  \
                         s_q[3][i], cq_);                                            \
        for (int c = 0; c < 6; ++c) s_cq[c][i] = cq_[c];                             \
    } while (0)

// Two waves a SIMD for the plain step with more than one wave (its
// registers then stay within 256, so several worlds share a compute unit
// when the grid has more worlds than units); the learned tire model's LDS
// copy leaves room for one workgroup a unit anyway.
template <int BLOCK, bool SUR>
__global__ __launch_bounds__(BLOCK, SUR || BLOCK == 64 ? 1 : 2) void k_step(DevParams P, DevWorld Wd, DevSur Su, float *__restrict__ st,
                                                int *__restrict__ ist, const float *__restrict__ act,
                                                float h, int S, float *__restrict__ reward,
                                                uint8_t *__restrict__ done, uint8_t *__restrict__ events,
                                                uint32_t *__restrict__ rec, int *__restrict__ rec_cnt,
                                                int rec_cap, const int4 *__restrict__ items,
                                                int *__restrict__ queue) {
    constexpr int NWV = BLOCK / 64;
    const int N = Wd.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ float s_p[3][SF_MAXA], s_q[4][SF_MAXA], s_v[3][SF_MAXA], s_w[3][SF_MAXA];
    __shared__ float s_R[9][SF_MAXA];
    __shared__ float s_th[SF_MAXA], s_thd[SF_MAXA], s_taud[SF_MAXA], s_brk[SF_MAXA], s_tgt[SF_MAXA];
    __shared__ float s_hx[SF_MAXA], s_hy[SF_MAXA], s_muo[SF_MAXA];
    __shared__ int s_cq[6][SF_MAXA];
    __shared__ int s_act[SF_MAXA];
    __shared__ uint8_t s_coll[SF_MAXA], s_nan[SF_MAXA], s_forbid[SF_MAXA];
    __shared__ float2 s_p0[SF_MAXA];     // positions at the start of the control step
    __shared__ AgentTail s_tail[SF_MAXA];
    __shared__ SpawnRange s_spawn;
    __shared__ float s_om[4 * SF_MAXA];
    __shared__ float s_wf[6][4 * SF_MAXA];
    __shared__ float s_wmu[4 * SF_MAXA];
    __shared__ uint32_t s_pairs[SF_PAIR_CAP];
    __shared__ float s_cn[2][SF_CCAP], s_cpc[3][SF_CCAP], s_cwk[SF_CCAP], s_cb[SF_CCAP];
    __shared__ float s_clam[SF_CCAP], s_cdl[SF_CCAP];
    __shared__ int s_cij[SF_CCAP];
    __shared__ short s_bidx[2 * SF_CCAP];  // each body's contacts (CSR, list order)
    __shared__ int s_boff[SF_MAXA];
    __shared__ unsigned long long s_bmask[SF_MAXA];  // one-wave path: each body's contacts
    __shared__ int s_ovf;                  // contact points past SF_CCAP in a substep
    __shared__ float s_iw[6][SF_MAXA];   // world-frame inverse inertia (xx xy xz yy yz zz)
    __shared__ GridHdr s_tgrid;          // the world's triangle grid
    __shared__ float s_mu[SF_MAX_SURFACES];  // the world's friction per surface
    __shared__ bool s_anytri;
    __shared__ int s_bn[SF_MAXA];
    __shared__ int s_poff[BLOCK];        // first contact slot of each pair of a chunk
    __shared__ int s_scan[NWV];
    __shared__ int s_np;
    constexpr int NSW = NWV == 1 ? 1 : NWV - 1;  // waves that run wheels
    __shared__ __attribute__((aligned(16))) uint16_t s_sur[SUR ? NSW * SUR_ROWS * SUR_LD : 8];
    __shared__ __attribute__((aligned(16))) uint16_t s_surw[SUR ? SURW_BF16 : 8];
    __shared__ __attribute__((aligned(16))) float s_surb[SUR ? SURW_NB : 4];
    // wheels on the network / on the fallback in this workgroup (one global
    // update per workgroup at the end instead of one per wave and substep)
    __shared__ unsigned s_sur_cnt[2];
    if (SUR && tid < 2) s_sur_cnt[tid] = 0u;
    // the learned tire model's input envelope (lo then hi), read as vectors
    __shared__ __attribute__((aligned(16))) float s_env[SUR ? 2 * SF_SUR_IN : 4];
    if (SUR && tid < 2 * SF_SUR_IN) s_env[tid] = tid < SF_SUR_IN ? Su.lo[tid] : Su.hi[tid - SF_SUR_IN];
    // wheel mount points (an indexed read of the argument block per wheel
    // would be a memory gather on every substep)
    __shared__ float s_mount[12];
    if (tid < 12) s_mount[tid] = P.mount[tid / 3][tid % 3];

    if (SUR) {
        // the network's weights, once per block for all substeps: each matrix
        // as 16-byte chunks with shift-and-mask addressing (no per-chunk
        // branching), each block starting at its own chunk offset so that the
        // blocks' copies do not all hit the same memory lines at once, and
        // each thread's loads in flight before its stores
        const int rot = (int)(blockIdx.x % 64) * 64;
        // W2 and W3: 128 rows of 16 chunks, into rows of SUR_LD
        constexpr int N23 = (2048 + BLOCK - 1) / BLOCK;
        constexpr int B23 = N23 < 8 ? N23 : 8;
#pragma unroll 1
        for (int q0 = 0; q0 < N23; q0 += B23) {
            uint4 v2[B23], v3[B23];
#pragma unroll
            for (int q = 0; q < B23; ++q) {
                const int r = ((q0 + q) * BLOCK + tid + rot) & 2047;
                const int so = (r >> 4) * SF_SUR_HID + (r & 15) * 8;
                v2[q] = *reinterpret_cast<const uint4 *>(Su.Wb + SF_SURB_W2 + so);
                v3[q] = *reinterpret_cast<const uint4 *>(Su.Wb + SF_SURB_W3 + so);
            }
#pragma unroll
            for (int q = 0; q < B23; ++q) {
                const int r = ((q0 + q) * BLOCK + tid + rot) & 2047;
                const int d = (r >> 4) * SUR_LD + (r & 15) * 8;
                *reinterpret_cast<uint4 *>(s_surw + SURW_W2 + d) = v2[q];
                *reinterpret_cast<uint4 *>(s_surw + SURW_W3 + d) = v3[q];
            }
        }
        // W1: 128 rows of 16 inputs (2 chunks) then 16 zeros; W4: 3 rows of
        // 16 chunks
        for (int r = tid; r < 256 + 48; r += BLOCK) {
            if (r < 256) {
                const uint4 v = *reinterpret_cast<const uint4 *>(Su.Wb + SF_SURB_W1 + (r >> 1) * SF_SUR_IN + (r & 1) * 8);
                const int d = (r >> 1) * SURW_LD1 + (r & 1) * 8;
                *reinterpret_cast<uint4 *>(s_surw + d) = v;
                *reinterpret_cast<uint4 *>(s_surw + d + 16) = make_uint4(0u, 0u, 0u, 0u);
            } else {
                const int k = r - 256;
                const uint4 v = *reinterpret_cast<const uint4 *>(Su.Wb + SF_SURB_W4 + (k >> 4) * SF_SUR_HID + (k & 15) * 8);
                *reinterpret_cast<uint4 *>(s_surw + SURW_W4 + (k >> 4) * SUR_LD + (k & 15) * 8) = v;
            }
        }
        {
            float bv[(SURW_NB + BLOCK - 1) / BLOCK];
#pragma unroll
            for (int q = 0; q < (SURW_NB + BLOCK - 1) / BLOCK; ++q) {
                const int e = tid + q * BLOCK;
                bv[q] = e < 128 ? Su.P[SF_SUR_B1 + e] : e < 256 ? Su.P[SF_SUR_B2 + e - 128]
                      : e < 384 ? Su.P[SF_SUR_B3 + e - 256] : e < 387 ? Su.P[SF_SUR_B4 + e - 384] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < (SURW_NB + BLOCK - 1) / BLOCK; ++q)
                if (tid + q * BLOCK < SURW_NB) s_surb[tid + q * BLOCK] = bv[q];
        }
    }

    // Worlds in longest-first order, one descriptor each (world, first
    // agent, agents, any road triangles), so that the world's loads follow
    // a single read.  Without a queue, block b takes item b; with one (a
    // persistent grid smaller than W), a block that finishes a world takes
    // the next unclaimed item from an atomic counter.
    __shared__ int s_item;
    int item = blockIdx.x;
    while (item < Wd.W) {
        do {
            const int4 it = items[item];
            const int w = it.x, a0 = it.y, A = it.z;
            if (A <= 0) break;
            if (tid == 0) {
                s_tgrid = Wd.tgrid[w];
                s_anytri = it.w != 0;
                s_ovf = 0;
                const int s0 = Wd.soff[w];
                s_spawn = SpawnRange{s0, Wd.soff[w + 1] - s0};
            }
            if (tid < Wd.S) s_mu[tid] = Wd.mu[w * Wd.S + tid];
            // ---- load the world's agents; decode actions (Sec. "Action Space Details")
            for (int i = tid; i < A; i += BLOCK) {
                const int n = a0 + i;
                for (int c = 0; c < 3; ++c) {
                    s_p[c][i] = st[(SF_F_PX + c) * N + n];
                    s_v[c][i] = st[(SF_F_VX + c) * N + n];
                    s_w[c][i] = st[(SF_F_WX + c) * N + n];
                }
                for (int c = 0; c < 4; ++c) {
                    s_q[c][i] = st[(SF_F_QW + c) * N + n];
                    s_om[4 * i + c] = st[(SF_F_OM0 + c) * N + n];
                }
                s_th[i] = st[SF_F_STEER * N + n];
                s_thd[i] = st[SF_F_STEER_RATE * N + n];
                s_muo[i] = st[SF_F_MU * N + n];
                s_act[i] = ist[SF_I_ACTIVE * N + n];
                float al = act[2 * (size_t)n], sa = act[2 * (size_t)n + 1];
                uint8_t bad = 0;
                if (al != al) { al = 0.f; bad = 1; }
                if (sa != sa) { sa = 0.f; bad = 1; }
                al = fminf(fmaxf(al, -1.f), 1.f);
                s_taud[i] = al > 0.f ? al * P.tau_drive : 0.f;
                s_brk[i] = al < 0.f ? -al : 0.f;
                s_tgt[i] = fminf(fmaxf(sa, -P.steer_max), P.steer_max);
                s_nan[i] = bad;
                s_coll[i] = 0;
                s_forbid[i] = Wd.forbid ? Wd.forbid[n] : 0;
                s_p0[i] = make_float2(s_p[0][i], s_p[1][i]);
                s_tail[i] = load_tail(st, ist, N, n);
            }
            __syncthreads();

            for (int sub = 0; sub < S; ++sub) {
                const bool last = sub == S - 1;
                if (sub == 0) {
                    for (int i = tid; i < A; i += BLOCK)
                        if (s_act[i]) SF_PHASE_A(i);
                    __syncthreads();
                }

                // ---- B (last wave): overlapping circle pairs on the substep's input
                //      poses, compacted in canonical (i, j) order with wave ballots.
                // ---- C (the other waves; every thread when the block is one wave):
                //      wheels: raycast, suspension, tire, spin.  B and C overlap.
                const bool pair_wave = NWV == 1 || wave == NWV - 1;
                if (pair_wave) {
                    const int np_w = detect_pairs_wave(P, s_cq, s_act, A, s_pairs);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    if (rec) {
                        uint32_t *dst = rec + ((size_t)sub * Wd.W + w) * rec_cap;
                        for (int k = lane; k < np_w && k < rec_cap; k += 64) dst[k] = s_pairs[k];
                        if (lane == 0) rec_cnt[sub * Wd.W + w] = np_w;
                    }
                    for (int k = lane; k < np_w; k += 64) {
                        s_coll[s_pairs[k] & 0xFF] = 1;
                        s_coll[(s_pairs[k] >> 8) & 0xFF] = 1;
                    }
                    if (lane == 0) s_np = np_w;
                }
                const int wheel_threads = NWV == 1 ? BLOCK : BLOCK - 64;
                // the world's wheels spread evenly over the wheel waves (per_wave
                // consecutive wheels a wave and pass), so that a wave holds as
                // few wheels as the world allows: its ray test runs to the
                // longest record list of fewer lanes, and the learned tire model
                // runs fewer row passes
                const int npass = (4 * A + wheel_threads - 1) / wheel_threads;
                const int per_wave = (4 * A + npass * NSW - 1) / (npass * NSW);
                if (tid < wheel_threads) {
                    // the loop bound is the same for every lane of a wave (the
                    // surrogate's matrix products need the whole wave)
                    for (int pass = 0; pass < npass; ++pass) {
                        const int wi = (pass * NSW + wave) * per_wave + lane;
                        const bool valid = lane < per_wave && wi < 4 * A;
                        const int i = valid ? (wi >> 2) : 0, wh = wi & 3;
                        const bool live = valid && s_act[i];
                        float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                        float mu_seen = 0.f;
                        float R[9];
                        f3 v = mk3(0.f, 0.f, 0.f), om = v, rm = v, u = v, n = v, rc = v, ex = v, ey = v;
                        float Om = 0.f, td = 0.f, tb = 0.f, mu = 0.f, Fz = 0.f, vx = 0.f, vy = 0.f, x = 0.f, xd = 0.f, dl = 0.f;
                        bool hit = false, frame = false;
                        if (live) {
#pragma unroll
                            for (int c = 0; c < 9; ++c) R[c] = s_R[c][i];
                            const f3 pos = mk3(s_p[0][i], s_p[1][i], s_p[2][i]);
                            v = mk3(s_v[0][i], s_v[1][i], s_v[2][i]);
                            om = mk3(s_w[0][i], s_w[1][i], s_w[2][i]);
                            rm = Rmul(R, mk3(s_mount[3 * wh], s_mount[3 * wh + 1], s_mount[3 * wh + 2]));
                            u = mk3(-R[2], -R[5], -R[8]);
                            const RayHit H = raycast(P, Wd, s_tgrid, s_anytri, add3(pos, rm), u);
                            Om = s_om[wi];
                            td = wh < 2 ? s_taud[i] : 0.f;
                            tb = s_brk[i] * (wh < 2 ? P.tau_bf : P.tau_br);
                            hit = H.hit;
                            if (hit) {
                                n = H.n;
                                mu = s_mu[H.surf] * H.mus;
                                mu_seen = mu;
                                // massless spring-damper along the ray
                                x = P.ell - H.t;
                                const f3 vm = add3(v, cross3(om, rm));
                                xd = -dot3(n, vm) / (-dot3(n, u));
                                Fz = fmaxf(P.susp_k * x + P.susp_c * xd, 0.f);
                                rc = add3(rm, mul3(u, H.t));
                                // tire frame: wheel heading projected on the contact plane
                                dl = wh < 2 ? s_th[i] : 0.f;
                                const f3 hw = Rmul(R, mk3(cosf(dl), sinf(dl), 0.f));
                                ex = sub3(hw, mul3(n, dot3(hw, n)));
                                const float L = sqrtf(dot3(ex, ex));
                                if (L > 1e-9f) {
                                    frame = true;
                                    ex = mul3(ex, 1.f / L);
                                    ey = cross3(n, ex);
                                    const f3 vc = add3(v, cross3(om, rc));
                                    vx = dot3(vc, ex);
                                    vy = dot3(vc, ey);
                                } else {
                                    ex = mk3(0.f, 0.f, 0.f);
                                }
                            }
                        }
                        // the surrogate's domain: a loaded wheel at |v_x| >= 3 m/s
                        const bool dom = frame && Fz > 0.f && fabsf(vx) >= 3.f;
                        float feat[SF_SUR_IN];
                        if (SUR || Su.log) {
                            if (dom) {
                                const float D = fmaxf(fabsf(vx), P.v_eps), iD = 1.f / D;
                                const f3 axle = Rmul(R, mk3(-sinf(dl), cosf(dl), 0.f));
                                feat[0] = (P.rw * Om - vx) * iD;
                                feat[1] = atanf(vy * iD);
                                feat[2] = Fz * (1.f / 4000.f);
                                feat[3] = mu;
                                feat[4] = P.rw * Om * (1.f / 30.f);
                                feat[5] = asinf(fminf(fmaxf(dot3(axle, n), -1.f), 1.f));
                                feat[6] = vx * (1.f / 30.f);
                                feat[7] = vy * 0.2f;
                                feat[8] = dl;
                                feat[9] = x * 5.f;
                                feat[10] = xd * 0.5f;
                                feat[11] = td / P.tau_drive;
                                feat[12] = tb / P.tau_bf;
                                // the slip vector over mu, at most 2 long
                                float sx = 0.f, sy = 0.f;
                                if (mu > 0.f) {
                                    const float imu = 1.f / mu;
                                    sx = feat[0] * imu;
                                    sy = vy * iD * imu;
                                    const float L = sqrtf(sx * sx + sy * sy);
                                    if (L > 2.f) { sx *= 2.f / L; sy *= 2.f / L; }
                                }
                                feat[13] = sx;
                                feat[14] = sy;
                                feat[15] = om.z * 0.5f;
                            } else {
#pragma unroll
                                for (int q = 0; q < SF_SUR_IN; ++q) feat[q] = 0.f;
                            }
                        }
                        // ---- training samples: inputs and the plain model's outputs (before the
                        //      network, so that the features are not kept across it)
                        if (Su.log && valid) {
                            const long long slot = (Su.log_base + (long long)sub * 4 * N + 4ll * (a0 + i) + wh) % Su.log_cap;
                            float *dst = Su.log + slot * SF_SUR_SAMPLE;
                            if (dom) {
                                float Fxp, Fyp, omp;
                                tire(P, h, Fz, mu, vx, vy, Om, td, tb, Fxp, Fyp, omp);
                                const float lim = mu * Fz;
#pragma unroll
                                for (int q = 0; q < SF_SUR_IN; ++q) dst[q] = feat[q];
                                dst[SF_SUR_IN] = lim > 0.f ? Fxp / lim : 0.f;
                                dst[SF_SUR_IN + 1] = lim > 0.f ? Fyp / lim : 0.f;
                                dst[SF_SUR_IN + 2] = lim > 0.f ? -Fyp / lim : 0.f;
                                dst[SF_SUR_IN + 3] = 1.f;
                            } else {
                                dst[SF_SUR_IN + 3] = 0.f;
                            }
                        }
                        // ---- learned tire model for the wave's wheels, if enabled
                        bool use = false;
                        float Fxs = 0.f, Fys = 0.f, Mzs = 0.f;
                        if (SUR) {
                            bool inside = dom;
#pragma unroll
                            for (int q = 0; q < SF_SUR_IN; q += 4) {
                                const float4 lo = *reinterpret_cast<const float4 *>(s_env + q);
                                const float4 hi = *reinterpret_cast<const float4 *>(s_env + SF_SUR_IN + q);
                                inside = inside && feat[q] >= lo.x && feat[q] <= hi.x && feat[q + 1] >= lo.y &&
                                         feat[q + 1] <= hi.y && feat[q + 2] >= lo.z && feat[q + 2] <= hi.z &&
                                         feat[q + 3] >= lo.w && feat[q + 3] <= hi.w;
                            }
                            if (__ballot(inside)) {
                                float y[3];
                                sur_mlp_wave(s_sur + wave * SUR_ROWS * SUR_LD, feat, inside, s_surw, s_surb, y);
                                if (inside) {
                                    const float lim = mu * Fz;
                                    Fxs = lim * y[0];
                                    Fys = lim * y[1];
                                    Mzs = P.trail * lim * y[2];
                                    const float kap = (P.rw * Om - vx) / fabsf(vx);
                                    // residual checks: inside the friction circle (2 %
                                    // slack) and longitudinal force along the slip
                                    use = sqrtf(Fxs * Fxs + Fys * Fys) <= 1.02f * lim &&
                                          (fabsf(kap) <= 0.02f || ((Fxs > 0.f) == (kap > 0.f)));
                                }
                            }
                            // one counter update per wave, not per wheel
                            const unsigned long long bu = __ballot(dom && use), bf = __ballot(dom && !use);
                            if (lane == 0 && bu) atomicAdd(&s_sur_cnt[0], (unsigned)__popcll(bu));
                            if (lane == 0 && bf) atomicAdd(&s_sur_cnt[1], (unsigned)__popcll(bf));
                        }
                        if (live) {
                            float Fx = 0.f, Fy = 0.f, Mz = 0.f, om1;
                            if (frame) {
                                if (use) {
                                    Fx = Fxs;
                                    Fy = Fys;
                                    Mz = Mzs;
                                    const float a = h / P.Iw, Bs = Om + a * (td - P.rw * Fx);
                                    const float mag = fmaxf(fabsf(Bs) - a * tb, 0.f);
                                    om1 = Bs > 0.f ? mag : (Bs < 0.f ? -mag : 0.f);
                                } else {
                                    tire(P, h, Fz, mu, vx, vy, Om, td, tb, Fx, Fy, om1);
                                    Mz = -P.trail * Fy;
                                }
                            } else {
                                // airborne wheel or no usable tire frame: no load
                                tire(P, h, 0.f, hit ? mu : 0.f, 0.f, 0.f, Om, td, tb, Fx, Fy, om1);
                            }
                            if (hit) {
                                const f3 fw = add3(add3(mul3(n, Fz), mul3(ex, Fx)), mul3(ey, Fy));
                                const f3 tq = add3(cross3(rc, fw), mul3(n, Mz));
                                f[0] = fw.x; f[1] = fw.y; f[2] = fw.z;
                                f[3] = tq.x; f[4] = tq.y; f[5] = tq.z;
                            }
                            s_om[wi] = om1;
                        }
                        if (valid) {
#pragma unroll
                            for (int c = 0; c < 6; ++c) s_wf[c][wi] = f[c];
                            s_wmu[wi] = mu_seen;
                        }
                    }
                }

                __syncthreads();
                const int np = s_np;
                // A world with at most 64 contact points (one a lane) solves them on
                // wave 0, which holds every agent, with wave-level ordering only
                // (phases D to G below, then H, with no workgroup barrier); more
                // points take the workgroup-wide path.  Every wave reaches the
                // same choice from the pair list.
                int nsw = 0;
                if (np > 0 && np <= 64) nsw = wave_sum(lane < np ? __popc(s_pairs[lane] >> 16) : 0);
                const bool sw = np > 0 && np <= 64 && nsw <= 64;
                // ---- D: contact points of the compacted pairs, in list order
                int nc = 0;
                for (int base = 0; base < (sw ? 0 : np); base += BLOCK) {
                    const int k = base + tid;
                    uint32_t pr = k < np ? s_pairs[k] : 0u;
                    int cnt = __popc(pr >> 16);
                    int x = cnt;
                    for (int o = 1; o < 64; o <<= 1) {
                        int y = __shfl_up(x, o, 64);
                        if (lane >= o) x += y;
                    }
                    if (lane == 63) s_scan[wave] = x;
                    __syncthreads();
                    int off = 0, tot = 0;
#pragma unroll
                    for (int v = 0; v < NWV; ++v) {
                        if (v < wave) off += s_scan[v];
                        tot += s_scan[v];
                    }
                    // first contact slot of each pair of this chunk
                    if (k < np) s_poff[tid] = nc + off + x - cnt;
                    __syncthreads();
                    // one thread per (pair, circle combination) present in the
                    // pair's mask; its slot is the pair's first plus the number
                    // of the mask's lower bits (the list order is unchanged)
                    const int npk = min(np - base, BLOCK);
                    for (int t = tid; t < 9 * npk; t += BLOCK) {
                        const int kk = t / 9, ab = t - 9 * kk;
                        const uint32_t prk = s_pairs[base + kk];
                        const uint32_t mask = prk >> 16;
                        if (!(mask & (1u << ab))) continue;
                        const int pos = s_poff[kk] + __popc(mask & ((1u << ab) - 1u));
                        if (pos < SF_CCAP) {
                            const int i = prk & 0xFF, j = (prk >> 8) & 0xFF;
                            const CPoint cp = contact_point(P, h, s_p, s_hx, s_hy, i, j, ab);
                            s_cn[0][pos] = cp.nx;
                            s_cn[1][pos] = cp.ny;
                            s_cpc[0][pos] = cp.px;
                            s_cpc[1][pos] = cp.py;
                            s_cpc[2][pos] = cp.pz;
                            s_cb[pos] = cp.b;
                            s_clam[pos] = 0.f;
                            s_cij[pos] = i | (j << 8);
                        }
                    }
                    nc += tot;
                    __syncthreads();
                }
                // points past the world's capacity are left out of the solve
                // for both bodies (momentum stays exact) and reported
                if (nc > SF_CCAP) {
                    if (tid == 0) {
                        s_ovf = 1;
                        if (Wd.ovf) atomicAdd(Wd.ovf, 1ull);
                    }
                    nc = SF_CCAP;
                }
                // (np, nc and sw are the same in every thread: without pairs, or on
                //  the one-wave path, D wrote nothing)
                if (np > 0 && !sw) __syncthreads();

                // ---- E: chassis velocities (semi-implicit Euler, explicit gyroscopic
                //      term) and each body's contact list in list order
                for (int i = tid; i < A; i += BLOCK) {
                    if (!s_act[i]) { s_bn[i] = 0; continue; }
                    float R[9];
#pragma unroll
                    for (int c = 0; c < 9; ++c) R[c] = s_R[c][i];
                    f3 F = mk3(0.f, 0.f, -P.mass * P.g);
                    f3 T = mk3(0.f, 0.f, -P.yaw_damping * s_w[2][i]);
#pragma unroll
                    for (int wh = 0; wh < 4; ++wh) {
                        const int wi = 4 * i + wh;
                        F = add3(F, mk3(s_wf[0][wi], s_wf[1][wi], s_wf[2][wi]));
                        T = add3(T, mk3(s_wf[3][wi], s_wf[4][wi], s_wf[5][wi]));
                    }
                    if (last) s_muo[i] = (s_wmu[4 * i] + s_wmu[4 * i + 1] + s_wmu[4 * i + 2] + s_wmu[4 * i + 3]) * 0.25f;
                    const f3 om = mk3(s_w[0][i], s_w[1][i], s_w[2][i]);
                    const f3 wb = RTmul(R, om), Tb = RTmul(R, T);
                    const f3 Lb = mk3(P.inertia[0] * wb.x, P.inertia[1] * wb.y, P.inertia[2] * wb.z);
                    const f3 gy = cross3(wb, Lb);
                    const f3 wb1 = mk3(wb.x + h * (Tb.x - gy.x) * P.inv_inertia[0],
                                       wb.y + h * (Tb.y - gy.y) * P.inv_inertia[1],
                                       wb.z + h * (Tb.z - gy.z) * P.inv_inertia[2]);
                    const f3 om1 = Rmul(R, wb1);
                    for (int c = 0; c < 3; ++c) s_v[c][i] += h * (&F.x)[c] * P.inv_mass;
                    s_w[0][i] = om1.x; s_w[1][i] = om1.y; s_w[2][i] = om1.z;
                    // R diag(1/I) R^T, for the contact solve
                    {
                        const float a0 = P.inv_inertia[0], a1 = P.inv_inertia[1], a2 = P.inv_inertia[2];
                        s_iw[0][i] = R[0] * R[0] * a0 + R[1] * R[1] * a1 + R[2] * R[2] * a2;
                        s_iw[1][i] = R[0] * R[3] * a0 + R[1] * R[4] * a1 + R[2] * R[5] * a2;
                        s_iw[2][i] = R[0] * R[6] * a0 + R[1] * R[7] * a1 + R[2] * R[8] * a2;
                        s_iw[3][i] = R[3] * R[3] * a0 + R[4] * R[4] * a1 + R[5] * R[5] * a2;
                        s_iw[4][i] = R[3] * R[6] * a0 + R[4] * R[7] * a1 + R[5] * R[8] * a2;
                        s_iw[5][i] = R[6] * R[6] * a0 + R[7] * R[7] * a1 + R[8] * R[8] * a2;
                    }
                    int cnt = 0;
                    for (int c = 0; c < nc; ++c) {
                        const int ij = s_cij[c];
                        cnt += ((ij & 0xFF) == i) | (((ij >> 8) & 0xFF) == i);
                    }
                    s_bn[i] = cnt;
                }

                if (sw) {
                    if (wave == 0) {
                        // ---- D on one wave: pair k (lane k) takes contact slots from
                        //      the prefix sum of its mask's bits, in list order
                        wave_sync();
                        const bool own = lane < nsw;
                        // all contacts of one pair: the short solve below
                        const bool one_pair = np == 1 && nsw <= 16;   // a pair has at most 16 points
                        uint32_t kpr = s_pairs[0];
                        int koff = 0;
                        if (!one_pair) {
                            const uint32_t pr = lane < np ? s_pairs[lane] : 0u;
                            const int pcnt = __popc(pr >> 16);
                            int incl = pcnt;
#pragma unroll
                            for (int o = 1; o < 64; o <<= 1) {
                                const int y = __shfl_up(incl, o, 64);
                                if (lane >= o) incl += y;
                            }
                            const int poff = incl - pcnt;
                            for (int q = 0; q < pcnt; ++q) s_poff[poff + q] = lane;
                            if (lane < A) s_bmask[lane] = 0ull;
                            wave_sync();
                            const int kq = own ? s_poff[lane] : 0;
                            koff = __shfl(poff, kq, 64);
                            kpr = __shfl((int)pr, kq, 64);
                        }
                        int ci = 0, cj = 0;
                        float cnx = 0.f, cny = 0.f, cbb = 0.f, cwk = 0.f, clam = 0.f;
                        f3 cri = mk3(0.f, 0.f, 0.f), crj = cri;
                        if (own) {
                            // the (lane - koff)-th set bit of the pair's mask
                            uint32_t m = kpr >> 16;
                            for (int r = lane - koff; r > 0; --r) m &= m - 1u;
                            ci = kpr & 0xFF;
                            cj = (kpr >> 8) & 0xFF;
                            const CPoint cp = contact_point(P, h, s_p, s_hx, s_hy, ci, cj, __ffs(m) - 1);
                            cnx = cp.nx;
                            cny = cp.ny;
                            cbb = cp.b;
                            cri = sub3(mk3(cp.px, cp.py, cp.pz), mk3(s_p[0][ci], s_p[1][ci], s_p[2][ci]));
                            crj = sub3(mk3(cp.px, cp.py, cp.pz), mk3(s_p[0][cj], s_p[1][cj], s_p[2][cj]));
                            if (!one_pair) {
                                s_cn[0][lane] = cp.nx;
                                s_cn[1][lane] = cp.ny;
                                s_cpc[0][lane] = cp.px;
                                s_cpc[1][lane] = cp.py;
                                s_cpc[2][lane] = cp.pz;
                                s_cij[lane] = ci | (cj << 8);
                                // each body's contacts as a bit set over the list
                                atomicOr(&s_bmask[ci], 1ull << lane);
                                atomicOr(&s_bmask[cj], 1ull << lane);
                            }
                        }
                        if (one_pair) {
                            // ---- F and G for one pair (bodies bi, bj): every contact
                            //      belongs to both, so the contact lanes keep both
                            //      bodies' velocities themselves and sum the contacts'
                            //      impulses across the row, with no trip through LDS
                            const int bi = s_pairs[0] & 0xFF, bj = (s_pairs[0] >> 8) & 0xFF;
                            if (own) {
                                float Ri[9], Rj[9];
#pragma unroll
                                for (int q = 0; q < 9; ++q) { Ri[q] = s_R[q][ci]; Rj[q] = s_R[q][cj]; }
                                const f3 n = mk3(cnx, cny, 0.f);
                                const f3 xi = cross3(cri, n), xj = cross3(crj, n);
                                const float keff = 2.f * P.inv_mass + dot3(xi, inv_inertia(P, Ri, xi)) +
                                                   dot3(xj, inv_inertia(P, Rj, xj));
                                cwk = 1.f / ((float)nsw * keff);
                            }
                            float vix = s_v[0][bi], viy = s_v[1][bi], wix = s_w[0][bi], wiy = s_w[1][bi],
                                  wiz = s_w[2][bi];
                            float vjx = s_v[0][bj], vjy = s_v[1][bj], wjx = s_w[0][bj], wjy = s_w[1][bj],
                                  wjz = s_w[2][bj];
                            float ii[6], ij[6];
#pragma unroll
                            for (int q = 0; q < 6; ++q) { ii[q] = s_iw[q][bi]; ij[q] = s_iw[q][bj]; }
                            for (int it = 0; it < P.jacobi_iters; ++it) {
                                float dl = 0.f;
                                if (own) {
                                    const f3 wi = cross3(mk3(wix, wiy, wiz), cri);
                                    const f3 wj = cross3(mk3(wjx, wjy, wjz), crj);
                                    const float vn = ((vjx + wj.x) - (vix + wi.x)) * cnx + ((vjy + wj.y) - (viy + wi.y)) * cny;
                                    const float lam1 = fmaxf(clam + cwk * (-vn + cbb), 0.f);
                                    dl = lam1 - clam;
                                    clam = lam1;
                                }
                                // this contact's impulse on bj (along +n) and on bi (-n),
                                // with their torques, summed over the pair's contacts
                                // (at most 16, lanes 0-15: one DPP row) and handed to
                                // every lane
                                const float Jx = dl * cnx, Jy = dl * cny;
                                float sm[8] = {Jx, Jy, -(crj.z * Jy), crj.z * Jx, crj.x * Jy - crj.y * Jx,
                                               cri.z * Jy, -(cri.z * Jx), -(cri.x * Jy - cri.y * Jx)};
#pragma unroll
                                for (int q = 0; q < 8; ++q) sm[q] = row0_sum(sm[q]);
                                vix -= sm[0] * P.inv_mass;
                                viy -= sm[1] * P.inv_mass;
                                wix += ii[0] * sm[5] + ii[1] * sm[6] + ii[2] * sm[7];
                                wiy += ii[1] * sm[5] + ii[3] * sm[6] + ii[4] * sm[7];
                                wiz += ii[2] * sm[5] + ii[4] * sm[6] + ii[5] * sm[7];
                                vjx += sm[0] * P.inv_mass;
                                vjy += sm[1] * P.inv_mass;
                                wjx += ij[0] * sm[2] + ij[1] * sm[3] + ij[2] * sm[4];
                                wjy += ij[1] * sm[2] + ij[3] * sm[3] + ij[4] * sm[4];
                                wjz += ij[2] * sm[2] + ij[4] * sm[3] + ij[5] * sm[4];
                            }
                            if (lane == 0) {
                                s_v[0][bi] = vix;
                                s_v[1][bi] = viy;
                                s_w[0][bi] = wix;
                                s_w[1][bi] = wiy;
                                s_w[2][bi] = wiz;
                                s_v[0][bj] = vjx;
                                s_v[1][bj] = vjy;
                                s_w[0][bj] = wjx;
                                s_w[1][bj] = wjy;
                                s_w[2][bj] = wjz;
                            }
                            wave_sync();
                        } else {
                        wave_sync();
                        // ---- F: effective mass, relaxed by the larger contact count
                        if (own) {
                            float Ri[9], Rj[9];
#pragma unroll
                            for (int q = 0; q < 9; ++q) { Ri[q] = s_R[q][ci]; Rj[q] = s_R[q][cj]; }
                            const f3 n = mk3(cnx, cny, 0.f);
                            const f3 xi = cross3(cri, n), xj = cross3(crj, n);
                            const float keff = 2.f * P.inv_mass + dot3(xi, inv_inertia(P, Ri, xi)) +
                                               dot3(xj, inv_inertia(P, Rj, xj));
                            const int nmax = max(__popcll(s_bmask[ci]), __popcll(s_bmask[cj]));
                            cwk = 1.f / ((float)nmax * keff);
                        }
                        // body lane b: its first SW_K contacts in list order with their
                        // normals (signed toward the body: the sign flip is exact) and
                        // lever arms, its velocities and inertia
                        constexpr int SW_K = 9;
                        const int b = lane;
                        unsigned long long bm = b < A ? s_bmask[b] : 0ull;
                        const int bcnt = __popcll(bm);
                        const int kmax = wave_max(min(bcnt, SW_K));
                        int kc[SW_K];
                        float kx[SW_K], ky[SW_K], krx[SW_K], kry[SW_K], krz[SW_K];
                        const float pbx = b < A ? s_p[0][b] : 0.f, pby = b < A ? s_p[1][b] : 0.f,
                                    pbz = b < A ? s_p[2][b] : 0.f;
                        // the slots' contact indices first (bit operations only),
                        // then every slot's reads at once (a slot past the body's
                        // count reads contact 0 and is zeroed)
#pragma unroll
                        for (int u = 0; u < SW_K; ++u) {
                            kc[u] = bm ? __ffsll((long long)bm) - 1 : 0;
                            bm &= bm - 1ull;
                        }
                        int kij[SW_K];
#pragma unroll
                        for (int u = 0; u < SW_K; ++u) {
                            kij[u] = s_cij[kc[u]];
                            kx[u] = s_cn[0][kc[u]];
                            ky[u] = s_cn[1][kc[u]];
                            krx[u] = s_cpc[0][kc[u]];
                            kry[u] = s_cpc[1][kc[u]];
                            krz[u] = s_cpc[2][kc[u]];
                        }
                        __builtin_amdgcn_sched_group_barrier(0x100, 6 * SW_K, 0);
#pragma unroll
                        for (int u = 0; u < SW_K; ++u) {
                            const bool in = u < bcnt, toward = ((kij[u] >> 8) & 0xFF) == b;
                            kx[u] = in ? (toward ? kx[u] : -kx[u]) : 0.f;
                            ky[u] = in ? (toward ? ky[u] : -ky[u]) : 0.f;
                            krx[u] = in ? krx[u] - pbx : 0.f;
                            kry[u] = in ? kry[u] - pby : 0.f;
                            krz[u] = in ? krz[u] - pbz : 0.f;
                        }
                        // bm now holds the contacts past the first SW_K
                        float ev0 = 0.f, ev1 = 0.f, ew0 = 0.f, ew1 = 0.f, ew2 = 0.f;
                        float iw0 = 0.f, iw1 = 0.f, iw2 = 0.f, iw3 = 0.f, iw4 = 0.f, iw5 = 0.f;
                        if (bcnt > 0) {
                            ev0 = s_v[0][b];
                            ev1 = s_v[1][b];
                            ew0 = s_w[0][b];
                            ew1 = s_w[1][b];
                            ew2 = s_w[2][b];
                            iw0 = s_iw[0][b];
                            iw1 = s_iw[1][b];
                            iw2 = s_iw[2][b];
                            iw3 = s_iw[3][b];
                            iw4 = s_iw[4][b];
                            iw5 = s_iw[5][b];
                        }
                        // ---- G: Jacobi sweeps; a body adds its contacts in list order
                        for (int it = 0; it < P.jacobi_iters; ++it) {
                            if (own) {
                                // every load first, then the arithmetic
                                const float wix = s_w[0][ci], wiy = s_w[1][ci], wiz = s_w[2][ci];
                                const float wjx = s_w[0][cj], wjy = s_w[1][cj], wjz = s_w[2][cj];
                                const float vix = s_v[0][ci], viy = s_v[1][ci];
                                const float vjx = s_v[0][cj], vjy = s_v[1][cj];
                                const f3 wi = cross3(mk3(wix, wiy, wiz), cri);
                                const f3 wj = cross3(mk3(wjx, wjy, wjz), crj);
                                const float vn = ((vjx + wj.x) - (vix + wi.x)) * cnx + ((vjy + wj.y) - (viy + wi.y)) * cny;
                                const float lam1 = fmaxf(clam + cwk * (-vn + cbb), 0.f);
                                s_cdl[lane] = lam1 - clam;
                                clam = lam1;
                            }
                            wave_sync();
                            if (bcnt > 0) {
                                // no branches: a slot past the body's count adds zero
                                // (its delta is selected to 0, its normal is 0)
                                float d[SW_K];
#pragma unroll
                                for (int u = 0; u < SW_K; ++u) d[u] = s_cdl[kc[u]];
                                float jx = 0.f, jy = 0.f, tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll
                                for (int u = 0; u < SW_K; ++u) {
                                    if (u < kmax) {
                                        const float du = u < bcnt ? d[u] : 0.f;
                                        const float Jx = du * kx[u], Jy = du * ky[u];
                                        jx += Jx;
                                        jy += Jy;
                                        tx -= krz[u] * Jy;
                                        ty += krz[u] * Jx;
                                        tz += krx[u] * Jy - kry[u] * Jx;
                                    }
                                }
                                for (unsigned long long rest = bm; rest; rest &= rest - 1ull) {
                                    const int c = __ffsll((long long)rest) - 1;
                                    const float cd = s_cdl[c];
                                    const float dl = ((s_cij[c] >> 8) & 0xFF) == b ? cd : -cd;
                                    const float Jx = dl * s_cn[0][c], Jy = dl * s_cn[1][c];
                                    const float rx = s_cpc[0][c] - pbx, ry = s_cpc[1][c] - pby,
                                                rz = s_cpc[2][c] - pbz;
                                    jx += Jx;
                                    jy += Jy;
                                    tx -= rz * Jy;
                                    ty += rz * Jx;
                                    tz += rx * Jy - ry * Jx;
                                }
                                ev0 += jx * P.inv_mass;
                                ev1 += jy * P.inv_mass;
                                ew0 += iw0 * tx + iw1 * ty + iw2 * tz;
                                ew1 += iw1 * tx + iw3 * ty + iw4 * tz;
                                ew2 += iw2 * tx + iw4 * ty + iw5 * tz;
                                s_v[0][b] = ev0;
                                s_v[1][b] = ev1;
                                s_w[0][b] = ew0;
                                s_w[1][b] = ew1;
                                s_w[2][b] = ew2;
                            }
                            wave_sync();
                        }
                        }
                    }
                } else if (nc > 0) {
                    __syncthreads();
                    // ---- each body's contacts as one range of a CSR list, in list
                    //      order (every contact appears once for each of its bodies)
                    if (wave == 0) {
                        const int x = lane < A ? s_bn[lane] : 0;
                        int incl = x;
#pragma unroll
                        for (int o = 1; o < 64; o <<= 1) {
                            const int y = __shfl_up(incl, o, 64);
                            if (lane >= o) incl += y;
                        }
                        if (lane < A) s_boff[lane] = incl - x;
                    }
                    __syncthreads();
                    for (int i = tid; i < A; i += BLOCK) {
                        if (!s_bn[i]) continue;
                        int k = s_boff[i];
                        for (int c = 0; c < nc; ++c) {
                            const int ij = s_cij[c];
                            if ((ij & 0xFF) == i || ((ij >> 8) & 0xFF) == i) s_bidx[k++] = (short)c;
                        }
                    }
                    __syncthreads();
                    // ---- F: effective mass along each normal, relaxed by the larger
                    //      contact count of the two bodies
                    for (int c = tid; c < nc; c += BLOCK) {
                        const int i = s_cij[c] & 0xFF, j = (s_cij[c] >> 8) & 0xFF;
                        const f3 n = mk3(s_cn[0][c], s_cn[1][c], 0.f);
                        const f3 pc = mk3(s_cpc[0][c], s_cpc[1][c], s_cpc[2][c]);
                        float Ri[9], Rj[9];
#pragma unroll
                        for (int q = 0; q < 9; ++q) { Ri[q] = s_R[q][i]; Rj[q] = s_R[q][j]; }
                        const f3 ri = sub3(pc, mk3(s_p[0][i], s_p[1][i], s_p[2][i]));
                        const f3 rj = sub3(pc, mk3(s_p[0][j], s_p[1][j], s_p[2][j]));
                        const f3 xi = cross3(ri, n), xj = cross3(rj, n);
                        const float keff = 2.f * P.inv_mass + dot3(xi, inv_inertia(P, Ri, xi)) +
                                           dot3(xj, inv_inertia(P, Rj, xj));
                        const int nmax = max(s_bn[i], s_bn[j]);
                        s_cwk[c] = 1.f / ((float)nmax * keff);
                    }
                    __syncthreads();
                    // ---- G: Jacobi sweeps: every contact reads the previous sweep's
                    //      velocities; each body then sums its contacts in list order
                    for (int it = 0; it < P.jacobi_iters; ++it) {
                        for (int c = tid; c < nc; c += BLOCK) {
                            const int i = s_cij[c] & 0xFF, j = (s_cij[c] >> 8) & 0xFF;
                            const f3 pc = mk3(s_cpc[0][c], s_cpc[1][c], s_cpc[2][c]);
                            const f3 ri = sub3(pc, mk3(s_p[0][i], s_p[1][i], s_p[2][i]));
                            const f3 rj = sub3(pc, mk3(s_p[0][j], s_p[1][j], s_p[2][j]));
                            const f3 wi = cross3(mk3(s_w[0][i], s_w[1][i], s_w[2][i]), ri);
                            const f3 wj = cross3(mk3(s_w[0][j], s_w[1][j], s_w[2][j]), rj);
                            const float vn = ((s_v[0][j] + wj.x) - (s_v[0][i] + wi.x)) * s_cn[0][c] +
                                             ((s_v[1][j] + wj.y) - (s_v[1][i] + wi.y)) * s_cn[1][c];
                            const float lam = s_clam[c];
                            const float lam1 = fmaxf(lam + s_cwk[c] * (-vn + s_cb[c]), 0.f);
                            s_cdl[c] = lam1 - lam;
                            s_clam[c] = lam1;
                        }
                        __syncthreads();
                        // four lanes per body split its contacts (q = g, g + 4, ...),
                        // then add their partial sums in a fixed butterfly order;
                        // one application of 1/m and the world inverse inertia
                        for (int e0 = 0; e0 < 4 * A; e0 += BLOCK) {
                            const int e = e0 + tid, b = e >> 2, g = e & 3;
                            float jx = 0.f, jy = 0.f, tx = 0.f, ty = 0.f, tz = 0.f;
                            const int cnt = b < A ? s_bn[b] : 0;
                            if (cnt > 0) {
                                const float pbx = s_p[0][b], pby = s_p[1][b], pbz = s_p[2][b];
                                const short *bl = s_bidx + s_boff[b];
#pragma unroll 4
                                for (int q = g; q < cnt; q += 4) {
                                    const int c = bl[q];
                                    const float dl = ((s_cij[c] >> 8) & 0xFF) == b ? s_cdl[c] : -s_cdl[c];
                                    const float Jx = dl * s_cn[0][c], Jy = dl * s_cn[1][c];
                                    const float rx = s_cpc[0][c] - pbx, ry = s_cpc[1][c] - pby,
                                                rz = s_cpc[2][c] - pbz;
                                    jx += Jx;
                                    jy += Jy;
                                    tx -= rz * Jy;
                                    ty += rz * Jx;
                                    tz += rx * Jy - ry * Jx;
                                }
                            }
#pragma unroll
                            for (int m = 2; m > 0; m >>= 1) {
                                jx += lane_xor_f(jx, m);
                                jy += lane_xor_f(jy, m);
                                tx += lane_xor_f(tx, m);
                                ty += lane_xor_f(ty, m);
                                tz += lane_xor_f(tz, m);
                            }
                            if (cnt > 0 && g == 0) {
                                s_v[0][b] += jx * P.inv_mass;
                                s_v[1][b] += jy * P.inv_mass;
                                s_w[0][b] += s_iw[0][b] * tx + s_iw[1][b] * ty + s_iw[2][b] * tz;
                                s_w[1][b] += s_iw[1][b] * tx + s_iw[3][b] * ty + s_iw[4][b] * tz;
                                s_w[2][b] += s_iw[2][b] * tx + s_iw[4][b] * ty + s_iw[5][b] * tz;
                            }
                        }
                        __syncthreads();
                    }
                }

                // ---- H: positions and orientations (agent i is on the thread that ran its
                //      E, so without contacts no barrier separates the two)
                for (int i = tid; i < A; i += BLOCK) {
                    if (!s_act[i]) continue;
                    const float vx = s_v[0][i], vy = s_v[1][i], vz = s_v[2][i];
                    s_p[0][i] += h * vx;
                    s_p[1][i] += h * vy;
                    s_p[2][i] += h * vz;
                    float qw = s_q[0][i], qx = s_q[1][i], qy = s_q[2][i], qz = s_q[3][i];
                    const float wx = s_w[0][i], wy = s_w[1][i], wz = s_w[2][i];
                    const float dw = -(wx * qx + wy * qy + wz * qz);
                    const float dx = wx * qw + (wy * qz - wz * qy);
                    const float dy = wy * qw + (wz * qx - wx * qz);
                    const float dz = wz * qw + (wx * qy - wy * qx);
                    qw += 0.5f * h * dw; qx += 0.5f * h * dx; qy += 0.5f * h * dy; qz += 0.5f * h * dz;
                    const float L = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
                    s_q[0][i] = qw / L; s_q[1][i] = qx / L; s_q[2][i] = qy / L; s_q[3][i] = qz / L;
                    if (!last) SF_PHASE_A(i);
                }
                __syncthreads();
            }

            // ---- events, reward, termination, write-back (Sec. "Reward Design Details")
            for (int i = tid; i < A; i += BLOCK) {
                const int n = a0 + i;
                if (!s_act[i]) {
                    reward[n] = 0.f;
                    done[n] = 0;
                    events[n] = 0;
                    continue;
                }
                float dyn[SF_F_MU];
                for (int c = 0; c < 3; ++c) {
                    dyn[SF_F_PX + c] = s_p[c][i];
                    dyn[SF_F_VX + c] = s_v[c][i];
                    dyn[SF_F_WX + c] = s_w[c][i];
                }
                for (int c = 0; c < 4; ++c) {
                    dyn[SF_F_QW + c] = s_q[c][i];
                    dyn[SF_F_OM0 + c] = s_om[4 * i + c];
                }
                dyn[SF_F_STEER] = s_th[i];
                dyn[SF_F_STEER_RATE] = s_thd[i];
                finish_agent(P, Wd, st, ist, N, n, w, i, dyn, s_muo[i], s_coll[i] != 0, s_nan[i] != 0, s_ovf != 0,
                             s_forbid[i] != 0, s_p0[i], s_tail[i], s_spawn, reward, done, events);
            }
        } while (0);
        if (!queue) break;
        __syncthreads();   // the world's LDS is no longer read
        if (tid == 0) s_item = atomicAdd(queue, 1) + (int)gridDim.x;
        __syncthreads();
        item = s_item;
    }
    if (SUR) {
        __syncthreads();
        if (tid == 0 && s_sur_cnt[0]) atomicAdd(Su.counts, (unsigned long long)s_sur_cnt[0]);
        if (tid == 1 && s_sur_cnt[1]) atomicAdd(Su.counts + 1, (unsigned long long)s_sur_cnt[1]);
    }
    // the last block out re-arms the queue for the next launch
    if (queue && tid == 0 && atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
        queue[0] = 0;
        queue[1] = 0;
    }
}

#undef SF_PHASE_A

void launch_step(const DevParams &P, const DevWorld &Wd, const DevSur &Su, bool use_sur, float *st, int *ist,
                 const float *act, float h, int S, float *reward, uint8_t *done, uint8_t *events, uint32_t *rec,
                 int *rec_cnt, int rec_cap, const int4 *items, int block, int grid, int *queue, hipStream_t s) {
    if (Wd.W == 0) return;
    // a persistent grid pulls worlds from the queue; a full grid needs none
    if (grid <= 0 || grid >= Wd.W) {
        grid = Wd.W;
        queue = nullptr;
    }
    // the surrogate step always takes 256 threads: the network's LDS copy
    // leaves room for at most three wheel waves, and with fewer a wave's
    // wheels fill more 32-row network passes (each a chain of products on
    // one SIMD)
    if (use_sur) {
        sf_launch(k_step<256, true>, dim3(grid), dim3(256), 0, s, P, Wd, Su, st, ist, act, h, S, reward, done,
                  events, rec, rec_cnt, rec_cap, items, queue);
        return;
    }
#define SF_STEP_LAUNCH(B)                                                                                   \
    sf_launch(k_step<B, false>, dim3(grid), dim3(B), 0, s, P, Wd, Su, st, ist, act, h, S, reward, done, events, \
              rec, rec_cnt, rec_cap, items, queue)
    if (block <= 64) SF_STEP_LAUNCH(64);
    else if (block <= 128) SF_STEP_LAUNCH(128);
    else if (block <= 192) SF_STEP_LAUNCH(192);
    else if (block <= 256) SF_STEP_LAUNCH(256);
    else SF_STEP_LAUNCH(320);
#undef SF_STEP_LAUNCH
}

// ------------------------------------------------------ kinematic bicycle
// The lightweight backend (Sec. "Vehicle Dynamics Ablation"): the same
// actions drive a kinematic single-track model, advanced once per control
// tick by forward Euler, with no suspension, tires or contact forces.  Slip
// angle at the centre of mass beta = atan(l_r tan(delta) / (l_f + l_r)),
// yaw rate v sin(beta) / l_r; front-drive force 2 tau_drive a / r_w, brake
// force 2 (tau_bf + tau_br) |a| / r_w, and braking stops at v = 0 (no
// reversing).  Vehicle pairs whose circles overlap on the tick's input
// poses count as collisions (the articulated step takes them on each
// substep's input poses).  One wave per world, one lane per vehicle; the state keeps
// its shared layout (level chassis at ride height, yaw-only orientation,
// planar velocity along the direction of travel, rolling wheels, steering
// angle = command, no friction seen).
__global__ __launch_bounds__(64) void k_step_bicycle(DevParams P, DevWorld Wd, float *__restrict__ st,
                                                     int *__restrict__ ist, const float *__restrict__ act, float dt,
                                                     float *__restrict__ reward, uint8_t *__restrict__ done,
                                                     uint8_t *__restrict__ events, uint32_t *__restrict__ rec,
                                                     int *__restrict__ rec_cnt, int rec_cap,
                                                     const int4 *__restrict__ items) {
    __shared__ int s_cq[6][SF_MAXA];
    __shared__ int s_act[SF_MAXA];
    __shared__ uint8_t s_coll[SF_MAXA];
    __shared__ uint32_t s_pairs[SF_PAIR_CAP];
    const int4 it = items[blockIdx.x];
    const int w = it.x, a0 = it.y, A = it.z, N = Wd.N, i = threadIdx.x, n = a0 + i;
    if (A <= 0) return;
    const bool mine = i < A;
    const bool on = mine && ist[SF_I_ACTIVE * N + n] != 0;
    if (mine) {
        s_act[i] = on;
        s_coll[i] = 0;
    }
    if (on) {
        int cq[6];
        circle_centres_q(P, st[SF_F_PX * N + n], st[SF_F_PY * N + n], st[SF_F_QW * N + n], st[SF_F_QX * N + n],
                         st[SF_F_QY * N + n], st[SF_F_QZ * N + n], cq);
        for (int c = 0; c < 6; ++c) s_cq[c][i] = cq[c];
    }
    wave_sync();
    const int np = detect_pairs_wave(P, s_cq, s_act, A, s_pairs);
    wave_sync();
    if (rec) {
        for (int k = i; k < np && k < rec_cap; k += 64) rec[(size_t)w * rec_cap + k] = s_pairs[k];
        if (i == 0) rec_cnt[w] = np;
    }
    for (int k = i; k < np; k += 64) {
        s_coll[s_pairs[k] & 0xFF] = 1;
        s_coll[(s_pairs[k] >> 8) & 0xFF] = 1;
    }
    wave_sync();
    if (!mine) return;
    if (!on) {
        reward[n] = 0.f;
        done[n] = 0;
        events[n] = 0;
        return;
    }
    float dyn[SF_F_MU];
    bool bad = false;
    const float2 p0 = make_float2(st[SF_F_PX * N + n], st[SF_F_PY * N + n]);
    {
        float al = act[2 * (size_t)n], sa = act[2 * (size_t)n + 1];
        if (al != al) { al = 0.f; bad = true; }
        if (sa != sa) { sa = 0.f; bad = true; }
        al = fminf(fmaxf(al, -1.f), 1.f);
        const float delta = fminf(fmaxf(sa, -P.steer_max), P.steer_max);
        const float qw = st[SF_F_QW * N + n], qx = st[SF_F_QX * N + n];
        const float qy = st[SF_F_QY * N + n], qz = st[SF_F_QZ * N + n];
        const float psi = atan2f(2.f * (qw * qz + qx * qy), 1.f - 2.f * (qy * qy + qz * qz));
        const float v = hypotf(st[SF_F_VX * N + n], st[SF_F_VY * N + n]);
        const float lf = P.mount[0][0], lr = -P.mount[2][0];
        const float beta = atanf(lr / (lf + lr) * tanf(delta));
        const float acc = al > 0.f ? 2.f * P.tau_drive * al / (P.rw * P.mass)
                        : al < 0.f ? -2.f * (P.tau_bf + P.tau_br) * (-al) / (P.rw * P.mass) : 0.f;
        const float psi1 = psi + v * sinf(beta) / lr * dt;
        const float v1 = fmaxf(v + acc * dt, 0.f);
        dyn[SF_F_PX] = st[SF_F_PX * N + n] + v * cosf(psi + beta) * dt;
        dyn[SF_F_PY] = st[SF_F_PY * N + n] + v * sinf(psi + beta) * dt;
        dyn[SF_F_PZ] = P.z_ride;
        dyn[SF_F_QW] = cosf(0.5f * psi1);
        dyn[SF_F_QX] = 0.f;
        dyn[SF_F_QY] = 0.f;
        dyn[SF_F_QZ] = sinf(0.5f * psi1);
        dyn[SF_F_VX] = v1 * cosf(psi1 + beta);
        dyn[SF_F_VY] = v1 * sinf(psi1 + beta);
        dyn[SF_F_VZ] = 0.f;
        dyn[SF_F_WX] = 0.f;
        dyn[SF_F_WY] = 0.f;
        dyn[SF_F_WZ] = v1 * sinf(beta) / lr;
        for (int c = 0; c < 4; ++c) dyn[SF_F_OM0 + c] = v1 / P.rw;
        dyn[SF_F_STEER] = delta;
        dyn[SF_F_STEER_RATE] = 0.f;
    }
    finish_agent(P, Wd, st, ist, N, n, w, i, dyn, 0.f, s_coll[i] != 0, bad, false, Wd.forbid && Wd.forbid[n],
                 p0, load_tail(st, ist, N, n), SpawnRange{Wd.soff[w], Wd.soff[w + 1] - Wd.soff[w]}, reward, done,
                 events);
}

void launch_step_bicycle(const DevParams &P, const DevWorld &Wd, float *st, int *ist, const float *act, float dt,
                         float *reward, uint8_t *done, uint8_t *events, uint32_t *rec, int *rec_cnt, int rec_cap,
                         const int4 *items, hipStream_t s) {
    if (Wd.W == 0) return;
    sf_launch(k_step_bicycle, dim3(Wd.W), dim3(64), 0, s, P, Wd, st, ist, act, dt, reward, done, events, rec, rec_cnt,
              rec_cap, items);
}

// ------------------------------------------------------------------ reset
__global__ void k_reset(DevParams P, DevWorld Wd, float *st, int *ist, const uint8_t *mask, int bump) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= Wd.N) return;
    if (mask && !mask[n]) return;
    int w = Wd.world_of[n];
    if (bump) ist[SF_I_EPISODE * Wd.N + n] += 1;
    spawn_agent(P, Wd, st, ist, Wd.N, n, w, n - Wd.aoff[w]);
}

void launch_reset(const DevParams &P, const DevWorld &Wd, float *st, int *ist, const uint8_t *mask,
                  int bump_episode, hipStream_t s) {
    if (Wd.N == 0) return;
    k_reset<<<(Wd.N + 255) / 256, 256, 0, s>>>(P, Wd, st, ist, mask, bump_episode);
}

// ---------------------------------------------------------- debug raycast
__global__ void k_debug_raycast(DevParams P, DevWorld Wd, const float *st, float *out) {
    int wi = blockIdx.x * blockDim.x + threadIdx.x;
    if (wi >= 4 * Wd.N) return;
    const int N = Wd.N, n = wi >> 2, wh = wi & 3;
    float R[9];
    quat_R(st[SF_F_QW * N + n], st[SF_F_QX * N + n], st[SF_F_QY * N + n], st[SF_F_QZ * N + n], R);
    const f3 rm = Rmul(R, mount_of(P, wh));
    const f3 m = add3(mk3(st[SF_F_PX * N + n], st[SF_F_PY * N + n], st[SF_F_PZ * N + n]), rm);
    const int w = Wd.world_of[n];
    RayHit H = raycast(P, Wd, Wd.tgrid[w], Wd.toff[w + 1] > Wd.toff[w], m, mk3(-R[2], -R[5], -R[8]));
    out[4 * (size_t)wi + 0] = (float)H.hit;
    out[4 * (size_t)wi + 1] = H.hit ? H.t : 0.f;
    out[4 * (size_t)wi + 2] = (float)H.surf;
    out[4 * (size_t)wi + 3] = (float)H.tri;
}

void launch_debug_raycast(const DevParams &P, const DevWorld &Wd, const float *st, float *out,
                          hipStream_t s) {
    if (Wd.N == 0) return;
    k_debug_raycast<<<(4 * Wd.N + 255) / 256, 256, 0, s>>>(P, Wd, st, out);
}
