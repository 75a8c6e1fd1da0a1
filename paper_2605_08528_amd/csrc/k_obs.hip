// Observation gather (Sec. "Observation Space Details"): one wavefront per
// agent.  Ego block, the 64 road points with the smallest quantised
// distance (grid-ring search, exact selection on integer keys, emitted in
// point-index order), and the 8 nearest active neighbours with swept-circle
// time to collision.  The row is staged in LDS and written as one coalesced
// 1 KB store per wave.
#include <algorithm>

#include "sf_dev.h"

__device__ __forceinline__ unsigned long long lane_lt() {
    unsigned lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        unsigned long long o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        unsigned long long o = shfl_xor_u64(v, m);
        v = o > v ? o : v;
    }
    return v;
}

#define KPL (SF_CAND_CAP / 64)  // candidate keys per lane
// points loaded per lane and batch: after a prune (64 kept) a full batch
// still fits the candidate buffer
#define BATCH ((SF_CAND_CAP - 64) / 64 < 8 ? (SF_CAND_CAP - 64) / 64 : 8)

// number of buffered keys <= x among the first `slots` register slots
__device__ __forceinline__ int count_le(const unsigned long long kv[KPL], unsigned long long x, int slots) {
    int c = 0;
#pragma unroll
    for (int s = 0; s < KPL; ++s)
        if (s < slots) c += __popcll(__ballot(kv[s] <= x));
    return c;
}

// The K-th smallest key (1-based) of n >= K distinct keys held in the first
// `slots` register slots of the wave (unused entries hold ~0): binary search
// on the distance part, then on the index only when distances tie.
__device__ unsigned long long kth_smallest(const unsigned long long kv[KPL], int K, int slots) {
    unsigned long long lo = ~0ull, hi = 0;
#pragma unroll
    for (int s = 0; s < KPL; ++s) {
        if (s >= slots) break;
        lo = kv[s] < lo ? kv[s] : lo;
        if (kv[s] != ~0ull) hi = kv[s] > hi ? kv[s] : hi;
    }
    lo = wave_min_u64(lo);
    hi = wave_max_u64(hi);
    unsigned long long dlo = lo >> 20, dhi = hi >> 20;
    while (dlo < dhi) {
        const unsigned long long mid = dlo + ((dhi - dlo) >> 1);
        if (count_le(kv, (mid << 20) | 0xFFFFFull, slots) >= K) dhi = mid; else dlo = mid + 1;
    }
    // keys with distance < dlo number below K; if exactly K have distance
    // <= dlo, the K-th key is the largest of them
    const unsigned long long top = (dlo << 20) | 0xFFFFFull;
    if (count_le(kv, top, slots) == K) {
        unsigned long long m = 0;
#pragma unroll
        for (int s = 0; s < KPL; ++s)
            if (s < slots && kv[s] <= top) m = kv[s] > m ? kv[s] : m;
        return wave_max_u64(m);
    }
    unsigned long long ilo = dlo << 20, ihi = top;
    while (ilo < ihi) {
        const unsigned long long mid = ilo + ((ihi - ilo) >> 1);
        if (count_le(kv, mid, slots) >= K) ihi = mid; else ilo = mid + 1;
    }
    return ilo;
}

// Keep the 64 smallest of nc > 64 distinct buffered keys (nc == 64: keep
// all); returns the largest kept key.
__device__ unsigned long long keep64(unsigned long long *cand, int &nc) {
    const int lane = threadIdx.x & 63;
    wave_sync();
    unsigned long long kv[KPL];
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
        const int slot = lane + 64 * t;
        kv[t] = slot < nc ? cand[slot] : ~0ull;
    }
    if (nc == 64) return wave_max_u64(kv[0]);
    const unsigned long long k64 = kth_smallest(kv, 64, (nc + 63) >> 6);
    wave_sync();
    int keep = 0;
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
        const bool f = kv[t] <= k64;
        const unsigned long long bal = __ballot(f);
        if (f) cand[keep + __popcll(bal & lane_lt())] = kv[t];
        keep += __popcll(bal);
    }
    nc = keep;
    wave_sync();
    return k64;
}

// the smallest key above every point closer than r metres (quantised)
__device__ __forceinline__ unsigned long long hint_key(float r) {
    const double rq = (double)r * 1024.0 + 1.0;
    return ((unsigned long long)sat_key((long long)(rq * rq) + 1) << 20) | 0xFFFFFull;
}

// Append to the candidate buffer the keys below kthr of every point of the
// segments seg(j, s, e), j < nseg (each lane fills the point range [s, e) of
// its segment, or leaves it empty), flattened across the wave and loaded in
// batches of BATCH points per lane; a full buffer is first cut to its 64
// best, which also lowers kthr.
template <class SEG>
__device__ __forceinline__ void gather(const DevWorld &Wd, int nseg, SEG seg, const int4 *__restrict__ pts, int QX,
                                       int QY,
                                       unsigned long long *cand, int *segs, int *segp, int &nc,
                                       unsigned long long &kthr) {
    const int lane = threadIdx.x & 63;
    for (int sb = 0; sb < nseg; sb += 64) {
        int s = 0, e = 0;
        if (sb + lane < nseg) seg(sb + lane, s, e);
        const int len = e - s;
        int incl = len;
        for (int o = 1; o < 64; o <<= 1) {
            const int y2 = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y2;
        }
        const int total = __shfl(incl, 63, 64);
        if (total == 0) continue;
        segs[lane] = s;
        segp[lane] = incl - len;
        wave_sync();
        // all loads of a batch are issued before any key is appended
        for (int f0 = 0; f0 < total; f0 += 64 * BATCH) {
            const int nslot = min(BATCH, (total - f0 + 63) >> 6);
            if (nc + 64 * nslot > SF_CAND_CAP) kthr = keep64(cand, nc);
            int4 pq[BATCH];
#pragma unroll
            for (int t = 0; t < BATCH; ++t) {
                const int f = f0 + 64 * t + lane;
                pq[t] = make_int4(0, 0, 0, -1);
                if (t < nslot && f < total) {
                    // the segment holding flat index f: the last one whose
                    // prefix is <= f (it is never empty)
                    int lo = 0, hi = min(63, nseg - 1 - sb);
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (segp[mid] <= f) lo = mid; else hi = mid - 1;
                    }
                    pq[t] = pts[segs[lo] + (f - segp[lo])];
                    if (Wd.touch) touch(Wd, SF_T_PT, segs[lo] + (f - segp[lo]));
                }
            }
#pragma unroll
            for (int t = 0; t < BATCH; ++t) {
                if (t >= nslot) break;
                unsigned long long key = ~0ull;
                if (pq[t].w == 0) {
                    const long long dx = (long long)pq[t].x - QX, dy = (long long)pq[t].y - QY;
                    key = ((unsigned long long)sat_key(dx * dx + dy * dy) << 20) | (unsigned)pq[t].z;
                }
                const bool has = key < kthr;
                const unsigned long long bal = __ballot(has);
                if (has) cand[nc + __popcll(bal & lane_lt())] = key;
                nc += __popcll(bal);
            }
        }
        wave_sync();
    }
}

// XCD-aware block order: blocks are dealt round-robin to the 8 XCDs, so
// give each XCD a contiguous range of agents (neighbouring agents share a
// world and its road grid, which then stays in one L2).  First agent of the
// block for `waves` agents per block.
__device__ __forceinline__ int xcd_agent(int waves) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return (x * q + min(x, r) + (b >> 3)) * waves;
}

// Appendix "Reward Design Details" on the pose this observation sees, from
// the road points it selected (one per lane, my_idx) and the neighbours'
// times to collision (nb_ttc, 10 s in lanes without one): whether a
// vehicle circle overlaps a road-edge segment (read by the next step), and
// after a step the six dense terms added to that step's reward of an agent
// that carries on.  Every road point stands for the 0.5 m segment of its
// polyline centred on it; the decisions are integer predicates on
// quantised values, so that they match the oracle's bit for bit.
__device__ __forceinline__ bool circle_hits_segment(long long cx, long long cy, int2 pq, float2 dir, long long R2) {
    const long long hx = qpos(0.25f * dir.x), hy = qpos(0.25f * dir.y);
    const long long ax = pq.x - hx, ay = pq.y - hy, vx = 2 * hx, vy = 2 * hy;
    const long long wx = cx - ax, wy = cy - ay;
    if (wx > 4096 || wx < -4096 || wy > 4096 || wy < -4096) return false;
    const long long len2 = vx * vx + vy * vy, t = wx * vx + wy * vy;
    if (len2 == 0 || t <= 0) return wx * wx + wy * wy < R2;
    if (t >= len2) {
        const long long ex = wx - vx, ey = wy - vy;
        return ex * ex + ey * ey < R2;
    }
    return (wx * wx + wy * wy) * len2 - t * t < R2 * len2;
}

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = fminf(v, lane_xor_f(v, m));
    return v;
}

__device__ void shaping(const DevParams &P, const DevWorld &Wd, int n, int r0, int my_idx, float px, float py,
                        float qw, float qx, float qy, float qz, float hx, float hy, float vx, float vy, float goal_x,
                        float goal_y, float nb_ttc) {
    const int lane = threadIdx.x & 63;
    const long long QX = qpos(px), QY = qpos(py);
    int cq[6];
    circle_centres_q(P, px, py, qw, qx, qy, qz, cq);
    const long long R2 = (long long)(P.Qr2 >> 2);   // Qr2 = (2 round(r 2^10))^2
    // planar heading of the quantised quaternion (unnormalised integers)
    const long long iqw = qquat(qw), iqx = qquat(qx), iqy = qquat(qy), iqz = qquat(qz);
    const long long ihx = (1ll << 28) - 2 * (iqy * iqy + iqz * iqz), ihy = 2 * (iqx * iqy + iqw * iqz);
    const long long nh = isqrt64(ihx * ihx + ihy * ihy);
    const float vf = hx * vx + hy * vy;
    bool forbid = false;
    unsigned long long lkey = ~0ull;
    float etau = INFINITY;
    if (my_idx != 0x7fffffff) {
        const int q = r0 + my_idx;
        const int ty = Wd.road_type[q];
        const int2 pq = Wd.road_q[q];
        const long long ex = (long long)pq.x - QX, ey = (long long)pq.y - QY;
        if (ty == 15 || ty == 16) {
            const float2 rd = Wd.road_dir[q];
#pragma unroll
            for (int a = 0; a < 3; ++a) forbid = forbid || circle_hits_segment(cq[2 * a], cq[2 * a + 1], pq, rd, R2);
            // road-edge time to collision: edge points ahead in the corridor
            if (vf > 0.f && ex <= (1 << 20) && ex >= -(1 << 20) && ey <= (1 << 20) && ey >= -(1 << 20)) {
                const long long along = ex * ihx + ey * ihy, side = -ex * ihy + ey * ihx;
                if (along > 0 && side <= Wd.edge_half_q * nh && side >= -Wd.edge_half_q * nh) {
                    const float2 rp = Wd.road_xy[q];
                    const float xb = hx * (rp.x - px) + hy * (rp.y - py);
                    etau = fmaxf(xb - (P.cd + P.cr), 0.f) / vf;
                }
            }
        }
        if (ty == 1 || ty == 2) lkey = ((unsigned long long)sat_key(ex * ex + ey * ey) << 20) | (unsigned)my_idx;
    }
    forbid = __ballot(forbid) != 0ull;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const unsigned long long o = shfl_xor_u64(lkey, m);
        lkey = o < lkey ? o : lkey;
    }
    etau = wave_min_f(etau);
    const float tau = wave_min_f(lane < 8 ? nb_ttc : 10.f);
    if (lane != 0) return;
    Wd.forbid[n] = forbid;
    if (!Wd.shape_add || Wd.done_out[n]) return;
    float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f, t4, t5 = 0.f;
    bool off = true;
    if (lkey != ~0ull) {
        const int q = r0 + (int)(lkey & 0xFFFFF);
        const float2 rd = Wd.road_dir[q];
        float tx = rd.x, ty = rd.y;
        // the lane's direction turned toward the goal (integer sign)
        const long long gdx = (long long)qpos(goal_x) - QX, gdy = (long long)qpos(goal_y) - QY;
        if ((long long)qquat(tx) * gdx + (long long)qquat(ty) * gdy < 0) { tx = -tx; ty = -ty; }
        const float2 d = Wd.disp[n];
        t0 = 2.f * fminf(fmaxf(d.x * tx + d.y * ty, -2.f), 2.f);
        const float2 rp = Wd.road_xy[q];
        const float lat = (px - rp.x) * (-ty) + (py - rp.y) * tx;
        const float al = hx * tx + hy * ty;
        t1 = 0.08f * expf(-(lat / 1.75f) * (lat / 1.75f)) * (0.2f + 0.8f * fmaxf(al, 0.f));
        const int2 pq = Wd.road_q[q];
        long long latq = (QX - pq.x) * (-(long long)qquat(ty)) + (QY - pq.y) * (long long)qquat(tx);
        if (latq < 0) latq = -latq;
        off = latq > 54525952ll /* 3.25 m in 2^-24 m */ || (long long)(lkey >> 20) > 6144ll * 6144ll;
    }
    if (off) t2 = -0.5f;
    const long long qvx = qpos(vx), qvy = qpos(vy);
    if (qvx * qvx + qvy * qvy < 1024ll * 1024ll) t3 = -0.05f;
    t4 = -fminf(0.10f / fmaxf(tau, 0.5f), 0.35f);
    if (etau < INFINITY) t5 = -fminf(0.07f / fmaxf(etau, 0.5f), 0.40f);
    Wd.reward_out[n] += ((((t0 + t1) + t2) + t3) + t4) + t5;
}

// One agent's observation row (one wave): written to obs and left in the
// wave's LDS row; returns false for an inactive agent (row of zeros in
// memory, LDS row untouched).
__device__ bool obs_agent(const DevParams &P, const DevWorld &Wd, const float *__restrict__ st,
                          const int *__restrict__ ist, float *__restrict__ obs, int *__restrict__ dbg,
                          float4 *__restrict__ hint, int n, unsigned long long *cand, float *row, int *sel,
                          int *segs, int *segp) {
    const int lane = threadIdx.x & 63;
    const int N = Wd.N;
    float4 *dst = reinterpret_cast<float4 *>(obs + (size_t)n * SF_OBS_DIM);

    // every load that depends only on the agent goes out together, its
    // world's offsets and road grid header included (per-agent copies), so
    // the first group is one memory round trip
    const int active = ist[SF_I_ACTIVE * N + n];
    const float px = st[SF_F_PX * N + n], py = st[SF_F_PY * N + n];
    const float qw = st[SF_F_QW * N + n], qx = st[SF_F_QX * N + n];
    const float qy = st[SF_F_QY * N + n], qz = st[SF_F_QZ * N + n];
    const float vx = st[SF_F_VX * N + n], vy = st[SF_F_VY * N + n];
    const float goal_x = st[SF_F_GOAL_X * N + n], goal_y = st[SF_F_GOAL_Y * N + n];
    const float mu_seen = st[SF_F_MU * N + n];
    const float4 hv = hint[n];
    const int4 aw = Wd.agent_world[n];
    const int a0 = aw.x, A = aw.y, r0 = aw.z, PW = aw.w;
    const GridHdr g = Wd.agent_grid[n];
    if (!active) {
        if (Wd.forbid && lane == 0) Wd.forbid[n] = 0;
        dst[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (dbg) dbg[(size_t)n * 72 + lane] = -1;
        if (dbg && lane < 8) dbg[(size_t)n * 72 + 64 + lane] = -1;
        return false;
    }
    // the agent's road-grid cell and the first ring that holds points
    int cx = (int)floorf((px - g.x0) * g.inv_cell);
    int cy = (int)floorf((py - g.y0) * g.inv_cell);
    cx = max(0, min(cx, g.nx - 1));
    cy = max(0, min(cy, g.ny - 1));
    const int rr_first = PW > 0 ? Wd.pt_occ[g.cbase + cy * g.nx + cx] : 0;
    if (PW > 0) touch(Wd, SF_T_PT_OCC, g.cbase + cy * g.nx + cx);
    float hx = 1.f - 2.f * (qy * qy + qz * qz), hy = 2.f * (qx * qy + qw * qz);
    {
        float L = sqrtf(hx * hx + hy * hy);
        if (L < 1e-12f) { hx = 1.f; hy = 0.f; } else { hx /= L; hy /= L; }
    }
    // The 64th road distance of this agent's previous observation, grown by
    // the distance moved since, bounds this one (triangle inequality), so
    // cells and points beyond it are skipped from the start.  No bound yet:
    // not a number.
    const float moved = sqrtf((px - hv.x) * (px - hv.x) + (py - hv.y) * (py - hv.y));
    const float rhint = hv.z == hv.z ? hv.z + moved + 0.01f : INFINITY;
    for (int k = lane; k < SF_OBS_DIM; k += 64) row[k] = 0.f;
    wave_sync();

    // ---- ego: goal in the body frame, heading error, distance, velocity, mu
    if (lane < 8) {
        const float gx = goal_x - px, gy = goal_y - py;
        const float gbx = hx * gx + hy * gy, gby = -hy * gx + hx * gy;
        const float dist = sqrtf(gx * gx + gy * gy);
        float e;
        switch (lane) {
            case 0: e = gbx / 100.f; break;
            case 1: e = gby / 100.f; break;
            case 2: e = dist > 0.f ? gby / dist : 0.f; break;
            case 3: e = dist > 0.f ? gbx / dist : 1.f; break;
            case 4: e = dist / 100.f; break;
            case 5: e = (hx * vx + hy * vy) / 10.f; break;
            case 6: e = (-hy * vx + hx * vy) / 10.f; break;
            default: e = mu_seen; break;
        }
        row[lane] = e;
    }
    const int QX = qpos(px), QY = qpos(py);
    float nb_ttc = 10.f;     // time to collision of this lane's neighbour (10 s: none)
    int nb_ttc_lane = 1;

    // ---- neighbours: 8 nearest other active agents of the world
    {
        // lane l holds agent a0 + l of the world (all of its planar state,
        // so that the 8 nearest need no second round of loads)
        unsigned long long key = ~0ull;
        float ox = 0.f, oy = 0.f, oqw = 1.f, oqx = 0.f, oqy = 0.f, oqz = 0.f, ovx = 0.f, ovy = 0.f;
        if (lane < A) {
            const int m = a0 + lane;
            const int act_m = ist[SF_I_ACTIVE * N + m];
            ox = st[SF_F_PX * N + m];
            oy = st[SF_F_PY * N + m];
            oqw = st[SF_F_QW * N + m];
            oqx = st[SF_F_QX * N + m];
            oqy = st[SF_F_QY * N + m];
            oqz = st[SF_F_QZ * N + m];
            ovx = st[SF_F_VX * N + m];
            ovy = st[SF_F_VY * N + m];
            if (m != n && act_m) {
                long long dx = (long long)qpos(ox) - QX;
                long long dy = (long long)qpos(oy) - QY;
                key = ((unsigned long long)sat_key(dx * dx + dy * dy) << 8) | (unsigned)lane;
            }
        }
        // every key sits in a lane below A: with A <= 32 the first half of
        // the wavefront holds them all
        key = A <= 32 ? wave_sort_u64<32>(key) : wave_sort_u64<64>(key);
        int jn = key == ~0ull ? -1 : (int)(key & 0xFF);
        if (dbg && lane < 8) dbg[(size_t)n * 72 + 64 + lane] = jn;
        // the state of the neighbour of rank `lane`, from lane jn
        const int src = jn < 0 ? 0 : jn;
        const float mx = __shfl(ox, src, 64), my = __shfl(oy, src, 64);
        const float mqw = __shfl(oqw, src, 64), mqx = __shfl(oqx, src, 64);
        const float mqy = __shfl(oqy, src, 64), mqz = __shfl(oqz, src, 64);
        const float mvx = __shfl(ovx, src, 64), mvy = __shfl(ovy, src, 64);
        if (lane < 8 && jn >= 0) {
            float jx = 1.f - 2.f * (mqy * mqy + mqz * mqz), jy = 2.f * (mqx * mqy + mqw * mqz);
            nb_ttc_lane = 0;   // this lane holds a neighbour (its time to collision below)
            float L = sqrtf(jx * jx + jy * jy);
            if (L < 1e-12f) { jx = 1.f; jy = 0.f; } else { jx /= L; jy /= L; }
            const float dx = mx - px, dy = my - py;
            const float bx = hx * dx + hy * dy, by = -hy * dx + hx * dy;
            float dpsi = atan2f(hx * jy - hy * jx, hx * jx + hy * jy);
            if (dpsi == -3.14159265358979f) dpsi = 3.14159265358979f;
            // swept circles, constant planar velocities; 0 if touching
            const float ttc = bx >= 0.f ? ttc_swept(P, px, py, hx, hy, vx, vy, mx, my, jx, jy, mvx, mvy, 10.f) : 10.f;
            nb_ttc = ttc;
            float *o = row + 200 + 7 * lane;
            o[0] = bx / 100.f;
            o[1] = by / 100.f;
            o[2] = P.length / 100.f;
            o[3] = P.width / 100.f;
            o[4] = dpsi / 3.14159265358979f;
            o[5] = sqrtf(mvx * mvx + mvy * mvy) / 10.f;
            o[6] = ttc / 10.f;
        }
    }

    // ---- road: exact 64 nearest points by (quantised squared distance, index)
    int my_idx = 0x7fffffff;
    if (PW > 0) {
        int nc = 0;  // buffered candidates (uniform)
        // once 64 candidates are known: the largest of the 64 best so far.
        // A point with a larger key can no longer be selected, and a cell
        // farther than that distance (plus a margin for the quantisation of
        // positions) need not be read at all.
        unsigned long long kthr = ~0ull;
        float rcull = INFINITY;
        const int4 *__restrict__ pts = Wd.pt_cell;
        // keep the 64 best of nc >= 64 candidates; set the threshold and radius
        auto settle = [&]() {
            kthr = keep64(cand, nc);
            // squared distance of the 64th point, back in metres; the margin
            // covers the quantisation of both positions
            rcull = sqrtf((float)(kthr >> 20) * (1.f / 1048576.f)) + 0.01f;
        };
        bool found = false;
        // a bound stays tight while the agent moves little; after a
        // teleport (respawn, set state) the ring search is cheaper
        if (rhint <= 64.f * g.cell && moved <= 2.f * g.cell) {
            // one pass over the rows of cells that meet the disk of radius
            // rhint (which holds the 64 nearest): per row, the cells the
            // widest chord of the disk in that row spans
            kthr = hint_key(rhint);
            const int k = (int)(rhint * g.inv_cell) + 1;
            gather(Wd, 2 * k + 1, [&](int j, int &s, int &e) {
                const int y = cy - k + j;
                if (y < 0 || y >= g.ny) return;
                const float ry0 = g.y0 + (float)y * g.cell, ry1 = ry0 + g.cell;
                const float ddy = fmaxf(fmaxf(ry0 - py, py - ry1), 0.f);
                if (ddy > rhint) return;
                const float hw = sqrtf(rhint * rhint - ddy * ddy) + 1e-3f;
                const int xa = max((int)floorf((px - hw - g.x0) * g.inv_cell), 0);
                const int xb = min((int)floorf((px + hw - g.x0) * g.inv_cell), g.nx - 1);
                if (xa > xb) return;
                const int c0 = g.cbase + y * g.nx;
                s = Wd.pt_cell_start[c0 + xa];
                e = Wd.pt_cell_start[c0 + xb + 1];
                touch(Wd, SF_T_PT_START, c0 + xa);
                touch(Wd, SF_T_PT_START, c0 + xb + 1);
            }, pts, QX, QY, cand, segs, segp, nc, kthr);
            if (nc >= 64) {
                settle();
                found = true;
            } else {
                nc = 0;  // not a bound after all: search from scratch
                kthr = ~0ull;
            }
        }
        // rings closer than the distance to the nearest non-empty cell hold
        // no points: start there
        for (int rr = min(rr_first, max(g.nx, g.ny)); !found; ++rr) {
            // the ring's cells as contiguous row segments (top row, bottom
            // row, single cells of the left and right columns), one segment
            // per lane, their points flattened across the wave
            gather(Wd, rr == 0 ? 1 : 4 * rr, [&](int j, int &s, int &e) {
                int y, xa, xb;
                if (rr == 0) { y = cy; xa = xb = cx; }
                else if (j == 0) { y = cy - rr; xa = cx - rr; xb = cx + rr; }
                else if (j == 1) { y = cy + rr; xa = cx - rr; xb = cx + rr; }
                else {
                    const int qq = j - 2;
                    y = cy - rr + 1 + (qq >> 1);
                    xa = xb = (qq & 1) ? cx + rr : cx - rr;
                }
                xa = max(xa, 0);
                xb = min(xb, g.nx - 1);
                if (y < 0 || y >= g.ny || xa > xb) return;
                // distance from the agent to the segment's rectangle
                const float rx0 = g.x0 + (float)xa * g.cell, rx1 = g.x0 + (float)(xb + 1) * g.cell;
                const float ry0 = g.y0 + (float)y * g.cell, ry1 = ry0 + g.cell;
                const float ddx = fmaxf(fmaxf(rx0 - px, px - rx1), 0.f);
                const float ddy = fmaxf(fmaxf(ry0 - py, py - ry1), 0.f);
                if (ddx * ddx + ddy * ddy > rcull * rcull) return;
                const int c0 = g.cbase + y * g.nx;
                s = Wd.pt_cell_start[c0 + xa];
                e = Wd.pt_cell_start[c0 + xb + 1];
                touch(Wd, SF_T_PT_START, c0 + xa);
                touch(Wd, SF_T_PT_START, c0 + xb + 1);
            }, pts, QX, QY, cand, segs, segp, nc, kthr);
            if (nc >= 64) settle();
            // lower bound on the distance to any point outside the visited square
            float bnd = INFINITY;
            if (cx - rr > 0) bnd = fminf(bnd, px - (g.x0 + (float)(cx - rr) * g.cell));
            if (cx + rr < g.nx - 1) bnd = fminf(bnd, (g.x0 + (float)(cx + rr + 1) * g.cell) - px);
            if (cy - rr > 0) bnd = fminf(bnd, py - (g.y0 + (float)(cy - rr) * g.cell));
            if (cy + rr < g.ny - 1) bnd = fminf(bnd, (g.y0 + (float)(cy + rr + 1) * g.cell) - py);
            if (bnd == INFINITY) break;
            // every unvisited point is farther than the 64th candidate
            if (nc >= 64 && bnd > rcull) break;
        }
        wave_sync();
        // the 64 best among the buffered candidates, compacted into lanes
        unsigned long long kv[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            int slot = lane + 64 * t;
            kv[t] = slot < nc ? cand[slot] : ~0ull;
        }
        const unsigned long long kmax = nc > 64 ? kth_smallest(kv, 64, (nc + 63) >> 6) : ~0ull - 1;
        int pos = 0;
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            const bool f = kv[t] <= kmax;
            const unsigned long long bal = __ballot(f);
            const int at = pos + __popcll(bal & lane_lt());
            if (f && at < 64) sel[at] = (int)(kv[t] & 0xFFFFF);
            pos += __popcll(bal);
        }
        wave_sync();
        my_idx = lane < min(pos, 64) ? sel[lane] : 0x7fffffff;
        if (lane == 0)
            hint[n] = make_float4(px, py, nc >= 64 ? sqrtf((float)(kthr >> 20) * (1.f / 1048576.f)) : NAN, 0.f);
        // point-index order: sort the member indices across lanes
        my_idx = (int)wave_sort_u32((unsigned)my_idx);
    }
    if (dbg) dbg[(size_t)n * 72 + lane] = my_idx == 0x7fffffff ? -1 : my_idx;
    if (my_idx != 0x7fffffff) {
        touch(Wd, SF_T_ROAD, r0 + my_idx);
        const float2 rp = Wd.road_xy[r0 + my_idx];
        const float dx = rp.x - px, dy = rp.y - py;
        float *o = row + 8 + 3 * lane;
        o[0] = (hx * dx + hy * dy) / 10.f;
        o[1] = (-hy * dx + hx * dy) / 10.f;
        o[2] = (float)Wd.road_type[r0 + my_idx] / 20.f;
    }
    (void)nb_ttc_lane;
    if (Wd.forbid) shaping(P, Wd, n, r0, my_idx, px, py, qw, qx, qy, qz, hx, hy, vx, vy, goal_x, goal_y, nb_ttc);
    wave_sync();
    dst[lane] = reinterpret_cast<const float4 *>(row)[lane];
    return true;
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_obs(DevParams P, DevWorld Wd, const float *__restrict__ st,
                                                   const int *__restrict__ ist, float *__restrict__ obs,
                                                   int *__restrict__ dbg, float4 *__restrict__ hint) {
    __shared__ unsigned long long s_cand[WAVES][SF_CAND_CAP];
    __shared__ float s_row[WAVES][SF_OBS_DIM];
    __shared__ int s_sel[WAVES][64];
    __shared__ int s_segs[WAVES][64], s_segp[WAVES][64];
    const int wv = threadIdx.x >> 6;
    const int n = xcd_agent(WAVES) + wv;
    if (n >= Wd.N) return;
    obs_agent(P, Wd, st, ist, obs, dbg, hint, n, s_cand[wv], s_row[wv], s_sel[wv], s_segs[wv], s_segp[wv]);
}

// The observation of 16 agents (one wave each) followed by the policy MLP on
// their rows (the network of k_policy.hip: 256 -> 256 -> 256 -> 2, ELU,
// tanh head; bf16 operands, fp32 accumulation), so that the next control
// step's actions are ready when the observation is: the policy's own launch
// and its re-read of the observations disappear, and a workgroup whose
// agents were quick runs its network while others still search.  Wave w
// computes output columns [16 w, 16 w + 16) of each hidden layer; as soon
// as its observation is done (its registers free again) it issues the loads
// of all its weight fragments for both layers, which then arrive while the
// workgroup waits for its slowest agent.
#define OP_LD (SF_OBS_DIM + 8)  // padded bf16 activation row
#define OP_KS (SF_OBS_DIM / 32)  // k-steps of 32 per layer

// this lane's B fragments of wave w's 16 columns, all k-steps
__device__ __forceinline__ void op_fetch(const uint16_t *__restrict__ W, bf16x8 (&f)[OP_KS]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
    const uint16_t *wrow = W + (size_t)(wv * 16 + r16) * SF_OBS_DIM + kq * 8;
#pragma unroll
    for (int kk = 0; kk < OP_KS; ++kk) f[kk] = *reinterpret_cast<const bf16x8 *>(wrow + 32 * kk);
}

__device__ __forceinline__ void op_layer(const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                         const bf16x8 (&f)[OP_KS], const float *__restrict__ b) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < OP_KS; ++kk) {
        const bf16x8 af = *reinterpret_cast<const bf16x8 *>(in + r16 * OP_LD + kk * 32 + kq * 8);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, f[kk], acc, 0, 0, 0);
    }
    const int col = wv * 16 + r16;
    const float bias = b[col];
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(kq * 4 + j) * OP_LD + col] = f2bf(elu_fast(acc[j] + bias));
}

__global__ __launch_bounds__(1024) void k_obs_policy(DevParams P, DevWorld Wd, const float *__restrict__ st,
                                                     const int *__restrict__ ist, float *__restrict__ obs,
                                                     float4 *__restrict__ hint, const uint16_t *__restrict__ W1,
                                                     const float *__restrict__ b1, const uint16_t *__restrict__ W2,
                                                     const float *__restrict__ b2, const uint16_t *__restrict__ W3,
                                                     const float *__restrict__ b3, float steer_max,
                                                     float *__restrict__ act) {
    __shared__ unsigned long long s_cand[16][SF_CAND_CAP];
    __shared__ float s_row[16][SF_OBS_DIM];
    __shared__ int s_sel[16][64];
    __shared__ int s_segs[16][64], s_segp[16][64];
    __shared__ __attribute__((aligned(16))) uint16_t s_pa[16 * OP_LD], s_pb[16 * OP_LD];
    __shared__ uint16_t s_w3[2 * SF_OBS_DIM];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n0 = xcd_agent(16), n = n0 + wv;
    if (threadIdx.x < 2 * SF_OBS_DIM) s_w3[threadIdx.x] = W3[threadIdx.x];
    bool ok = false;
    if (n < Wd.N)
        ok = obs_agent(P, Wd, st, ist, obs, nullptr, hint, n, s_cand[wv], s_row[wv], s_sel[wv], s_segs[wv],
                       s_segp[wv]);
    bf16x8 f1[OP_KS], f2[OP_KS];
    op_fetch(W1, f1);
    op_fetch(W2, f2);
    // the row as bf16 (zeros for an inactive agent or past the end)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 4 * lane + q;
        s_pa[wv * OP_LD + c] = f2bf(ok ? s_row[wv][c] : 0.f);
    }
    __syncthreads();
    op_layer(s_pa, s_pb, f1, b1);
    __syncthreads();
    op_layer(s_pb, s_pa, f2, b2);
    __syncthreads();
    // head: 32 outputs, each split over 32 lanes and summed in a fixed
    // butterfly order
    {
        const int out = threadIdx.x >> 5, part = threadIdx.x & 31;
        const int row = out >> 1, o = out & 1;
        const uint16_t *h = s_pa + row * OP_LD + part * 8;
        const uint16_t *w = s_w3 + o * SF_OBS_DIM + part * 8;
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) a += bf2f(h[k]) * bf2f(w[k]);
#pragma unroll
        for (int m = 16; m > 0; m >>= 1) a += lane_xor_f(a, m);
        if (part == 0 && n0 + row < Wd.N) {
            const float z = tanhf(a + b3[o]);
            act[2 * (size_t)(n0 + row) + o] = o == 0 ? z : steer_max * z;
        }
    }
}

void launch_obs_policy(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, float *obs,
                       float4 *hint, const uint16_t *W1, const float *b1, const uint16_t *W2, const float *b2,
                       const uint16_t *W3, const float *b3, float steer_max, float *act, hipStream_t s) {
    if (Wd.N == 0) return;
    sf_launch(k_obs_policy, dim3((Wd.N + 15) / 16), dim3(1024), 0, s, P, Wd, st, ist, obs, hint, W1, b1, W2, b2, W3,
              b3, steer_max, act);
}

void launch_obs(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, float *obs,
                int *dbg_idx, float4 *hint, int waves, hipStream_t s) {
    if (Wd.N == 0) return;
    if (waves <= 1) {
        sf_launch(k_obs<1>, dim3(Wd.N), dim3(64), 0, s, P, Wd, st, ist, obs, dbg_idx, hint);
    } else if (waves <= 2) {
        sf_launch(k_obs<2>, dim3((Wd.N + 1) / 2), dim3(128), 0, s, P, Wd, st, ist, obs, dbg_idx, hint);
    } else {
        sf_launch(k_obs<4>, dim3((Wd.N + 3) / 4), dim3(256), 0, s, P, Wd, st, ist, obs, dbg_idx, hint);
    }
}

// no bound known yet for any agent
__global__ void k_hint_clear(float4 *hint, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) hint[k] = make_float4(0.f, 0.f, NAN, 0.f);
}

void launch_hint_clear(float4 *hint, int n, hipStream_t s) {
    if (n > 0) k_hint_clear<<<(n + 255) / 256, 256, 0, s>>>(hint, n);
}

// ------------------------------------------------------------ measuring
// items set in each of the SF_T_N bit ranges, added to acc[k]
__global__ void k_touch_count(const unsigned *__restrict__ bits, long long b0, long long b1,
                              unsigned long long *acc) {
    unsigned long long c = 0;
    const long long w0 = b0 >> 5, w1 = (b1 + 31) >> 5;
    for (long long wd = w0 + blockIdx.x * (long long)blockDim.x + threadIdx.x; wd < w1;
         wd += (long long)gridDim.x * blockDim.x) {
        unsigned v = bits[wd];
        // only the bits inside [b0, b1)
        if (wd == w0) v &= ~0u << (unsigned)(b0 & 31);
        if (wd == w1 - 1 && (b1 & 31)) v &= ~0u >> (32u - (unsigned)(b1 & 31));
        c += __popc(v);
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(acc, c);
}

void launch_touch_count(const unsigned *bits, const long long *off, unsigned long long *acc, hipStream_t s) {
    for (int k = 0; k < SF_T_N; ++k) {
        if (off[k + 1] <= off[k]) continue;
        const long long words = ((off[k + 1] + 31) >> 5) - (off[k] >> 5);
        const int blocks = (int)std::min<long long>((words + 255) / 256, 1024);
        k_touch_count<<<blocks, 256, 0, s>>>(bits, off[k], off[k + 1], acc + k);
    }
}
