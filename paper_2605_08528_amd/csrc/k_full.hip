// The paper's observation and network at their own shapes (appendix
// "Observation Space Details", appendix "Network Architecture Details"):
//   k_obs_full: per agent 1929 floats = ego 11 (7 + the weather token of
//     Eq. weather_obs) | every road point within 10 m in point-index order,
//     the first 350, x 5 | the 24 nearest active agents x 7; plus the number
//     of valid road and neighbour slots;
//   k_actor_critic: the late-fusion actor-critic on those rows: per network
//     (actor, critic) ego, road and vehicle encoders, masked max-pools over
//     the valid slots, a 256 -> 128 -> 64 trunk and a head; bf16 operands on
//     the matrix cores, fp32 accumulation.
#include <climits>

#include "sf_dev.h"

#define FULL_EGO SF_FULL_EGO
#define FULL_RK SF_FULL_ROAD_K
#define FULL_VK SF_FULL_NEIGH_K
#define FULL_DIM SF_FULL_DIM
#define FULL_CAND 2048   // road candidates a wave buffers before keeping the 350 lowest indices

// ascending bitonic sort of a[0..n) in LDS by one wave (padded with INT_MAX
// up to a power of two m <= cap)
__device__ void lds_sort_ints(int *a, int n) {
    const int lane = threadIdx.x & 63;
    int m = 64;
    while (m < n) m <<= 1;
    for (int k = n + lane; k < m; k += 64) a[k] = INT_MAX;
    wave_sync();
    for (int k = 2; k <= m; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < (m >> 1); t += 64) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));   // i has bit j clear
                const int l = i | j;
                const bool up = (i & k) == 0;
                const int x = a[i], y = a[l];
                if ((x > y) == up) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            wave_sync();
        }
}

// agent of this wave: consecutive workgroups go to different XCDs, so the
// agents of one XCD (one L2) are contiguous and share their worlds' data
__device__ __forceinline__ int full_agent(int waves) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return (x * q + min(x, r) + (b >> 3)) * waves + (threadIdx.x >> 6);
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_obs_full(DevParams P, DevWorld Wd, const float *__restrict__ st,
                                                         const int *__restrict__ ist, const float *__restrict__ film,
                                                         const uint8_t *__restrict__ pav, float *__restrict__ obs,
                                                         int *__restrict__ counts) {
    __shared__ int s_cand[WAVES][FULL_CAND];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = full_agent(WAVES);
    if (n >= Wd.N) return;
    int *cand = s_cand[wv];
    const int N = Wd.N;
    float *row = obs + (size_t)n * FULL_DIM;
    const int active = ist[SF_I_ACTIVE * N + n];
    if (!active) {
        for (int k = lane; k < FULL_DIM; k += 64) row[k] = 0.f;
        if (lane == 0) { counts[2 * n] = 0; counts[2 * n + 1] = 0; }
        return;
    }
    const float px = st[SF_F_PX * N + n], py = st[SF_F_PY * N + n];
    const float qw = st[SF_F_QW * N + n], qx = st[SF_F_QX * N + n];
    const float qy = st[SF_F_QY * N + n], qz = st[SF_F_QZ * N + n];
    const float vx = st[SF_F_VX * N + n], vy = st[SF_F_VY * N + n];
    const int4 aw = Wd.agent_world[n];
    const int a0 = aw.x, A = aw.y, r0 = aw.z, PW = aw.w;
    const int w = Wd.world_of[n];
    const GridHdr g = Wd.agent_grid[n];
    float hx = 1.f - 2.f * (qy * qy + qz * qz), hy = 2.f * (qx * qy + qw * qz);
    {
        const float L = sqrtf(hx * hx + hy * hy);
        if (L < 1e-12f) { hx = 1.f; hy = 0.f; } else { hx /= L; hy /= L; }
    }

    // ---- ego: goal in the body frame, its bearing and distance, body
    //      velocity, then the world's weather token (film / 1 mm, pavement)
    if (lane < FULL_EGO) {
        const float gx = st[SF_F_GOAL_X * N + n] - px, gy = st[SF_F_GOAL_Y * N + n] - py;
        const float gbx = hx * gx + hy * gy, gby = -hy * gx + hx * gy;
        const float dist = sqrtf(gx * gx + gy * gy);
        const int pv = pav ? (pav[w] <= 2 ? pav[w] : 0) : 0;
        float e;
        switch (lane) {
            case 0: e = gbx / 100.f; break;
            case 1: e = gby / 100.f; break;
            case 2: e = dist > 0.f ? gby / dist : 0.f; break;
            case 3: e = dist > 0.f ? gbx / dist : 1.f; break;
            case 4: e = dist / 100.f; break;
            case 5: e = (hx * vx + hy * vy) / 10.f; break;
            case 6: e = (-hy * vx + hx * vy) / 10.f; break;
            case 7: e = film ? film[w] / 1.f : 0.f; break;
            default: e = (lane - 8 == pv) ? 1.f : 0.f; break;
        }
        row[lane] = e;
    }

    // ---- road: every point within 10 m (quantised squared distance,
    //      inclusive), the 350 lowest point indices, in index order
    const long long QX = qpos(px), QY = qpos(py);
    const long long R2 = 10240ll * 10240ll;
    int nc = 0;
    if (PW > 0) {
        // the cells that meet the square around the agent (with 1 cm for the
        // quantisation of positions)
        const float rr = 10.01f;
        const int xa = max((int)floorf((px - rr - g.x0) * g.inv_cell), 0);
        const int xb = min((int)floorf((px + rr - g.x0) * g.inv_cell), g.nx - 1);
        const int ya = max((int)floorf((py - rr - g.y0) * g.inv_cell), 0);
        const int yb = min((int)floorf((py + rr - g.y0) * g.inv_cell), g.ny - 1);
        for (int y = ya; y <= yb && xa <= xb; ++y) {
            const int c0 = g.cbase + y * g.nx;
            const int s0 = Wd.pt_cell_start[c0 + xa], e0 = Wd.pt_cell_start[c0 + xb + 1];
            for (int base = s0; base < e0; base += 64) {
                const int k = base + lane;
                bool in = false;
                int idx = 0;
                if (k < e0) {
                    const int4 pc = Wd.pt_cell[k];
                    const long long dx = pc.x - QX, dy = pc.y - QY;
                    in = dx * dx + dy * dy <= R2;
                    idx = pc.z;
                }
                const unsigned long long bal = __ballot(in);
                const int cnt = __popcll(bal);
                if (nc + cnt > FULL_CAND) {
                    // keep the 350 lowest indices found so far (a later
                    // point can only displace them with a lower index)
                    lds_sort_ints(cand, nc);
                    nc = min(nc, FULL_RK);
                }
                const unsigned long long below = lane ? (bal & (~0ull >> (64 - lane))) : 0ull;
                if (in) cand[nc + __popcll(below)] = idx;
                nc += cnt;
            }
        }
        wave_sync();
        lds_sort_ints(cand, nc);
    }
    const int nr = min(nc, FULL_RK);
    float *road = row + FULL_EGO;
    for (int k = lane; k < FULL_RK; k += 64) {
        float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f, f4 = 0.f;
        if (k < nr) {
            const int q = r0 + cand[k];
            const float2 rp = Wd.road_xy[q], rd = Wd.road_dir[q];
            const float dx = rp.x - px, dy = rp.y - py;
            f0 = (hx * dx + hy * dy) / 10.f;
            f1 = (-hy * dx + hx * dy) / 10.f;
            f2 = (float)Wd.road_type[q] / 20.f;
            f3 = hx * rd.x + hy * rd.y;
            f4 = -hy * rd.x + hx * rd.y;
        }
        float *o = road + 5 * k;
        o[0] = f0; o[1] = f1; o[2] = f2; o[3] = f3; o[4] = f4;
    }

    // ---- neighbours: the 24 nearest other active agents, ascending
    //      (quantised squared distance, ties by lower index)
    unsigned long long key = ~0ull;
    float ox = 0.f, oy = 0.f, oqw = 1.f, oqx = 0.f, oqy = 0.f, oqz = 0.f, ovx = 0.f, ovy = 0.f;
    if (lane < A) {
        const int m = a0 + lane;
        ox = st[SF_F_PX * N + m];
        oy = st[SF_F_PY * N + m];
        oqw = st[SF_F_QW * N + m];
        oqx = st[SF_F_QX * N + m];
        oqy = st[SF_F_QY * N + m];
        oqz = st[SF_F_QZ * N + m];
        ovx = st[SF_F_VX * N + m];
        ovy = st[SF_F_VY * N + m];
        if (m != n && ist[SF_I_ACTIVE * N + m]) {
            const long long dx = (long long)qpos(ox) - QX, dy = (long long)qpos(oy) - QY;
            key = ((unsigned long long)sat_key(dx * dx + dy * dy) << 8) | (unsigned)lane;
        }
    }
    key = A <= 32 ? wave_sort_u64<32>(key) : wave_sort_u64<64>(key);
    const int jn = key == ~0ull ? -1 : (int)(key & 0xFF);
    const unsigned long long valid = __ballot(jn >= 0 && lane < FULL_VK);
    const int nv = __popcll(valid);
    const int src = jn < 0 ? 0 : jn;
    const float mx = __shfl(ox, src, 64), my = __shfl(oy, src, 64);
    const float mqw = __shfl(oqw, src, 64), mqx = __shfl(oqx, src, 64);
    const float mqy = __shfl(oqy, src, 64), mqz = __shfl(oqz, src, 64);
    const float mvx = __shfl(ovx, src, 64), mvy = __shfl(ovy, src, 64);
    if (lane < FULL_VK) {
        float v[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (jn >= 0) {
            float jx = 1.f - 2.f * (mqy * mqy + mqz * mqz), jy = 2.f * (mqx * mqy + mqw * mqz);
            const float L = sqrtf(jx * jx + jy * jy);
            if (L < 1e-12f) { jx = 1.f; jy = 0.f; } else { jx /= L; jy /= L; }
            const float dx = mx - px, dy = my - py;
            const float bx = hx * dx + hy * dy, by = -hy * dx + hx * dy;
            float dpsi = atan2f(hx * jy - hy * jx, hx * jx + hy * jy);
            if (dpsi == -3.14159265358979f) dpsi = 3.14159265358979f;
            const float ttc = bx >= 0.f ? ttc_swept(P, px, py, hx, hy, vx, vy, mx, my, jx, jy, mvx, mvy, 10.f) : 10.f;
            v[0] = bx / 100.f;
            v[1] = by / 100.f;
            v[2] = P.length / 100.f;
            v[3] = P.width / 100.f;
            v[4] = dpsi / 3.14159265358979f;
            v[5] = sqrtf(mvx * mvx + mvy * mvy) / 10.f;
            v[6] = ttc / 10.f;
        }
        float *o = row + FULL_EGO + 5 * FULL_RK + 7 * lane;
#pragma unroll
        for (int c = 0; c < 7; ++c) o[c] = v[c];
    }
    if (lane == 0) {
        counts[2 * n] = nr;
        counts[2 * n + 1] = nv;
    }
}

void launch_obs_full(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, const float *film,
                     const uint8_t *pav, float *obs, int *counts, hipStream_t s) {
    if (Wd.N == 0) return;
    constexpr int WAVES = 4;
    sf_launch(k_obs_full<WAVES>, dim3((Wd.N + WAVES - 1) / WAVES), dim3(WAVES * 64), 0, s, P, Wd, st, ist, film, pav,
              obs, counts);
}

// ------------------------------------------------------------ actor-critic
#include "ac_layout.h"

// bf16 copies of the weight matrices in the padded layout above (one thread
// per element of both networks' blocks)
__global__ void k_ac_pack(const float *__restrict__ Pf, uint16_t *__restrict__ Wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * ACB_NET) return;
    const int net = e / ACB_NET, k = e - net * ACB_NET;
    const float *F = Pf + (size_t)net * (SF_AC_BODY + 3 * 64 + 3 + 3);
    float v = 0.f;
    if (k < ACB_EW2) { const int r = k / 12, c = k % 12; v = c < 11 ? F[ACF_EW1 + r * 11 + c] : 0.f; }
    else if (k < ACB_RW1) v = F[ACF_EW2 + (k - ACB_EW2)];
    else if (k < ACB_RW2) { const int q = k - ACB_RW1, r = q / 8, c = q % 8; v = c < 5 ? F[ACF_RW1 + r * 5 + c] : 0.f; }
    else if (k < ACB_VW1) v = F[ACF_RW2 + (k - ACB_RW2)];
    else if (k < ACB_VW2) { const int q = k - ACB_VW1, r = q / 8, c = q % 8; v = c < 7 ? F[ACF_VW1 + r * 7 + c] : 0.f; }
    else if (k < ACB_TW1) v = F[ACF_VW2 + (k - ACB_VW2)];
    else if (k < ACB_TW2) v = F[ACF_TW1 + (k - ACB_TW1)];
    else v = F[ACF_TW2 + (k - ACB_TW2)];
    Wb[e] = f2bf(v);
}

void launch_ac_pack(const float *Pf, uint16_t *Wb, hipStream_t s) {
    k_ac_pack<<<(2 * ACB_NET + 255) / 256, 256, 0, s>>>(Pf, Wb);
}

#define AC_AGENTS 8           // agents per workgroup (4 waves, 2 agents each; two workgroups per CU)
#define AC_ROWS 16            // rows of the trunk's matrix tiles (those past AC_AGENTS are zero)
#define AC_W2LD 104           // padded LDS row of a 96-wide bf16 matrix
#define AC_HLD 104            // padded row of the 32-point activation tile
#define AC_ELD 264            // padded embedding row (256)
#define AC_TLD 136            // padded trunk row (128)

__device__ __forceinline__ float bfr(float x) { return bf2f(f2bf(x)); }

// One set encoder on the valid slots of one agent (one wave): rows of K1
// features at `x` (stride K1) -> K1 -> 96 -> 96 with ELU, bf16 activations,
// then the maximum over the rows (an empty set gives 0).  32 slots per
// pass, weights as the row operand so that a lane's results are four
// consecutive features of one slot.  Returns this lane's pooled values for
// features 16 ft + 4 (lane / 16) + j in pool[ft][j].
template <int K1, bool ARG>
__device__ __forceinline__ void set_encoder(const float *__restrict__ x, int rows, const bf16x8 (&w1)[6],
                                            const float *__restrict__ b1, const uint16_t *__restrict__ w2,
                                            const float *__restrict__ b2, uint16_t *__restrict__ h,
                                            float (&pool)[6][4], int (&amax)[6][4]) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int ft = 0; ft < 6; ++ft)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            pool[ft][j] = -INFINITY;
            amax[ft][j] = -1;
        }
    for (int base = 0; base < rows; base += 32) {
        // layer 1: B fragments, slot = base + 16 g + r16, features k in [0, K1)
        bf16x8 xb[2];
#pragma unroll
        for (int gq = 0; gq < 2; ++gq) {
            const int slot = base + 16 * gq + r16;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float v = 0.f;
                if (kq == 0 && k < K1 && slot < rows) v = x[(size_t)slot * K1 + k];
                xb[gq][k] = (__bf16)v;
            }
        }
#pragma unroll
        for (int ft = 0; ft < 6; ++ft) {
            const float4 bb = *reinterpret_cast<const float4 *>(b1 + 16 * ft + 4 * kq);
#pragma unroll
            for (int gq = 0; gq < 2; ++gq) {
                f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[ft], xb[gq], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                uint16_t *o = h + (16 * gq + r16) * AC_HLD + 16 * ft + 4 * kq;
                o[0] = f2bf(elu_fast(acc[0] + bb.x));
                o[1] = f2bf(elu_fast(acc[1] + bb.y));
                o[2] = f2bf(elu_fast(acc[2] + bb.z));
                o[3] = f2bf(elu_fast(acc[3] + bb.w));
            }
        }
        wave_sync();
        // layer 2: 96 x 96 over the 32 slots
        f32x4 acc[6][2];
#pragma unroll
        for (int ft = 0; ft < 6; ++ft) acc[ft][0] = acc[ft][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) {
            const int k0 = 32 * ks + 8 * kq;
            const bf16x8 hb0 = ld8(h + r16 * AC_HLD + k0), hb1 = ld8(h + (16 + r16) * AC_HLD + k0);
#pragma unroll
            for (int ft = 0; ft < 6; ++ft) {
                const bf16x8 wa = ld8(w2 + (16 * ft + r16) * AC_W2LD + k0);
                acc[ft][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, hb0, acc[ft][0], 0, 0, 0);
                acc[ft][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, hb1, acc[ft][1], 0, 0, 0);
            }
        }
        wave_sync();   // h is overwritten by the next pass
#pragma unroll
        for (int ft = 0; ft < 6; ++ft) {
            const float4 bb = *reinterpret_cast<const float4 *>(b2 + 16 * ft + 4 * kq);
            const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int gq = 0; gq < 2; ++gq) {
                const int slot = base + 16 * gq + r16;
                if (slot >= rows) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v = bfr(elu_fast(acc[ft][gq][j] + bv[j]));
                    if (ARG) {
                        // a lane sees its slots in increasing order: the
                        // first maximum is kept
                        if (v > pool[ft][j]) {
                            pool[ft][j] = v;
                            amax[ft][j] = slot;
                        }
                    } else {
                        pool[ft][j] = fmaxf(pool[ft][j], v);
                    }
                }
            }
        }
    }
    // maximum over the 16 slot lanes of each group of four features (with
    // ARG: the lowest slot among equal maxima)
#pragma unroll
    for (int ft = 0; ft < 6; ++ft)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = pool[ft][j];
            int a = amax[ft][j];
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) {
                const float ov = lane_xor_f(v, m);
                if (ARG) {
                    const int oa = lane_xor(a, m);
                    if (ov > v || (ov == v && (unsigned)oa < (unsigned)a)) {
                        v = ov;
                        a = oa;
                    }
                } else {
                    v = fmaxf(v, ov);
                }
            }
            pool[ft][j] = rows > 0 ? v : 0.f;
            amax[ft][j] = rows > 0 ? a : -1;
        }
}

// SAVE: row n also leaves, per network, what the backward pass needs (see
// AC_SAVE_* in the header): the ego and trunk pre-activations, the
// embedding, and for each pooled feature the slot it came from.  rows (or
// null): row n reads the observation of sample rows[n].
template <bool SAVE>
__device__ __forceinline__ void actor_critic_body(const float *__restrict__ obs, const int *__restrict__ counts,
                                                      const int *__restrict__ rows, int N,
                                                      const float *__restrict__ Pf,
                                                      const uint16_t *__restrict__ Wb, float *__restrict__ mean,
                                                      float *__restrict__ value, float *__restrict__ act,
                                                      float steer_max, float *__restrict__ save) {
    __shared__ __attribute__((aligned(16))) uint16_t s_w2[96 * AC_W2LD];   // one set encoder's W2 at a time
    __shared__ __attribute__((aligned(16))) uint16_t s_h[4][32 * AC_HLD];
    __shared__ __attribute__((aligned(16))) uint16_t s_emb[AC_ROWS * AC_ELD];
    __shared__ __attribute__((aligned(16))) uint16_t s_t1[AC_ROWS * AC_TLD];
    __shared__ __attribute__((aligned(16))) uint16_t s_t2[AC_ROWS * 72];
    __shared__ float s_ego[4][64];
    __shared__ float s_mean[AC_AGENTS][3];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, kq = lane >> 4;
    const int n0 = blockIdx.x * AC_AGENTS;
    for (int net = 0; net < 2; ++net) {
        const float *F = Pf + (size_t)net * (SF_AC_BODY + 3 * 64 + 3 + 3);
        const uint16_t *B = Wb + (size_t)net * ACB_NET;
        // the road encoder's 96 x 96 matrix into LDS (padded rows); the
        // vehicle encoder's takes its place after the road pass
        for (int e = tid; e < 96 * 12; e += 256) {
            const int r = e / 12, c = (e % 12) * 8;
            *reinterpret_cast<uint4 *>(s_w2 + r * AC_W2LD + c) = *reinterpret_cast<const uint4 *>(B + ACB_RW2 + r * 96 + c);
        }
        // the trunk tiles' rows past the workgroup's agents stay zero
        for (int e = tid; e < (AC_ROWS - AC_AGENTS) * AC_ELD; e += 256) s_emb[AC_AGENTS * AC_ELD + e] = 0;
        __syncthreads();
        // ---- ego and road encoders: wave wv, its agents one after the other
        {
            // first-layer fragments (rows 16 ft + r16, inputs 0..7 in the
            // first quarter of the lanes, zero elsewhere)
            bf16x8 rw1[6];
#pragma unroll
            for (int ft = 0; ft < 6; ++ft) rw1[ft] = kq == 0 ? ld8(B + ACB_RW1 + (16 * ft + r16) * 8) : zero8();
            for (int t = 0; t < AC_AGENTS / 4; ++t) {
                const int a = wv * (AC_AGENTS / 4) + t, n = n0 + a;
                uint16_t *emb = s_emb + a * AC_ELD;
                if (n >= N) {
                    for (int k = lane; k < 256; k += 64) emb[k] = 0;
                    continue;
                }
                const int src = rows ? rows[n] : n;
                const float *o = obs + (size_t)src * FULL_DIM;
                const int nr = counts[2 * src];
                float *sv = SAVE ? save + (size_t)n * AC_SAVE_ROW + net * AC_SAVE : nullptr;
                // ego 11 -> 64 -> 64 (lane = feature)
                {
                    float acc = F[ACF_EB1 + lane];
                    for (int k = 0; k < 11; ++k) acc += bf2f(B[ACB_EW1 + lane * 12 + k]) * bfr(o[k]);
                    s_ego[wv][lane] = bfr(elu_fast(acc));
                    wave_sync();
                    float acc2 = F[ACF_EB2 + lane];
                    const uint16_t *w2 = B + ACB_EW2 + lane * 64;
                    for (int k = 0; k < 64; ++k) acc2 += bf2f(w2[k]) * s_ego[wv][k];
                    emb[lane] = f2bf(elu_fast(acc2));
                    if (SAVE) {
                        sv[AC_SAVE_ZE1 + lane] = acc;
                        sv[AC_SAVE_ZE2 + lane] = acc2;
                    }
                    wave_sync();
                }
                float pool[6][4];
                int amax[6][4];
                set_encoder<5, SAVE>(o + FULL_EGO, min(nr, FULL_RK), rw1, F + ACF_RB1, s_w2, F + ACF_RB2, s_h[wv],
                                     pool, amax);
                if (r16 == 0) {
#pragma unroll
                    for (int ft = 0; ft < 6; ++ft)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            emb[64 + 16 * ft + 4 * kq + j] = f2bf(pool[ft][j]);
                            if (SAVE) sv[AC_SAVE_AR + 16 * ft + 4 * kq + j] = __int_as_float(amax[ft][j]);
                        }
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < 96 * 12; e += 256) {
            const int r = e / 12, c = (e % 12) * 8;
            *reinterpret_cast<uint4 *>(s_w2 + r * AC_W2LD + c) = *reinterpret_cast<const uint4 *>(B + ACB_VW2 + r * 96 + c);
        }
        __syncthreads();
        // ---- vehicle encoder
        {
            bf16x8 vw1[6];
#pragma unroll
            for (int ft = 0; ft < 6; ++ft) vw1[ft] = kq == 0 ? ld8(B + ACB_VW1 + (16 * ft + r16) * 8) : zero8();
            for (int t = 0; t < AC_AGENTS / 4; ++t) {
                const int a = wv * (AC_AGENTS / 4) + t, n = n0 + a;
                if (n >= N) continue;
                uint16_t *emb = s_emb + a * AC_ELD;
                const int src = rows ? rows[n] : n;
                const float *o = obs + (size_t)src * FULL_DIM;
                const int nv = counts[2 * src + 1];
                float *sv = SAVE ? save + (size_t)n * AC_SAVE_ROW + net * AC_SAVE : nullptr;
                float pool[6][4];
                int amax[6][4];
                set_encoder<7, SAVE>(o + FULL_EGO + 5 * FULL_RK, min(nv, FULL_VK), vw1, F + ACF_VB1, s_w2, F + ACF_VB2,
                                     s_h[wv], pool, amax);
                if (r16 == 0) {
#pragma unroll
                    for (int ft = 0; ft < 6; ++ft)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            emb[160 + 16 * ft + 4 * kq + j] = f2bf(pool[ft][j]);
                            if (SAVE) sv[AC_SAVE_AV + 16 * ft + 4 * kq + j] = __int_as_float(amax[ft][j]);
                        }
                }
                if (SAVE) {
                    wave_sync();
                    for (int k = lane; k < 256; k += 64) sv[AC_SAVE_EMB + k] = bf2f(emb[k]);
                }
            }
        }
        __syncthreads();
        // ---- trunk 256 -> 128: wave wv owns output columns [32 wv, 32 wv + 32)
        {
            f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const int k0 = 32 * ks + 8 * kq;
                const bf16x8 ea = ld8(s_emb + r16 * AC_ELD + k0);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const bf16x8 wb = ld8(B + ACB_TW1 + (size_t)(32 * wv + 16 * c + r16) * 256 + k0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea, wb, acc[c], 0, 0, 0);
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int col = 32 * wv + 16 * c + r16;
                const float bb = F[ACF_TB1 + col];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    s_t1[(4 * kq + j) * AC_TLD + col] = f2bf(elu_fast(acc[c][j] + bb));
                    if (SAVE && 4 * kq + j < AC_AGENTS && n0 + 4 * kq + j < N)
                        save[(size_t)(n0 + 4 * kq + j) * AC_SAVE_ROW + net * AC_SAVE + AC_SAVE_ZT1 + col] = acc[c][j] + bb;
                }
            }
        }
        __syncthreads();
        // ---- trunk 128 -> 64: wave wv owns columns [16 wv, 16 wv + 16)
        {
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k0 = 32 * ks + 8 * kq;
                const bf16x8 ta = ld8(s_t1 + r16 * AC_TLD + k0);
                const bf16x8 wb = ld8(B + ACB_TW2 + (size_t)(16 * wv + r16) * 128 + k0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ta, wb, acc, 0, 0, 0);
            }
            const int col = 16 * wv + r16;
            const float bb = F[ACF_TB2 + col];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s_t2[(4 * kq + j) * 72 + col] = f2bf(elu_fast(acc[j] + bb));
                if (SAVE && 4 * kq + j < AC_AGENTS && n0 + 4 * kq + j < N)
                    save[(size_t)(n0 + 4 * kq + j) * AC_SAVE_ROW + net * AC_SAVE + AC_SAVE_ZT2 + col] = acc[j] + bb;
            }
        }
        __syncthreads();
        // ---- heads: actor mean (3 per agent), critic value (1 per agent)
        const int nout = net == 0 ? 3 : 1;
        if (tid < AC_AGENTS * nout) {
            const int a = tid / nout, o = tid % nout, n = n0 + a;
            const float *Wh = F + ACF_HEAD + o * 64;
            float acc = F[ACF_HEAD + nout * 64 + o];
            for (int k = 0; k < 64; ++k) acc += bfr(Wh[k]) * bf2f(s_t2[a * 72 + k]);
            if (n < N) {
                if (net == 0) {
                    mean[3 * (size_t)n + o] = acc;
                    s_mean[a][o] = acc;
                } else {
                    value[n] = acc;
                }
            }
        }
        __syncthreads();
        // actions from the actor's mean: throttle and brake rectified to
        // [0, 1], steering clamped to [-1, 1] (appendix "Action Space
        // Details"), then (a_long, steer) = (throttle - brake, steer_max s)
        if (net == 0 && act && tid < AC_AGENTS && n0 + tid < N) {
            const float thr = fminf(fmaxf(s_mean[tid][0], 0.f), 1.f);
            const float str = fminf(fmaxf(s_mean[tid][1], -1.f), 1.f);
            const float brk = fminf(fmaxf(s_mean[tid][2], 0.f), 1.f);
            act[2 * (size_t)(n0 + tid)] = thr - brk;
            act[2 * (size_t)(n0 + tid) + 1] = steer_max * str;
        }
    }
}

// inference: two workgroups per CU (the registers fit without spilling)
__global__ __launch_bounds__(256, 2) void k_actor_critic(const float *__restrict__ obs,
                                                         const int *__restrict__ counts, int N,
                                                         const float *__restrict__ Pf,
                                                         const uint16_t *__restrict__ Wb, float *__restrict__ mean,
                                                         float *__restrict__ value, float *__restrict__ act,
                                                         float steer_max) {
    actor_critic_body<false>(obs, counts, nullptr, N, Pf, Wb, mean, value, act, steer_max, nullptr);
}

// the training forward pass (pooled slots in registers: one workgroup per CU)
__global__ __launch_bounds__(256) void k_actor_critic_save(const float *__restrict__ obs,
                                                           const int *__restrict__ counts,
                                                           const int *__restrict__ rows, int M,
                                                           const float *__restrict__ Pf,
                                                           const uint16_t *__restrict__ Wb, float *__restrict__ mean,
                                                           float *__restrict__ value, float *__restrict__ save) {
    actor_critic_body<true>(obs, counts, rows, M, Pf, Wb, mean, value, nullptr, 0.f, save);
}

void launch_actor_critic(const float *obs, const int *counts, int N, const float *Pf, const uint16_t *Wb,
                         float *mean, float *value, float *act, float steer_max, hipStream_t s) {
    if (N == 0) return;
    sf_launch(k_actor_critic, dim3((N + AC_AGENTS - 1) / AC_AGENTS), dim3(256), 0, s, obs, counts, N, Pf, Wb, mean,
              value, act, steer_max);
}

void launch_actor_critic_save(const float *obs, const int *counts, const int *rows, int M, const float *Pf,
                              const uint16_t *Wb, float *mean, float *value, float *save, hipStream_t s) {
    if (M == 0) return;
    sf_launch(k_actor_critic_save, dim3((M + AC_AGENTS - 1) / AC_AGENTS), dim3(256), 0, s, obs, counts, rows, M, Pf,
              Wb, mean, value, save);
}
