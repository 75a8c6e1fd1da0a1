// Device-side definitions of the batched driving-physics step (gfx950).
//
// Layout in HBM
//   state   : float [SF_NUM_FFIELDS][N] and int32 [SF_NUM_IFIELDS][N]
//             (structure of arrays: lane-contiguous loads per field)
//   worlds  : CSR offsets [W+1] for agents, road points, triangles, spawns
//   roads   : float2 xy [P], int2 quantised xy [P], u8 type [P]
//   tris    : float4 [T][4] = (v0, surface) (e1, 0) (e2, friction factor)
//             (unit normal, 0)
//   grids   : per world two uniform xy grids (road points; triangles, finer);
//             cells of all worlds are numbered globally (world w owns
//             [cbase, cbase + nx*ny)); CSR over cells with the items stored
//             contiguously in cell order: road points as (quantised x,
//             quantised y, local index), triangles as full records (so a ray
//             reads its candidates without an indirection); plus, per point
//             cell, the Chebyshev distance to the nearest non-empty cell
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sf.h"

#define SF_MAXA SF_MAX_AGENTS_PER_WORLD
#define SF_CCAP SF_MAX_CONTACTS_PER_WORLD  // contact points per world and substep
#define SF_PAIR_CAP (SF_MAXA * (SF_MAXA - 1) / 2)
#define SF_KEY_CAP (1ll << 43)   // saturation of kNN squared distances
#define SF_CAND_CAP 512           // road candidates kept per agent

// learned tire surrogate: 16 -> 128 -> 128 -> 128 -> 3, flat fp32 parameters
// W1[128][16] b1 W2[128][128] b2 W3[128][128] b3 W4[3][128] b4
#define SF_SUR_IN 16
#define SF_SUR_HID 128
#define SF_SUR_SAMPLE 20  // 16 inputs, 3 targets, valid flag
#define SF_SUR_W1 0
#define SF_SUR_B1 2048
#define SF_SUR_W2 2176
#define SF_SUR_B2 18560
#define SF_SUR_W3 18688
#define SF_SUR_B3 35072
#define SF_SUR_W4 35200
#define SF_SUR_B4 35584
#define SF_SUR_PARAMS 35587
// bf16 weight copies: row-major W1 W2 W3 W4, then transposed W2 and W3
#define SF_SURB_W1 0
#define SF_SURB_W2 2048
#define SF_SURB_W3 18432
#define SF_SURB_W4 34816
#define SF_SURB_W2T 35200
#define SF_SURB_W3T 51584
#define SF_SURB_TOTAL 67968

// learned surrogate inside the step (inference + fallback) and the log of
// training samples the plain step writes
struct DevSur {
    const uint16_t *Wb;            // bf16 weight copies (SF_SURB_* layout)
    const float *P;                // fp32 parameters (biases read from here)
    float lo[SF_SUR_IN], hi[SF_SUR_IN];  // input envelope of the training set
    unsigned long long *counts;    // [2] wheels on the surrogate / on the fallback
    float *log;                    // [log_cap][SF_SUR_SAMPLE] ring, or null
    long long log_cap, log_base;
};

struct GridHdr {
    float x0, y0, cell, inv_cell;
    int nx, ny, cbase, pad;
};

// Constants of the step (derived on the host at create, passed by value).
struct DevParams {
    float mass, inv_mass;
    float inertia[3], inv_inertia[3];
    float rw, Iw, susp_k, susp_c, ell;
    float mount[4][3];
    float length, width, cr, cd;
    int Qd, Qr2;                   // quantised circle offset, (2 Qp(r))^2 (fits int32)
    float tau_drive, tau_bf, tau_br;
    float kp, kd, tau_max, Is, steer_max;
    float c_kappa, c_alpha, v_eps, trail, yaw_damping, g;
    int jacobi_iters;
    float baumgarte, slop;
    int max_ep, warmup;
    unsigned flags;
    float z_ride;
};

struct DevWorld {
    int W, N, S;
    const int *aoff, *roff, *toff, *soff;
    const int *world_of;                 // [N]
    const float2 *road_xy;               // [P]
    const float2 *road_dir;              // [P] unit polyline direction (zero if not given)
    const int2 *road_q;                  // [P]
    const uint8_t *road_type;            // [P]
    const float4 *tri;                   // [T][4]
    const float *mu;                     // [W][S]
    const float *spawn;                  // [E][5]
    const GridHdr *grid;                 // [W] road-point grid
    const int4 *agent_world;             // [N] world's first agent, agents, first road point, road points
    const GridHdr *agent_grid;           // [N] the agent's world's road-point grid header
    const GridHdr *tgrid;                // [W] triangle grid (its own cell size)
    const int *tri_cell_start;           // [CT+1]
    const float4 *tri_rec;               // [items][3] (v0, id bits) (e1, surface) (e2, friction factor), cell order
    const int *pt_cell_start;            // [CP+1]
    const int4 *pt_cell;                 // (qx, qy, local idx, 0) in cell order
    const int *pt_occ;                   // [CP] Chebyshev distance to the nearest non-empty cell
    unsigned long long *ovf;             // world-substeps whose contact points exceeded SF_CCAP
    // dense shaping rewards and the lane-forbidden event (null when off):
    // the observation kernel sets forbid for the pose it sees and, after a
    // step (shape_add), adds the dense terms to that step's reward
    uint8_t *forbid;                     // [N] a vehicle circle overlaps a road-edge segment
    float2 *disp;                        // [N] displacement of the last control step
    float *reward_out;                   // [N] the step's reward
    const uint8_t *done_out;             // [N] the step's done flags
    int shape_add;
    long long edge_half_q;               // W / 2 + r in 2^-10 m (road-edge corridor)
    unsigned long long seed;
    // measuring only (null otherwise): one bit per road item a kernel read,
    // the items of array k at bits [touch_off[k], touch_off[k + 1])
    unsigned *touch;
    long long touch_off[7];
};

// road arrays whose reads the touch bitmaps record, and their item sizes
enum { SF_T_TRI_REC, SF_T_TRI_START, SF_T_PT, SF_T_PT_START, SF_T_PT_OCC, SF_T_ROAD, SF_T_N };
#define SF_T_BYTES {48, 4, 16, 4, 4, 9}

__device__ __forceinline__ void touch(const DevWorld &Wd, int kind, long long idx) {
    if (Wd.touch) {
        const long long b = Wd.touch_off[kind] + idx;
        atomicOr(Wd.touch + (b >> 5), 1u << (unsigned)(b & 31));
    }
}

// ------------------------------------------------------------ quantisers
// positions in units of 2^-10 m, nearest-even, saturating at 2^29
__device__ __forceinline__ int qpos(float x) {
    float y = x * 1024.0f;
    if (y != y) return 0;
    if (y >= 536870912.0f) return 536870912;
    if (y <= -536870912.0f) return -536870912;
    return (int)rintf(y);
}
// quaternion components in units of 2^-14
__device__ __forceinline__ int qquat(float x) {
    float y = x * 16384.0f;
    if (y != y) return 0;
    if (y >= 32768.0f) return 32768;
    if (y <= -32768.0f) return -32768;
    return (int)rintf(y);
}
// floor(sqrt(v)) for 0 <= v < 2^62: a double estimate corrected by integers
__device__ __forceinline__ long long isqrt64(long long v) {
    long long r = (long long)sqrt((double)v);
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// SplitMix64 (Steele, Lea, Flood 2014)
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

template <int RT, int CT>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[RT][CT]) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// acc (RT x CT tiles of 16 x 16) += A B^T over KS k-steps of 32 on the
// matrix cores (v_mfma_f32_16x16x32_bf16): fa(row, k0) / fb(col, k0) return
// the 8 consecutive-k bf16 values lane (row | col) = lane % 16,
// k0 = 32 ks + 8 (lane / 16) needs; the lane then holds
// acc[r][c][j] = C[16 r + 4 (lane / 16) + j][16 c + lane % 16]
template <int RT, int CT, int KS, class FA, class FB>
__device__ __forceinline__ void mfma_nt(f32x4 (&acc)[RT][CT], FA fa, FB fb) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 32 + kq * 8;
        bf16x8 b[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) b[c] = fb(c * 16 + r16, k0);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const bf16x8 a = fa(r * 16 + r16, k0);
#pragma unroll
            for (int c = 0; c < CT; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[c], acc[r][c], 0, 0, 0);
        }
    }
}

// make one lane's LDS writes visible to the other lanes of its wave
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// round-to-nearest-even float -> bf16 bits (gfx950 converts in hardware,
// v_cvt_pk_bf16_f32), and back
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ long long sat_key(long long d2) {
    return d2 < SF_KEY_CAP ? d2 : SF_KEY_CAP - 1;
}

// ------------------------------------------------------------ lane exchange
// the value of lane (lane ^ m): lane distances 1 and 2 as quad permutes,
// 4 and 8 as a row shift in either direction chosen per lane (data-parallel
// moves, no trip through the LDS crossbar), larger ones by permute
__device__ __forceinline__ int lane_xor(int v, int m) {
    const int lane = threadIdx.x & 63;
    switch (m) {
        case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 4: {
            const int up = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0xF, false);  // row_shl:4
            const int dn = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
            return (lane & 4) ? dn : up;
        }
        case 8: {
            const int up = __builtin_amdgcn_update_dpp(0, v, 0x108, 0xF, 0xF, false);  // row_shl:8
            const int dn = __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
            return (lane & 8) ? dn : up;
        }
        default: return __shfl_xor(v, m, 64);
    }
}
__device__ __forceinline__ float lane_xor_f(float v, int m) {
    return __int_as_float(lane_xor(__float_as_int(v), m));
}
// the sum of v over lanes 0-15, in every lane: an inclusive scan along the
// row by shifts of 1, 2, 4 and 8 lanes (a lane with no source adds 0), then
// lane 15's total read out (one fixed order of additions)
__device__ __forceinline__ float row0_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, false));  // row_shr:1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, false));  // row_shr:2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, false));  // row_shr:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, false));  // row_shr:8
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 15));
}

// ------------------------------------------------------------ activations
// ELU with a cheap exp(x) - 1: the Taylor series to x^4 near 0 (relative
// error < 3e-5 for |x| < 1/4, far below the bf16 rounding that follows) and
// the hardware exponential beyond
__device__ __forceinline__ float elu_fast(float x) {
    if (x > 0.f) return x;
    if (x > -0.25f) return x * (1.f + x * (0.5f + x * (1.f / 6.f + x * (1.f / 24.f))));
    return __expf(x) - 1.f;
}

// ------------------------------------------------------------ wave sorts
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    int lo = lane_xor((int)(unsigned)v, m);
    int hi = lane_xor((int)(unsigned)(v >> 32), m);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// ascending bitonic sort of one u32 key per lane across the whole
// wavefront (one exchange per stage)
__device__ __forceinline__ unsigned wave_sort_u32(unsigned key) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned o = (unsigned)lane_xor((int)key, j);
            const bool up = (lane & k) == 0, lower = (lane & j) == 0;
            key = (lower == up) ? (key < o ? key : o) : (key > o ? key : o);
        }
    return key;
}

// the same for one u64 key per lane within each group of WIDTH lanes (32:
// the two halves of the wavefront sorted separately)
template <int WIDTH>
__device__ __forceinline__ unsigned long long wave_sort_u64(unsigned long long key) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= WIDTH; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            unsigned long long o = shfl_xor_u64(key, j);
            bool up = (lane & k) == 0, lower = (lane & j) == 0;
            key = (lower == up) ? (key < o ? key : o) : (key > o ? key : o);
        }
    return key;
}

// ------------------------------------------------------------ small math
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 add3(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 sub3(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 mul3(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// rotation matrix (row major) of a unit quaternion (w, x, y, z)
__device__ __forceinline__ void quat_R(float w, float x, float y, float z, float R[9]) {
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}
__device__ __forceinline__ f3 Rmul(const float R[9], f3 a) {
    return {R[0] * a.x + R[1] * a.y + R[2] * a.z, R[3] * a.x + R[4] * a.y + R[5] * a.z,
            R[6] * a.x + R[7] * a.y + R[8] * a.z};
}
__device__ __forceinline__ f3 RTmul(const float R[9], f3 a) {
    return {R[0] * a.x + R[3] * a.y + R[6] * a.z, R[1] * a.x + R[4] * a.y + R[7] * a.z,
            R[2] * a.x + R[5] * a.y + R[8] * a.z};
}

// Quantised three-circle centres (rear, centre, front) of a pose, as
// (x, y) pairs in units of 2^-10 m: the planar heading comes from the
// quaternion quantised to 2^-14, so the pair predicate is exact integer
// arithmetic on both sides of the parity contract.
__device__ __forceinline__ void circle_centres_q(const DevParams &P, float px, float py, float fqw, float fqx,
                                                 float fqy, float fqz, int (&cq)[6]) {
    const long long X = qpos(px), Y = qpos(py);
    const long long qw = qquat(fqw), qx = qquat(fqx), qy = qquat(fqy), qz = qquat(fqz);
    const long long hx = (1ll << 28) - 2 * (qy * qy + qz * qz);
    const long long hy = 2 * (qx * qy + qw * qz);
    const long long nh = isqrt64(hx * hx + hy * hy);
    long long ox = 0, oy = 0;
    // |Qd h| < 2^39 and nh < 2^29: the double quotient truncates to the
    // exact integer quotient (cheaper than 64-bit division)
    if (nh > 0) {
        ox = (long long)((double)((long long)P.Qd * hx) / (double)nh);
        oy = (long long)((double)((long long)P.Qd * hy) / (double)nh);
    }
    cq[0] = (int)(X - ox); cq[1] = (int)(Y - oy);
    cq[2] = (int)X;        cq[3] = (int)Y;
    cq[4] = (int)(X + ox); cq[5] = (int)(Y + oy);
}

// Swept-circle time to collision of an ego vehicle (centre p, unit heading
// h, planar velocity v) with another (m, j, w) (Sec. "Neighbor vehicles"):
// the smallest t >= 0 at which any of the 3 x 3 circle pairs (offsets
// -d, 0, +d along each heading, radius r each) touch under constant planar
// velocities, 0 if one already touches, `cap` if none ever does.
__device__ __forceinline__ float ttc_swept(const DevParams &P, float px, float py, float hx, float hy, float vx,
                                           float vy, float mx, float my, float jx, float jy, float mvx,
                                           float mvy, float cap) {
    float ttc = cap;
    const float dvx = mvx - vx, dvy = mvy - vy;
    const float R2 = 4.f * P.cr * P.cr;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            const float cx = (mx + (float)(c - 1) * P.cd * jx) - (px + (float)(a - 1) * P.cd * hx);
            const float cy = (my + (float)(c - 1) * P.cd * jy) - (py + (float)(a - 1) * P.cd * hy);
            const float c0 = cx * cx + cy * cy - R2;
            float t;
            if (c0 <= 0.f) t = 0.f;
            else {
                const float bq = 2.f * (cx * dvx + cy * dvy);
                if (bq >= 0.f) continue;
                const float aq = dvx * dvx + dvy * dvy;
                const float disc = bq * bq - 4.f * aq * c0;
                if (disc < 0.f) continue;
                t = 2.f * c0 / (-bq + sqrtf(disc));
            }
            ttc = fminf(ttc, t);
        }
    return ttc;
}

// Spawn of agent n (world w, world-local slot j) for its current episode:
// the world's spawn entries rotated by SplitMix64(seed ^ w << 32 ^ episode).
// spawn entries [s0, s0 + M) of world w
__device__ __forceinline__ void spawn_agent(const DevParams &P, const DevWorld &Wd, float *st,
                                            int *ist, int N, int n, int w, int j, int s0, int M) {
    unsigned long long e = (unsigned long long)(unsigned)ist[SF_I_EPISODE * N + n];
    unsigned long long key = Wd.seed ^ ((unsigned long long)(unsigned)w << 32) ^ e;
    int off = (int)(splitmix64(key) % (unsigned long long)M);
    const float *sp = Wd.spawn + 5 * (size_t)(s0 + (j + off) % M);
    float yaw = sp[2];
    st[SF_F_PX * N + n] = sp[0];
    st[SF_F_PY * N + n] = sp[1];
    st[SF_F_PZ * N + n] = P.z_ride;
    st[SF_F_QW * N + n] = cosf(0.5f * yaw);
    st[SF_F_QX * N + n] = 0.f;
    st[SF_F_QY * N + n] = 0.f;
    st[SF_F_QZ * N + n] = sinf(0.5f * yaw);
    for (int c = SF_F_VX; c <= SF_F_MU; ++c) st[c * N + n] = 0.f;
    st[SF_F_GOAL_X * N + n] = sp[3];
    st[SF_F_GOAL_Y * N + n] = sp[4];
    st[SF_F_START_X * N + n] = sp[0];
    st[SF_F_START_Y * N + n] = sp[1];
    ist[SF_I_ACTIVE * N + n] = 1;
    ist[SF_I_EP_STEP * N + n] = 0;
    ist[SF_I_SINCE_SPAWN * N + n] = 0;
}
__device__ __forceinline__ void spawn_agent(const DevParams &P, const DevWorld &Wd, float *st,
                                            int *ist, int N, int n, int w, int j) {
    spawn_agent(P, Wd, st, ist, N, n, w, j, Wd.soff[w], Wd.soff[w + 1] - Wd.soff[w]);
}

// what the actor-critic's forward pass keeps per row and network for the
// backward pass (floats): ego pre-activations 64 + 64, the 256 embedding
// values (bf16 values), trunk pre-activations 128 + 64, and the slot each
// pooled road and vehicle feature came from (96 + 96 ints, -1: empty set)
#define AC_SAVE_ZE1 0
#define AC_SAVE_ZE2 64
#define AC_SAVE_EMB 128
#define AC_SAVE_ZT1 384
#define AC_SAVE_ZT2 512
#define AC_SAVE_AR 576
#define AC_SAVE_AV 672
#define AC_SAVE 768
#define AC_SAVE_ROW (2 * AC_SAVE)
// bf16 weight copies of the actor-critic (both networks, padded layout)
#define SF_AC_BF16 (2 * (64 * 12 + 64 * 64 + 96 * 8 + 96 * 96 + 96 * 8 + 96 * 96 + 128 * 256 + 64 * 128))

#include "sf_launch.h"
