// On-device PPO around the late-fusion actor-critic (Algorithm "SceneFactory
// Pipeline": after T rollout steps a PPO update on the transitions; appendix
// "PPO Hyperparameters"):
//   k_ppo_sample    actions drawn from the diagonal Gaussian policy (mean
//                   from the actor, state-independent log sigma) with the
//                   caller's standard normals, their log-density, and the
//                   2-action decode the step takes;
//   k_ppo_gae       generalised advantage estimation, one thread per agent
//                   walking the rollout backwards;
//   k_ppo_moments / k_ppo_normalise   advantages to zero mean, unit spread;
//   k_ppo_loss      per minibatch row: ratio, clipped surrogate, value
//                   error, KL to the rollout's policy, and the gradient of
//                   the loss with respect to the network's outputs;
//   k_ppo_backward  back-propagation through both networks for a tile of
//                   16 rows: trunk, heads and ego encoder as dense layers,
//                   each set encoder only through the slot its max-pool
//                   took each feature from; one partial gradient per tile;
//   k_ppo_reduce / k_ppo_sqnorm / k_ppo_adam   tile partials summed in a
//                   fixed order, the global norm clipped, Adam.
// Every sum runs in a fixed order, so an update is deterministic.
#include "sf_dev.h"
#include "ac_layout.h"

#define PPO_TILE 16
#define LOG_2PI 1.8378770664093453f

__device__ __forceinline__ float eluf(float x) { return elu_fast(x); }
// derivative of ELU at the pre-activation
__device__ __forceinline__ float elu_d(float z) { return z > 0.f ? 1.f : __expf(z); }
__device__ __forceinline__ float bfr1(float x) { return bf2f(f2bf(x)); }

// log N(u; mu, diag exp(2 ls)) over the 3 action dimensions
__device__ __forceinline__ float gauss_logp(const float (&u)[3], const float (&mu)[3], const float (&ls)[3]) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float z = (u[k] - mu[k]) / __expf(ls[k]);
        s += -0.5f * z * z - ls[k] - 0.5f * LOG_2PI;
    }
    return s;
}

// ------------------------------------------------------------------ rollout
__global__ void k_ppo_sample(const float *__restrict__ mean, const float *__restrict__ Pf,
                             const float *__restrict__ eps, int N, float *__restrict__ u_out,
                             float *__restrict__ logp, float *__restrict__ mu_out, float *__restrict__ act,
                             float steer_max) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float u[3], mu[3], ls[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ls[k] = Pf[ACF_LOGSTD + k];
        mu[k] = mean[3 * (size_t)n + k];
        u[k] = mu[k] + __expf(ls[k]) * eps[3 * (size_t)n + k];
        u_out[3 * (size_t)n + k] = u[k];
        mu_out[3 * (size_t)n + k] = mu[k];
    }
    logp[n] = gauss_logp(u, mu, ls);
    // the environment's actions: throttle and brake rectified, steering
    // clamped, as for the deterministic actions
    const float thr = fminf(fmaxf(u[0], 0.f), 1.f), str = fminf(fmaxf(u[1], -1.f), 1.f);
    const float brk = fminf(fmaxf(u[2], 0.f), 1.f);
    act[2 * (size_t)n] = thr - brk;
    act[2 * (size_t)n + 1] = steer_max * str;
}

void launch_ppo_sample(const float *mean, const float *Pf, const float *eps, int N, float *u, float *logp, float *mu,
                       float *act, float steer_max, hipStream_t s) {
    if (N > 0) k_ppo_sample<<<(N + 255) / 256, 256, 0, s>>>(mean, Pf, eps, N, u, logp, mu, act, steer_max);
}

// ---------------------------------------------------------------- advantages
// rew, done [T][N]; val [T + 1][N] (the last row: the bootstrap value)
__global__ void k_ppo_gae(const float *__restrict__ rew, const uint8_t *__restrict__ done,
                          const float *__restrict__ val, int T, int N, float gamma, float lam,
                          float *__restrict__ adv, float *__restrict__ ret) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float nv = val[(size_t)T * N + n], na = 0.f;
    for (int t = T - 1; t >= 0; --t) {
        const size_t i = (size_t)t * N + n;
        const float keep = done[i] ? 0.f : 1.f;
        const float v = val[i];
        const float delta = rew[i] + gamma * nv * keep - v;
        na = delta + gamma * lam * keep * na;
        adv[i] = na;
        ret[i] = na + v;
        nv = v;
    }
}

#define MOM_BLOCK 256
#define MOM_ITEMS 8
// per block: the sum and the sum of squares of its MOM_BLOCK * MOM_ITEMS
// consecutive advantages, in double, in a fixed tree order
__global__ __launch_bounds__(MOM_BLOCK) void k_ppo_moments(const float *__restrict__ a, long long n,
                                                          double *__restrict__ part) {
    __shared__ double s1[MOM_BLOCK], s2[MOM_BLOCK];
    const long long base = (long long)blockIdx.x * MOM_BLOCK * MOM_ITEMS;
    double x = 0.0, y = 0.0;
    for (int k = 0; k < MOM_ITEMS; ++k) {
        const long long i = base + (long long)k * MOM_BLOCK + threadIdx.x;
        if (i < n) {
            const double v = a[i];
            x += v;
            y += v * v;
        }
    }
    s1[threadIdx.x] = x;
    s2[threadIdx.x] = y;
    __syncthreads();
    for (int h = MOM_BLOCK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// every thread adds the block partials in order (a few hundred), then
// (a - mean) / (std + 1e-8), the population spread
__global__ void k_ppo_normalise(float *__restrict__ a, long long n, const double *__restrict__ part, int nb) {
    double s = 0.0, q = 0.0;
    for (int b = 0; b < nb; ++b) {
        s += part[2 * b];
        q += part[2 * b + 1];
    }
    const double mean = s / (double)n, var = fmax(q / (double)n - mean * mean, 0.0);
    const float m = (float)mean, inv = (float)(1.0 / (sqrt(var) + 1e-8));
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (a[i] - m) * inv;
}

void launch_ppo_advantages(const float *rew, const uint8_t *done, const float *val, int T, int N, float gamma,
                           float lam, float *adv, float *ret, double *part, hipStream_t s) {
    if (N == 0 || T == 0) return;
    k_ppo_gae<<<(N + 255) / 256, 256, 0, s>>>(rew, done, val, T, N, gamma, lam, adv, ret);
    const long long n = (long long)T * N;
    const int nb = (int)((n + MOM_BLOCK * MOM_ITEMS - 1) / (MOM_BLOCK * MOM_ITEMS));
    k_ppo_moments<<<nb, MOM_BLOCK, 0, s>>>(adv, n, part);
    k_ppo_normalise<<<(int)((n + 255) / 256), 256, 0, s>>>(adv, n, part, nb);
}

int ppo_moment_blocks(long long n) { return (int)((n + MOM_BLOCK * MOM_ITEMS - 1) / (MOM_BLOCK * MOM_ITEMS)); }

// --------------------------------------------------------------------- loss
#define LOSS_BLOCK 256
// Row r of the minibatch is rollout sample rows[r].  dout[r]: d loss / d
// (mean[3], value) of that row, already over the batch size; part[block]:
// the block's sums of the surrogate, squared value error, KL, clipped
// count and d loss / d log sigma (3), in a fixed tree order.
__global__ __launch_bounds__(LOSS_BLOCK) void k_ppo_loss(const int *__restrict__ rows, int B,
                                                        const float *__restrict__ mean_new,
                                                        const float *__restrict__ val_new,
                                                        const float *__restrict__ u_all,
                                                        const float *__restrict__ logp_old,
                                                        const float *__restrict__ mu_old,
                                                        const float *__restrict__ adv, const float *__restrict__ ret,
                                                        const float *__restrict__ Pf, float ls_old0, float ls_old1,
                                                        float ls_old2, float clip, float c_v,
                                                        float *__restrict__ dout, float *__restrict__ part) {
    __shared__ float red[7][LOSS_BLOCK];
    const int r = blockIdx.x * LOSS_BLOCK + threadIdx.x;
    float acc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (r < B) {
        const int i = rows[r];
        float u[3], mu[3], ls[3], mo[3];
        const float lso[3] = {ls_old0, ls_old1, ls_old2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            u[k] = u_all[3 * (size_t)i + k];
            mu[k] = mean_new[3 * (size_t)r + k];
            ls[k] = Pf[ACF_LOGSTD + k];
            mo[k] = mu_old[3 * (size_t)i + k];
        }
        const float lp = gauss_logp(u, mu, ls);
        const float ratio = __expf(lp - logp_old[i]);
        const float A = adv[i];
        const float s1 = -A * ratio, s2 = -A * fminf(fmaxf(ratio, 1.f - clip), 1.f + clip);
        // the unclipped branch carries the gradient when it is the larger
        const float glp = s1 >= s2 ? -A * ratio : 0.f;
        const float invB = 1.f / (float)B;
        acc[0] = fmaxf(s1, s2);
        const float dv = val_new[r] - ret[i];
        acc[1] = dv * dv;
        float kl = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float s = __expf(ls[k]), so = __expf(lso[k]);
            const float z = (u[k] - mu[k]) / s;
            dout[4 * (size_t)r + k] = glp * z / s * invB;
            acc[4 + k] = glp * (z * z - 1.f) * invB;
            kl += ls[k] - lso[k] + (so * so + (mo[k] - mu[k]) * (mo[k] - mu[k])) / (2.f * s * s) - 0.5f;
        }
        acc[2] = kl;
        acc[3] = fabsf(ratio - 1.f) > clip ? 1.f : 0.f;
        dout[4 * (size_t)r + 3] = 2.f * c_v * dv * invB;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = LOSS_BLOCK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 7; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 7) part[8 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// one block: the loss partials in order -> stats[8] = (surrogate, value
// error, KL) means, clipped fraction, d / d log sigma (3), rows
__global__ void k_ppo_stats(const float *__restrict__ part, int nb, int B, double *__restrict__ stats) {
    if (threadIdx.x >= 7) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[8 * b + threadIdx.x];
    stats[threadIdx.x] = threadIdx.x < 4 ? s / (double)B : s;
    if (threadIdx.x == 0) stats[7] = (double)B;
}

void launch_ppo_loss(const int *rows, int B, const float *mean_new, const float *val_new, const float *u,
                     const float *logp_old, const float *mu_old, const float *adv, const float *ret, const float *Pf,
                     const float *ls_old, float clip, float c_v, float *dout, float *part, double *stats,
                     hipStream_t s) {
    const int nb = (B + LOSS_BLOCK - 1) / LOSS_BLOCK;
    k_ppo_loss<<<nb, LOSS_BLOCK, 0, s>>>(rows, B, mean_new, val_new, u, logp_old, mu_old, adv, ret, Pf, ls_old[0],
                                         ls_old[1], ls_old[2], clip, c_v, dout, part);
    k_ppo_stats<<<1, 64, 0, s>>>(part, nb, B, stats);
}

// ----------------------------------------------------------------- backward
// LDS of one tile (floats).  Dense phase: the 16 rows' output gradients,
// activations and back-propagated vectors; encoder phase: the encoder's
// weights (bf16, W2 rows padded to 98 so that the lanes of a wave read
// different banks) and biases, per channel the layer-1 activations of the
// slot it pooled from (bf16), their ELU derivatives, the slot's inputs and
// the channel's layer-2 gradient.  The embedding gradient stays at the
// front through both.
#define W2P 98
#define BW_DEMB 0
#define BW_DENSE (BW_DEMB + PPO_TILE * 256)
#define BW_DO (BW_DENSE)
#define BW_T2 (BW_DO + PPO_TILE * 4)
#define BW_DZT2 (BW_T2 + PPO_TILE * 64)
#define BW_T1 (BW_DZT2 + PPO_TILE * 64)
#define BW_DZT1 (BW_T1 + PPO_TILE * 128)
#define BW_EMB (BW_DZT1 + PPO_TILE * 128)
#define BW_E1 (BW_EMB + PPO_TILE * 256)
#define BW_DZE2 (BW_E1 + PPO_TILE * 64)
#define BW_DZE1 (BW_DZE2 + PPO_TILE * 64)
#define BW_XEGO (BW_DZE1 + PPO_TILE * 64)
#define BW_DENSE_END (BW_XEGO + PPO_TILE * 12)
#define BW_W2 (BW_DENSE)                      // 96 x 98 bf16 = 4704 floats
#define BW_W1 (BW_W2 + 96 * W2P / 2)          // 96 x 8 bf16 = 384 floats
#define BW_B1 (BW_W1 + 96 * 8 / 2)
#define BW_B2 (BW_B1 + 96)
// per-channel rows padded to odd word pitches, so that the 64 lanes of a
// wave, one channel each, write their rows through different banks
#define HP 98                                 // bf16 per H row (49 words)
#define DP 97                                 // floats per D1 row
#define XP 9                                  // floats per X row
#define BW_H (BW_B2 + 96)                     // 96 x 98 bf16 = 4704 floats
#define BW_D1 (BW_H + 96 * HP / 2)
#define BW_X (BW_D1 + 96 * DP)
#define BW_DZ (BW_X + 96 * XP)
#define BW_ENC_END (BW_DZ + 96)
#define BW_FLOATS (BW_DENSE_END > BW_ENC_END ? BW_DENSE_END : BW_ENC_END)

// one set encoder's gradient over the tile's rows: K1 inputs per slot at
// `xoff` of the observation with stride K1, pooled slots at save offset
// `soff`, embedding gradient at columns [eoff, eoff + 96)
template <int K1>
__device__ void encoder_backward(float *sm, const float *__restrict__ obs, const int *__restrict__ rows, int B,
                                 int r0, const float *__restrict__ save, int net, int soff, int xoff, int eoff,
                                 const float *__restrict__ F, int fw1, int fb1, int fw2, int fb2,
                                 const uint16_t *__restrict__ bw1, const uint16_t *__restrict__ bw2,
                                 float *__restrict__ g) {
    const int tid = threadIdx.x;
    uint16_t *W2 = reinterpret_cast<uint16_t *>(sm + BW_W2), *W1 = reinterpret_cast<uint16_t *>(sm + BW_W1);
    uint16_t *H = reinterpret_cast<uint16_t *>(sm + BW_H);
    float *B1 = sm + BW_B1, *B2 = sm + BW_B2, *D1 = sm + BW_D1, *X = sm + BW_X, *DZ = sm + BW_DZ;
    // the encoder's weights and biases into LDS
    for (int e = tid; e < 96 * 96; e += 256) W2[(e / 96) * W2P + e % 96] = bw2[e];
    for (int e = tid; e < 96 * 8; e += 256) W1[e] = bw1[e];
    if (tid < 96) {
        B1[tid] = F[fb1 + tid];
        B2[tid] = F[fb2 + tid];
    }
    __syncthreads();
    float acc2[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) acc2[i] = 0.f;
    constexpr int N1 = 96 * K1 + 96 + 96;          // W1, b1, b2
    float acc1[(N1 + 255) / 256];
#pragma unroll
    for (int i = 0; i < (N1 + 255) / 256; ++i) acc1[i] = 0.f;
    __shared__ int s_slot[96];
    for (int s = 0; s < PPO_TILE; ++s) {
        const int r = r0 + s;
        if (r >= B) break;
        // the slot each channel pooled from and that slot's inputs
        if (tid < 96) {
            const int c = tid;
            const int slot = __float_as_int(save[(size_t)r * AC_SAVE_ROW + net * AC_SAVE + soff + c]);
            s_slot[c] = slot;
            const float *xs = obs + (size_t)rows[r] * SF_FULL_DIM + xoff + (size_t)(slot < 0 ? 0 : slot) * K1;
#pragma unroll
            for (int k = 0; k < K1; ++k) X[c * XP + k] = slot < 0 ? 0.f : bfr1(xs[k]);
        }
        __syncthreads();
        // layer 1 of channel c's slot, feature j, for every (c, j)
#pragma unroll 4
        for (int i = 0; i < 36; ++i) {
            const int e = tid + 256 * i, c = e / 96, j = e - 96 * c;
            float z1 = B1[j];
#pragma unroll
            for (int k = 0; k < K1; ++k) z1 += bf2f(W1[j * 8 + k]) * X[c * XP + k];
            H[c * HP + j] = f2bf(eluf(z1));
            D1[c * DP + j] = elu_d(z1);
        }
        __syncthreads();
        // channel c's layer-2 pre-activation and gradient
        if (tid < 96) {
            const int c = tid;
            float z2 = B2[c];
            const uint16_t *w2r = W2 + c * W2P;
            for (int j = 0; j < 96; ++j) z2 += bf2f(w2r[j]) * bf2f(H[c * HP + j]);
            DZ[c] = s_slot[c] < 0 ? 0.f : sm[BW_DEMB + s * 256 + eoff + c] * elu_d(z2);
        }
        __syncthreads();
        // layer 2 weights (thread-owned entries), and v_c[j] = dz_c W2[c][j]
        // ELU'(z1_c[j]) in place of the derivative
#pragma unroll
        for (int i = 0; i < 36; ++i) {
            const int e = tid + 256 * i, c = e / 96, j = e - 96 * c;
            const float dz = DZ[c];
            acc2[i] += dz * bf2f(H[c * HP + j]);
            D1[c * DP + j] = dz * bf2f(W2[c * W2P + j]) * D1[c * DP + j];
        }
        __syncthreads();
        // layer 1 weights and both biases
#pragma unroll
        for (int i = 0; i < (N1 + 255) / 256; ++i) {
            const int e = tid + 256 * i;
            if (e >= N1) break;
            float a = 0.f;
            if (e < 96 * K1) {
                const int j = e / K1, k = e - K1 * j;
                for (int c = 0; c < 96; ++c) a += D1[c * DP + j] * X[c * XP + k];
            } else if (e < 96 * K1 + 96) {
                const int j = e - 96 * K1;
                for (int c = 0; c < 96; ++c) a += D1[c * DP + j];
            } else {
                a = DZ[e - 96 * K1 - 96];
            }
            acc1[i] += a;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 36; ++i) g[fw2 + tid + 256 * i] = acc2[i];
#pragma unroll
    for (int i = 0; i < (N1 + 255) / 256; ++i) {
        const int e = tid + 256 * i;
        if (e >= N1) break;
        if (e < 96 * K1) g[fw1 + e] = acc1[i];
        else if (e < 96 * K1 + 96) g[fb1 + e - 96 * K1] = acc1[i];
        else g[fb2 + e - 96 * K1 - 96] = acc1[i];
    }
    __syncthreads();   // the encoder buffers are reused next
}

// y[s][k] = sum_i x[s][i] W[i][k] for the tile's rows, W row-major [n_in][ld]
// (bf16): thread k keeps the 16 rows' sums, so each weight is read once
__device__ __forceinline__ void tile_matvec_t(const float *x, int xld, const uint16_t *__restrict__ W, int ld,
                                              int n_in, int k, float (&acc)[PPO_TILE]) {
#pragma unroll
    for (int s = 0; s < PPO_TILE; ++s) acc[s] = 0.f;
    for (int i = 0; i < n_in; ++i) {
        const float w = bf2f(W[(size_t)i * ld + k]);
#pragma unroll
        for (int s = 0; s < PPO_TILE; ++s) acc[s] += x[s * xld + i] * w;
    }
}

// G[i][k] = sum_s dz[s][i] a[s][k] (+ bias column: sum_s dz[s][i]) for
// thread k: the 16 activations of column k stay in registers
__device__ __forceinline__ void tile_outer(const float *dz, int dzld, int n_out, const float *a, int ald, int k,
                                           float *__restrict__ G, int gld) {
    float ak[PPO_TILE];
#pragma unroll
    for (int s = 0; s < PPO_TILE; ++s) ak[s] = a[s * ald + k];
    for (int i = 0; i < n_out; ++i) {
        float v = 0.f;
#pragma unroll
        for (int s = 0; s < PPO_TILE; ++s) v += dz[s * dzld + i] * ak[s];
        G[(size_t)i * gld + k] = v;
    }
}

__global__ __launch_bounds__(256) void k_ppo_backward(const float *__restrict__ obs, const int *__restrict__ rows,
                                                     int B, const float *__restrict__ save,
                                                     const float *__restrict__ dout, const float *__restrict__ Pf,
                                                     const uint16_t *__restrict__ Wb, float *__restrict__ part) {
    extern __shared__ float sm[];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * PPO_TILE;
    float *gt = part + (size_t)blockIdx.x * SF_AC_PARAMS;
    for (int net = 0; net < 2; ++net) {
        const float *F = Pf + (size_t)net * ACF_NET0;
        const uint16_t *Bw = Wb + (size_t)net * ACB_NET;
        float *g = gt + (size_t)net * ACF_NET0;
        const int nout = net == 0 ? 3 : 1;
        // ---- load the tile's rows (rows past the batch are zero)
        for (int e = tid; e < PPO_TILE * 256; e += 256) {
            const int s = e >> 8, k = e & 255, r = r0 + s;
            const float *sv = save + (size_t)r * AC_SAVE_ROW + net * AC_SAVE;
            const bool ok = r < B;
            sm[BW_EMB + e] = ok ? sv[AC_SAVE_EMB + k] : 0.f;
            if (k < 128) sm[BW_T1 + s * 128 + k] = ok ? bfr1(eluf(sv[AC_SAVE_ZT1 + k])) : 0.f;
            if (k < 64) {
                sm[BW_T2 + s * 64 + k] = ok ? bfr1(eluf(sv[AC_SAVE_ZT2 + k])) : 0.f;
                sm[BW_E1 + s * 64 + k] = ok ? bfr1(eluf(sv[AC_SAVE_ZE1 + k])) : 0.f;
            }
            if (k < 12) sm[BW_XEGO + s * 12 + k] = ok && k < SF_FULL_EGO ? bfr1(obs[(size_t)rows[r] * SF_FULL_DIM + k]) : 0.f;
            if (k < 4) sm[BW_DO + s * 4 + k] = ok ? (net == 0 ? (k < 3 ? dout[4 * (size_t)r + k] : 0.f)
                                                              : (k == 0 ? dout[4 * (size_t)r + 3] : 0.f))
                                                  : 0.f;
        }
        __syncthreads();
        const float *svb = save + (size_t)r0 * AC_SAVE_ROW + net * AC_SAVE;   // row s at svb + s * AC_SAVE_ROW
        auto zsave = [&](int s, int off) -> float { return r0 + s < B ? svb[(size_t)s * AC_SAVE_ROW + off] : 0.f; };
        // ---- head -> trunk 2: dz_t2 = (W_head^T d_out) ELU'(z_t2)
        if (tid < 64) {
            const int k = tid;
            float w[3];
            for (int o = 0; o < nout; ++o) w[o] = bfr1(F[ACF_HEAD + o * 64 + k]);
            for (int s = 0; s < PPO_TILE; ++s) {
                float a = 0.f;
                for (int o = 0; o < nout; ++o) a += sm[BW_DO + s * 4 + o] * w[o];
                sm[BW_DZT2 + s * 64 + k] = r0 + s < B ? a * elu_d(zsave(s, AC_SAVE_ZT2 + k)) : 0.f;
            }
        }
        __syncthreads();
        float acc[PPO_TILE];
        // ---- trunk 2 -> trunk 1: dz_t1 = (W_t2^T dz_t2) ELU'(z_t1)
        if (tid < 128) {
            tile_matvec_t(sm + BW_DZT2, 64, Bw + ACB_TW2, 128, 64, tid, acc);
#pragma unroll
            for (int s = 0; s < PPO_TILE; ++s)
                sm[BW_DZT1 + s * 128 + tid] = r0 + s < B ? acc[s] * elu_d(zsave(s, AC_SAVE_ZT1 + tid)) : 0.f;
        }
        __syncthreads();
        // ---- trunk 1 -> embedding
        tile_matvec_t(sm + BW_DZT1, 128, Bw + ACB_TW1, 256, 128, tid, acc);
#pragma unroll
        for (int s = 0; s < PPO_TILE; ++s) sm[BW_DEMB + s * 256 + tid] = acc[s];
        __syncthreads();
        // ---- ego encoder: dz_e2 = d_emb[0:64] ELU'(z_e2); dz_e1 = (W_e2^T dz_e2) ELU'(z_e1)
        if (tid < 64) {
#pragma unroll
            for (int s = 0; s < PPO_TILE; ++s)
                sm[BW_DZE2 + s * 64 + tid] = r0 + s < B ? sm[BW_DEMB + s * 256 + tid] * elu_d(zsave(s, AC_SAVE_ZE2 + tid)) : 0.f;
        }
        __syncthreads();
        if (tid < 64) {
            tile_matvec_t(sm + BW_DZE2, 64, Bw + ACB_EW2, 64, 64, tid, acc);
#pragma unroll
            for (int s = 0; s < PPO_TILE; ++s)
                sm[BW_DZE1 + s * 64 + tid] = r0 + s < B ? acc[s] * elu_d(zsave(s, AC_SAVE_ZE1 + tid)) : 0.f;
        }
        __syncthreads();
        // ---- dense weight gradients: sums over the tile's rows
        // head W[o][k], b[o]
        for (int e = tid; e < nout * 65; e += 256) {
            const int o = e / 65, k = e - 65 * o;
            float a = 0.f;
            for (int s = 0; s < PPO_TILE; ++s) a += sm[BW_DO + s * 4 + o] * (k < 64 ? sm[BW_T2 + s * 64 + k] : 1.f);
            if (k < 64) g[ACF_HEAD + o * 64 + k] = a;
            else g[ACF_HEAD + nout * 64 + o] = a;
        }
        if (net == 0 && tid < 3) g[ACF_LOGSTD + tid] = 0.f;     // from the loss partials
        // trunk 1: W[i][k] (128 x 256), column k per thread
        tile_outer(sm + BW_DZT1, 128, 128, sm + BW_EMB, 256, tid, g + ACF_TW1, 256);
        // trunk 2: W[j][k] (64 x 128); ego 2: W[j][k] (64 x 64)
        if (tid < 128) tile_outer(sm + BW_DZT2, 64, 64, sm + BW_T1, 128, tid, g + ACF_TW2, 128);
        else if (tid < 192) tile_outer(sm + BW_DZE2, 64, 64, sm + BW_E1, 64, tid - 128, g + ACF_EW2, 64);
        // biases of trunk 1, trunk 2, ego 2
        if (tid < 128) {
            float a = 0.f;
            for (int s = 0; s < PPO_TILE; ++s) a += sm[BW_DZT1 + s * 128 + tid];
            g[ACF_TB1 + tid] = a;
        } else if (tid < 192) {
            float a = 0.f, b = 0.f;
            for (int s = 0; s < PPO_TILE; ++s) {
                a += sm[BW_DZT2 + s * 64 + tid - 128];
                b += sm[BW_DZE2 + s * 64 + tid - 128];
            }
            g[ACF_TB2 + tid - 128] = a;
            g[ACF_EB2 + tid - 128] = b;
        }
        // ego 1: W[j][k] (64 x 11), b[j]
        for (int e = tid; e < 64 * 12; e += 256) {
            const int j = e / 12, k = e - 12 * j;
            float a = 0.f;
            for (int s = 0; s < PPO_TILE; ++s) a += sm[BW_DZE1 + s * 64 + j] * (k < 11 ? sm[BW_XEGO + s * 12 + k] : 1.f);
            if (k < 11) g[ACF_EW1 + j * 11 + k] = a;
            else g[ACF_EB1 + j] = a;
        }
        __syncthreads();   // the dense buffers become the encoders' buffers
        // ---- set encoders through their pooled slots
        encoder_backward<5>(sm, obs, rows, B, r0, save, net, AC_SAVE_AR, SF_FULL_EGO, 64, F, ACF_RW1, ACF_RB1,
                            ACF_RW2, ACF_RB2, Bw + ACB_RW1, Bw + ACB_RW2, g);
        encoder_backward<7>(sm, obs, rows, B, r0, save, net, AC_SAVE_AV, SF_FULL_EGO + 5 * SF_FULL_ROAD_K, 160, F,
                            ACF_VW1, ACF_VB1, ACF_VW2, ACF_VB2, Bw + ACB_VW1, Bw + ACB_VW2, g);
    }
}

void launch_ppo_backward(const float *obs, const int *rows, int B, const float *save, const float *dout,
                         const float *Pf, const uint16_t *Wb, float *part, hipStream_t s) {
    if (B == 0) return;
    sf_launch(k_ppo_backward, dim3((B + PPO_TILE - 1) / PPO_TILE), dim3(256), sizeof(float) * BW_FLOATS, s, obs,
              rows, B, save, dout, Pf, Wb, part);
}

int ppo_tiles(int B) { return (B + PPO_TILE - 1) / PPO_TILE; }

// ------------------------------------------------------------ reduce, Adam
// two-level sum of the tile partials, each level in a fixed order: group
// g of the tiles into gpart[g] (grid y = group), then the groups in order
// into grad plus the log sigma terms of the loss (stats[4..6]) less the
// entropy coefficient
#define RED_GROUPS 16
__global__ void k_ppo_reduce_groups(const float *__restrict__ part, int tiles, float *__restrict__ gpart) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SF_AC_PARAMS) return;
    const int per = (tiles + RED_GROUPS - 1) / RED_GROUPS;
    const int t0 = blockIdx.y * per, t1 = min(tiles, t0 + per);
    float g = 0.f;
    for (int t = t0; t < t1; ++t) g += part[(size_t)t * SF_AC_PARAMS + p];
    gpart[(size_t)blockIdx.y * SF_AC_PARAMS + p] = g;
}

__global__ void k_ppo_reduce(const float *__restrict__ gpart, const double *__restrict__ stats, float c_e,
                             float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SF_AC_PARAMS) return;
    float g = 0.f;
    for (int q = 0; q < RED_GROUPS; ++q) g += gpart[(size_t)q * SF_AC_PARAMS + p];
    if (p >= ACF_LOGSTD && p < ACF_LOGSTD + 3) g += (float)stats[4 + p - ACF_LOGSTD] - c_e;
    grad[p] = g;
}

int ppo_reduce_groups() { return RED_GROUPS; }

#define SQ_BLOCK 256
__global__ __launch_bounds__(SQ_BLOCK) void k_ppo_sqnorm(const float *__restrict__ grad, double *__restrict__ part) {
    __shared__ double s[SQ_BLOCK];
    double a = 0.0;
    for (int p = blockIdx.x * SQ_BLOCK + threadIdx.x; p < SF_AC_PARAMS; p += gridDim.x * SQ_BLOCK) {
        const double v = grad[p];
        a += v * v;
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = SQ_BLOCK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// gradient scaled to at most max_norm (global norm), then Adam on the
// float32 masters; norm_out[0] receives the norm before clipping
__global__ void k_ppo_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ grad, const double *__restrict__ sq, int nsq, float max_norm,
                           float lr, float b1, float b2, float eps, float c1, float c2, float *__restrict__ norm_out) {
    double q = 0.0;
    for (int b = 0; b < nsq; ++b) q += sq[b];
    const float norm = (float)sqrt(q);
    const float scale = fminf(1.f, max_norm / (norm + 1e-6f));
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) norm_out[0] = norm;
    if (p >= SF_AC_PARAMS) return;
    const float g = grad[p] * scale;
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    P[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

#define SQ_BLOCKS 64
void launch_ppo_reduce(const float *part, int tiles, float *gpart, const double *stats, float c_e, float *grad,
                       double *sq, hipStream_t s) {
    k_ppo_reduce_groups<<<dim3((SF_AC_PARAMS + 255) / 256, RED_GROUPS), 256, 0, s>>>(part, tiles, gpart);
    k_ppo_reduce<<<(SF_AC_PARAMS + 255) / 256, 256, 0, s>>>(gpart, stats, c_e, grad);
    k_ppo_sqnorm<<<SQ_BLOCKS, SQ_BLOCK, 0, s>>>(grad, sq);
}

void launch_ppo_adam(float *P, float *m, float *v, const float *grad, const double *sq, float max_norm, float lr,
                     float b1, float b2, float eps, float c1, float c2, float *norm_out, hipStream_t s) {
    k_ppo_adam<<<(SF_AC_PARAMS + 255) / 256, 256, 0, s>>>(P, m, v, grad, sq, SQ_BLOCKS, max_norm, lr, b1, b2, eps, c1,
                                                         c2, norm_out);
}

// every entry of rows[0, n) inside [0, limit): flag[0] stays 0, else 1
__global__ void k_ppo_check_rows(const int *__restrict__ rows, long long n, int limit, int *__restrict__ flag) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (rows[i] < 0 || rows[i] >= limit)) atomicOr(flag, 1);
}

void launch_ppo_check_rows(const int *rows, long long n, int limit, int *flag, hipStream_t s) {
    if (n > 0) k_ppo_check_rows<<<(int)((n + 255) / 256), 256, 0, s>>>(rows, n, limit, flag);
}
