// Learned tire surrogate: training kernels (inference runs inside the step
// kernel, k_step.hip).
//
// Network 16 -> 128 -> 128 -> 128 -> 3, ReLU hidden, linear outputs
// (F_x, F_y, M_z / trail) / (mu F_z).  bf16 operands on the matrix cores
// (v_mfma_f32_16x16x32_bf16), fp32 accumulation, fp32 master weights and
// Adam moments.  One workgroup (4 waves) runs forward and backward for a
// tile of 64 samples with every activation in LDS (plus m-contiguous
// transposed copies for the weight-gradient products) and writes the tile's
// fp32 gradient; a second kernel sums the tiles in a fixed order (so the
// result is deterministic) and takes the Adam step.
#include "sf_dev.h"

#define TILE 64
#define LD0 40    // x0 row stride: 16 inputs, 16 zeros (k padded to 32), 8 pad
#define LDH 136   // hidden row stride
#define LDT 72    // transposed (m-contiguous) row stride

// ------------------------------------------------------------ collection
__global__ void k_sur_flags(const float *log, int n, int *flag) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) flag[k] = log[(size_t)k * SF_SUR_SAMPLE + SF_SUR_SAMPLE - 1] != 0.f;
}
__global__ void k_sur_compact(const float *log, int n, const int *pos, float *out, int max_out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (log[(size_t)k * SF_SUR_SAMPLE + SF_SUR_SAMPLE - 1] == 0.f) return;
    const int p = pos[k];
    if (p >= max_out) return;
    for (int c = 0; c < SF_SUR_SAMPLE; ++c) out[(size_t)p * SF_SUR_SAMPLE + c] = log[(size_t)k * SF_SUR_SAMPLE + c];
}

void launch_sur_collect(const float *log, int n, int *flag, int *pos, int *scan_tmp, float *out, int max_out,
                        hipStream_t s) {
    if (n == 0) return;
    k_sur_flags<<<(n + 255) / 256, 256, 0, s>>>(log, n, flag);
    launch_scan(flag, pos, n, scan_tmp, s);
    k_sur_compact<<<(n + 255) / 256, 256, 0, s>>>(log, n, pos, out, max_out);
}

// per-input [min, max] over M samples (the domain the surrogate was trained on)
__global__ __launch_bounds__(256) void k_sur_env_part(const float *x, int M, float *part) {
    __shared__ float slo[256], shi[256];
    const int f = blockIdx.y;
    float lo = INFINITY, hi = -INFINITY;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < M; k += gridDim.x * 256) {
        const float v = x[(size_t)k * SF_SUR_SAMPLE + f];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            slo[threadIdx.x] = fminf(slo[threadIdx.x], slo[threadIdx.x + o]);
            shi[threadIdx.x] = fmaxf(shi[threadIdx.x], shi[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * (f * gridDim.x + blockIdx.x)] = slo[0];
        part[2 * (f * gridDim.x + blockIdx.x) + 1] = shi[0];
    }
}
__global__ void k_sur_env_final(const float *part, int nb, float *lo, float *hi) {
    const int f = threadIdx.x;
    if (f >= SF_SUR_IN) return;
    float a = INFINITY, b = -INFINITY;
    for (int k = 0; k < nb; ++k) {
        a = fminf(a, part[2 * (f * nb + k)]);
        b = fmaxf(b, part[2 * (f * nb + k) + 1]);
    }
    lo[f] = a;
    hi[f] = b;
}

void launch_sur_envelope(const float *x, int M, float *part, float *lo, float *hi, hipStream_t s) {
    const int nb = 64;
    k_sur_env_part<<<dim3(nb, SF_SUR_IN), 256, 0, s>>>(x, M, part);
    k_sur_env_final<<<1, 64, 0, s>>>(part, nb, lo, hi);
}

// ------------------------------------------------------------------ init
// He-normal weights (Box-Muller on SplitMix64 counters), zero biases
__global__ void k_sur_init(float *P, unsigned long long seed) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SF_SUR_PARAMS) return;
    int fan = 0;
    if (p < SF_SUR_B1) fan = SF_SUR_IN;
    else if ((p >= SF_SUR_W2 && p < SF_SUR_B2) || (p >= SF_SUR_W3 && p < SF_SUR_B3) || (p >= SF_SUR_W4 && p < SF_SUR_B4))
        fan = SF_SUR_HID;
    if (!fan) { P[p] = 0.f; return; }
    const unsigned long long a = splitmix64(seed ^ (2ull * p)), b = splitmix64(seed ^ (2ull * p + 1));
    const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    P[p] = (float)(z * sqrt(2.0 / fan));
}

void launch_sur_init(float *P, unsigned long long seed, hipStream_t s) {
    k_sur_init<<<(SF_SUR_PARAMS + 255) / 256, 256, 0, s>>>(P, seed);
}

// bf16 copy of parameter p (row-major, and transposed for W2 / W3)
__device__ __forceinline__ void sur_pack_one(const float w, int p, uint16_t *Wb) {
    const uint16_t b = f2bf(w);
    if (p < SF_SUR_B1) {
        Wb[SF_SURB_W1 + p] = b;
    } else if (p >= SF_SUR_W2 && p < SF_SUR_B2) {
        const int q = p - SF_SUR_W2, n = q / SF_SUR_HID, k = q % SF_SUR_HID;
        Wb[SF_SURB_W2 + q] = b;
        Wb[SF_SURB_W2T + k * SF_SUR_HID + n] = b;
    } else if (p >= SF_SUR_W3 && p < SF_SUR_B3) {
        const int q = p - SF_SUR_W3, n = q / SF_SUR_HID, k = q % SF_SUR_HID;
        Wb[SF_SURB_W3 + q] = b;
        Wb[SF_SURB_W3T + k * SF_SUR_HID + n] = b;
    } else if (p >= SF_SUR_W4 && p < SF_SUR_B4) {
        Wb[SF_SURB_W4 + (p - SF_SUR_W4)] = b;
    }
}

__global__ void k_sur_pack(const float *P, uint16_t *Wb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < SF_SUR_PARAMS) sur_pack_one(P[p], p, Wb);
}

void launch_sur_pack(const float *P, uint16_t *Wb, hipStream_t s) {
    k_sur_pack<<<(SF_SUR_PARAMS + 255) / 256, 256, 0, s>>>(P, Wb);
}

// ------------------------------------------------------ forward / backward
struct SurLDS {
    uint16_t x0[TILE * LD0];
    uint16_t a1[TILE * LDH], a2[TILE * LDH], a3[TILE * LDH];
    uint16_t x0t[32 * LDT], a1t[SF_SUR_HID * LDT], a2t[SF_SUR_HID * LDT];
    uint16_t dz[TILE * LDH], dzt[SF_SUR_HID * LDT];
    float y[TILE][4], t[TILE][4];
    float loss[4];
};

// hidden layer out = relu(in W^T + b) for the tile's 64 rows; wave w owns
// output columns [32 w, 32 w + 32); bf16 row-major and, when outt is not
// null, transposed copies
template <int KS, class FA, class FB>
__device__ __forceinline__ void sur_hidden(FA fa, FB fb, const float *bias, uint16_t *out, uint16_t *outt) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[4][2];
    zero_acc(acc);
    mfma_nt<4, 2, KS>(acc, fa, [&](int c, int k0) { return fb(wv * 32 + c, k0); });
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = wv * 32 + c * 16 + r16;
        const float b = bias[col];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = r * 16 + kq * 4 + j;
                const uint16_t v = f2bf(fmaxf(acc[r][c][j] + b, 0.f));
                out[row * LDH + col] = v;
                if (outt) outt[col * LDT + row] = v;
            }
    }
}

// dW[n][k] (128 x K) = sum_m dZ[m][n] A[m][k] from dZ^T (m-contiguous) and
// A^T given by fb; wave w owns rows n in [32 w, 32 w + 32)
template <int CT, class FB>
__device__ __forceinline__ void sur_dweight(const uint16_t *dzt, FB fb, float *g, int K) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[2][CT];
    zero_acc(acc);
    mfma_nt<2, CT, TILE / 32>(acc, [&](int r, int k0) { return ld8(dzt + (wv * 32 + r) * LDT + k0); }, fb);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = wv * 32 + r * 16 + kq * 4 + j, k = c * 16 + r16;
                if (k < K) g[n * K + k] = acc[r][c][j];
            }
}

// dA[m][k] = sum_n dZ[m][n] W[n][k] (W^T row-major given), into registers;
// wave w owns columns k in [32 w, 32 w + 32)
__device__ __forceinline__ void sur_dact(const uint16_t *dz, const uint16_t *WT, f32x4 (&acc)[4][2]) {
    const int wv = threadIdx.x >> 6;
    zero_acc(acc);
    mfma_nt<4, 2, SF_SUR_HID / 32>(acc, [&](int r, int k0) { return ld8(dz + r * LDH + k0); },
                                   [&](int c, int k0) { return ld8(WT + (wv * 32 + c) * SF_SUR_HID + k0); });
}

// dZ = dA where the layer's activation is positive (ReLU'), bf16, both layouts
__device__ __forceinline__ void sur_store_dz(const f32x4 (&acc)[4][2], const uint16_t *a, uint16_t *dz,
                                             uint16_t *dzt) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = wv * 32 + c * 16 + r16;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = r * 16 + kq * 4 + j;
                const uint16_t b = f2bf(bf2f(a[row * LDH + col]) > 0.f ? acc[r][c][j] : 0.f);
                dz[row * LDH + col] = b;
                dzt[col * LDT + row] = b;
            }
    }
}

__device__ __forceinline__ void sur_dbias(const uint16_t *dzt, float *g) {
    const int n = threadIdx.x;
    if (n < SF_SUR_HID) {
        float s = 0.f;
        for (int m = 0; m < TILE; ++m) s += bf2f(dzt[n * LDT + m]);
        g[n] = s;
    }
}

// MODE 0: training tile (rows drawn with replacement by a counter-based
// hash of the seed, or consecutive rows when the seed is 0; writes the
// tile's gradient of the batch-mean squared error and its share of the
// loss); MODE 1: evaluation (consecutive rows, predictions)
template <int MODE>
__global__ __launch_bounds__(256) void k_sur_tile(const float *__restrict__ data, int M,
                                                  const float *__restrict__ P, const uint16_t *__restrict__ Wb,
                                                  unsigned long long seed, int batch, float *__restrict__ grad,
                                                  float *__restrict__ loss, float *__restrict__ pred) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    SurLDS &L = *reinterpret_cast<SurLDS *>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int tile = blockIdx.x;
    for (int e = tid; e < TILE * 32; e += 256) {
        const int r = e >> 5, f = e & 31;
        long long idx;
        if (MODE == 0 && seed != 0)
            idx = (long long)(splitmix64(seed ^ ((unsigned long long)(tile * TILE + r) << 22)) % (unsigned long long)M);
        else
            idx = (long long)tile * TILE + r;
        const bool ok = idx < M;
        const float v = (f < SF_SUR_IN && ok) ? data[idx * SF_SUR_SAMPLE + f] : 0.f;
        const uint16_t b = f2bf(v);
        L.x0[r * LD0 + f] = b;
        L.x0t[f * LDT + r] = b;
        if (f < 3) L.t[r][f] = ok ? data[idx * SF_SUR_SAMPLE + SF_SUR_IN + f] : 0.f;
        if (f == 3) L.t[r][3] = ok ? 1.f : 0.f;  // padding rows carry no loss
    }
    __syncthreads();
    // ---- forward
    sur_hidden<1>([&](int r, int k0) { return ld8(L.x0 + r * LD0 + k0); },
                  [&](int n, int k0) { return k0 < SF_SUR_IN ? ld8(Wb + SF_SURB_W1 + n * SF_SUR_IN + k0) : zero8(); },
                  P + SF_SUR_B1, L.a1, L.a1t);
    __syncthreads();
    sur_hidden<4>([&](int r, int k0) { return ld8(L.a1 + r * LDH + k0); },
                  [&](int n, int k0) { return ld8(Wb + SF_SURB_W2 + n * SF_SUR_HID + k0); }, P + SF_SUR_B2, L.a2,
                  L.a2t);
    __syncthreads();
    sur_hidden<4>([&](int r, int k0) { return ld8(L.a2 + r * LDH + k0); },
                  [&](int n, int k0) { return ld8(Wb + SF_SURB_W3 + n * SF_SUR_HID + k0); }, P + SF_SUR_B3, L.a3,
                  nullptr);
    __syncthreads();
    // output layer: fp32 dot products over bf16 operands
    if (tid < TILE * 3) {
        const int r = tid / 3, o = tid % 3;
        float acc = P[SF_SUR_B4 + o];
        for (int k = 0; k < SF_SUR_HID; ++k) acc += bf2f(L.a3[r * LDH + k]) * bf2f(Wb[SF_SURB_W4 + o * SF_SUR_HID + k]);
        L.y[r][o] = acc;
    }
    __syncthreads();
    if (MODE == 1) {
        if (tid < TILE * 3) {
            const int r = tid / 3, o = tid % 3;
            const long long idx = (long long)tile * TILE + r;
            if (idx < M) pred[idx * 3 + o] = L.y[r][o];
        }
        return;
    }
    // ---- loss and its gradient dY = 2 w (y - t) / (3 batch), kept in L.y;
    // a sample's weight w = 1 / max(|(t_x, t_y)|, 0.05)^2 makes its squared
    // error the squared relative force error
    float* g = grad + (size_t)tile * SF_SUR_PARAMS;
    float d2 = 0.f;
    if (tid < TILE * 3) {
        const int r = tid / 3, o = tid % 3;
        const float den = fmaxf(sqrtf(L.t[r][0] * L.t[r][0] + L.t[r][1] * L.t[r][1]), 0.05f);
        const float w = 1.f / (den * den);
        const float d = L.t[r][3] != 0.f ? L.y[r][o] - L.t[r][o] : 0.f;
        d2 = w * d * d;
        L.y[r][o] = 2.f * w * d / (3.f * (float)batch);
    }
    for (int o = 32; o > 0; o >>= 1) d2 += __shfl_xor(d2, o, 64);
    if (lane == 0) L.loss[wv] = d2;
    __syncthreads();
    if (tid == 0) loss[tile] = (L.loss[0] + L.loss[1] + L.loss[2] + L.loss[3]) / (3.f * (float)batch);
    // output layer gradients (fp32)
    for (int e = tid; e < 3 * SF_SUR_HID; e += 256) {
        const int o = e / SF_SUR_HID, k = e % SF_SUR_HID;
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += L.y[r][o] * bf2f(L.a3[r * LDH + k]);
        g[SF_SUR_W4 + e] = s;
    }
    if (tid < 3) {
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += L.y[r][tid];
        g[SF_SUR_B4 + tid] = s;
    }
    // dZ3 = (dY W4) relu'(a3)
    for (int e = tid; e < TILE * SF_SUR_HID; e += 256) {
        const int r = e / SF_SUR_HID, k = e % SF_SUR_HID;
        float v = 0.f;
        if (bf2f(L.a3[r * LDH + k]) > 0.f)
            for (int o = 0; o < 3; ++o) v += L.y[r][o] * bf2f(Wb[SF_SURB_W4 + o * SF_SUR_HID + k]);
        const uint16_t b = f2bf(v);
        L.dz[r * LDH + k] = b;
        L.dzt[k * LDT + r] = b;
    }
    __syncthreads();
    // layer 3
    sur_dweight<8>(L.dzt, [&](int c, int k0) { return ld8(L.a2t + c * LDT + k0); }, g + SF_SUR_W3, SF_SUR_HID);
    sur_dbias(L.dzt, g + SF_SUR_B3);
    f32x4 acc[4][2];
    sur_dact(L.dz, Wb + SF_SURB_W3T, acc);
    __syncthreads();
    sur_store_dz(acc, L.a2, L.dz, L.dzt);
    __syncthreads();
    // layer 2
    sur_dweight<8>(L.dzt, [&](int c, int k0) { return ld8(L.a1t + c * LDT + k0); }, g + SF_SUR_W2, SF_SUR_HID);
    sur_dbias(L.dzt, g + SF_SUR_B2);
    sur_dact(L.dz, Wb + SF_SURB_W2T, acc);
    __syncthreads();
    sur_store_dz(acc, L.a1, L.dz, L.dzt);
    __syncthreads();
    // layer 1 (inputs padded from 16 to 32 columns; only 16 written)
    sur_dweight<2>(L.dzt, [&](int c, int k0) { return ld8(L.x0t + c * LDT + k0); }, g + SF_SUR_W1, SF_SUR_IN);
    sur_dbias(L.dzt, g + SF_SUR_B1);
}

static bool g_sur_attr = false;
static void sur_attr() {
    if (g_sur_attr) return;
    (void)hipFuncSetAttribute((const void *)k_sur_tile<0>, hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(SurLDS));
    (void)hipFuncSetAttribute((const void *)k_sur_tile<1>, hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(SurLDS));
    g_sur_attr = true;
}

void launch_sur_grad(const float *data, int M, const float *P, const uint16_t *Wb, unsigned long long seed,
                     int tiles, float *grad, float *loss, hipStream_t s) {
    sur_attr();
    k_sur_tile<0><<<tiles, 256, sizeof(SurLDS), s>>>(data, M, P, Wb, seed, tiles * TILE, grad, loss, nullptr);
}

void launch_sur_grad_seq(const float *data, int M, const float *P, const uint16_t *Wb, float *grad, float *loss,
                         hipStream_t s) {
    sur_attr();
    const int tiles = (M + TILE - 1) / TILE;
    k_sur_tile<0><<<tiles, 256, sizeof(SurLDS), s>>>(data, M, P, Wb, 0, M, grad, loss, nullptr);
}

__global__ void k_sur_reduce(const float *grad, int tiles, float *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SF_SUR_PARAMS) return;
    float g = 0.f;
    for (int t = 0; t < tiles; ++t) g += grad[(size_t)t * SF_SUR_PARAMS + p];
    out[p] = g;
}

void launch_sur_reduce(const float *grad, int tiles, float *out, hipStream_t s) {
    k_sur_reduce<<<(SF_SUR_PARAMS + 255) / 256, 256, 0, s>>>(grad, tiles, out);
}

void launch_sur_eval(const float *data, int M, const float *P, const uint16_t *Wb, float *pred, hipStream_t s) {
    if (M == 0) return;
    sur_attr();
    k_sur_tile<1><<<(M + TILE - 1) / TILE, 256, sizeof(SurLDS), s>>>(data, M, P, Wb, 0, 0, nullptr, nullptr, pred);
}

// ------------------------------------------------------------------ Adam
// sum of the tiles' gradients (fixed order), Adam (Kingma and Ba 2015)
// with bias corrections c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t), and the
// refreshed bf16 copies
__global__ void k_sur_adam(float *P, float *m, float *v, const float *grad, int tiles, float lr, float b1,
                           float b2, float eps, float c1, float c2, uint16_t *Wb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SF_SUR_PARAMS) return;
    float g = 0.f;
    for (int t = 0; t < tiles; ++t) g += grad[(size_t)t * SF_SUR_PARAMS + p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float w = P[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    P[p] = w;
    sur_pack_one(w, p, Wb);
}

void launch_sur_adam(float *P, float *m, float *v, const float *grad, int tiles, float lr, float b1, float b2,
                     float eps, float c1, float c2, uint16_t *Wb, hipStream_t s) {
    k_sur_adam<<<(SF_SUR_PARAMS + 255) / 256, 256, 0, s>>>(P, m, v, grad, tiles, lr, b1, b2, eps, c1, c2, Wb);
}

// relative force error per sample: |d(F_x, F_y)| / max(|(F_x, F_y)|, 0.05)
// in units of mu F_z (the plain model's force is the reference)
__global__ void k_sur_errors(const float *data, int M, const float *pred, float *err) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const float tx = data[(size_t)k * SF_SUR_SAMPLE + SF_SUR_IN], ty = data[(size_t)k * SF_SUR_SAMPLE + SF_SUR_IN + 1];
    const float dx = pred[3 * (size_t)k] - tx, dy = pred[3 * (size_t)k + 1] - ty;
    err[k] = sqrtf(dx * dx + dy * dy) / fmaxf(sqrtf(tx * tx + ty * ty), 0.05f);
}

void launch_sur_errors(const float *data, int M, const float *pred, float *err, hipStream_t s) {
    if (M > 0) k_sur_errors<<<(M + 255) / 256, 256, 0, s>>>(data, M, pred, err);
}
