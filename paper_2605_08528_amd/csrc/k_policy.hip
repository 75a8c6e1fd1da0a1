// Policy MLP 256 -> 256 -> 256 -> 2 on the agents' observations (the
// on-device policy inference of Algorithm "SceneFactory Pipeline"): bf16
// inputs and weights on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16),
// fp32 accumulation, ELU hidden layers (Sec. "Network Architecture
// Details" uses ELU), tanh outputs scaled to (a_long, steer_max * steer).
//
// One workgroup (4 waves) owns TM agents.  The observation tile is converted
// to bf16 in LDS; each wave computes 64 output columns of a layer for all TM
// rows; hidden activations stay in LDS (ping-pong buffers); the 2-wide head
// is a plain fp32 dot product.
#include "sf_dev.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define PL_IN 256
#define PL_HID 256
#define PL_LD (PL_HID + 8)  // padded LDS row (bf16 elements) against bank conflicts

// one hidden layer: out[TM][256] = act(in[TM][256] W^T + b), bf16 in LDS
template <int TM>
__device__ __forceinline__ void dense_layer(const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                            const uint16_t *__restrict__ W, const float *__restrict__ b) {
    constexpr int RT = TM / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[RT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weight fragments of the next k-step are fetched before the current
    // step's matrix instructions issue (register double buffering)
    bf16x8 bnx[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        bnx[c] = *reinterpret_cast<const bf16x8 *>(W + (size_t)(wv * 64 + c * 16 + r16) * PL_IN + kq * 8);
#pragma unroll
    for (int kk = 0; kk < PL_IN / 32; ++kk) {
        const int k0 = kk * 32 + kq * 8;
        bf16x8 bfr[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bfr[c] = bnx[c];
        if (kk + 1 < PL_IN / 32) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                bnx[c] = *reinterpret_cast<const bf16x8 *>(W + (size_t)(wv * 64 + c * 16 + r16) * PL_IN + k0 + 32);
        }
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const bf16x8 afr = *reinterpret_cast<const bf16x8 *>(in + (r * 16 + r16) * PL_LD + k0);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[c], acc[r][c], 0, 0, 0);
        }
    }
    // lane holds D[4 * (lane / 16) + j][lane % 16] of each 16 x 16 tile
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int col = wv * 64 + c * 16 + r16;
        const float bias = b[col];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = r * 16 + kq * 4 + j;
                out[row * PL_LD + col] = f2bf(elu_fast(acc[r][c][j] + bias));
            }
    }
}

// head: 2 outputs per row, fp32 dot products over bf16 operands (W3 in
// LDS), each split over G = 256 / (2 TM) lanes and summed in a fixed
// butterfly order
template <int TM>
__device__ __forceinline__ void policy_head(const uint16_t *__restrict__ s_h, const uint16_t *__restrict__ s_w3,
                                            const float *__restrict__ b3, float steer_max, int r0, int N,
                                            float *__restrict__ act) {
    constexpr int G = 256 / (2 * TM), KP = PL_HID / G;
    const int t = threadIdx.x, out = t / G, part = t % G;
    const int row = out >> 1, o = out & 1;
    const uint16_t *h = s_h + row * PL_LD + part * KP;
    const uint16_t *w = s_w3 + o * PL_HID + part * KP;
    float acc = 0.f;
#pragma unroll 8
    for (int k = 0; k < KP; ++k) acc += bf2f(h[k]) * bf2f(w[k]);
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) acc += lane_xor_f(acc, m);
    if (part == 0 && r0 + row < N) {
        const float z = tanhf(acc + b3[o]);
        act[2 * (size_t)(r0 + row) + o] = o == 0 ? z : steer_max * z;
    }
}

template <int TM>
__global__ __launch_bounds__(256) void k_policy(const float *__restrict__ obs, int N,
                                                const uint16_t *__restrict__ W1, const float *__restrict__ b1,
                                                const uint16_t *__restrict__ W2, const float *__restrict__ b2,
                                                const uint16_t *__restrict__ W3, const float *__restrict__ b3,
                                                float steer_max, float *__restrict__ act) {
    __shared__ __attribute__((aligned(16))) uint16_t s_a[TM * PL_LD];
    __shared__ __attribute__((aligned(16))) uint16_t s_b[TM * PL_LD];
    __shared__ uint16_t s_w3[2 * PL_HID];
    const int r0 = blockIdx.x * TM;
    for (int e = threadIdx.x; e < 2 * PL_HID; e += 256) s_w3[e] = W3[e];
    // observation tile -> bf16 (coalesced float4 loads)
    for (int e = threadIdx.x; e < TM * (PL_IN / 4); e += 256) {
        const int row = e / (PL_IN / 4), c4 = e % (PL_IN / 4);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r0 + row < N) v = reinterpret_cast<const float4 *>(obs + (size_t)(r0 + row) * PL_IN)[c4];
        uint16_t *d = s_a + row * PL_LD + 4 * c4;
        d[0] = f2bf(v.x); d[1] = f2bf(v.y); d[2] = f2bf(v.z); d[3] = f2bf(v.w);
    }
    __syncthreads();
    dense_layer<TM>(s_a, s_b, W1, b1);
    __syncthreads();
    dense_layer<TM>(s_b, s_a, W2, b2);
    __syncthreads();
    // head: 2 outputs per row, fp32 dot products over bf16 operands
    policy_head<TM>(s_a, s_w3, b3, steer_max, r0, N, act);
}

// The same network with each hidden layer's weights staged whole in LDS:
// every thread issues its share of the 128 KB copy (16 loads of 16 bytes in
// flight at a time) instead of waiting on one weight fragment per k-step,
// and the layer's products then read both operands from LDS.  One
// workgroup per compute unit.
#define PL_WLD (PL_IN + 8)  // padded weight row (bf16)

__device__ __forceinline__ void stage_weights(const uint16_t *__restrict__ W, uint16_t *__restrict__ sw) {
    // 256 rows x 32 chunks of 8 bf16; thread t copies chunks t, t + 256, ...,
    // starting at a 4 KB offset of its own per block, so that the blocks'
    // copies do not all hit the same memory lines at once
    const int rot = (int)(blockIdx.x & 31) * 256;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        uint4 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = (threadIdx.x + 256 * (16 * b + q) + rot) & 8191;
            v[q] = reinterpret_cast<const uint4 *>(W)[c];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = (threadIdx.x + 256 * (16 * b + q) + rot) & 8191;
            *reinterpret_cast<uint4 *>(sw + (c >> 5) * PL_WLD + (c & 31) * 8) = v[q];
        }
    }
}

template <int TM>
__device__ __forceinline__ void dense_layer_lds(const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                                const uint16_t *__restrict__ sw, const float *__restrict__ b) {
    constexpr int RT = TM / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    f32x4 acc[RT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < PL_IN / 32; ++kk) {
        const int k0 = kk * 32 + kq * 8;
        bf16x8 bfr[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            bfr[c] = *reinterpret_cast<const bf16x8 *>(sw + (wv * 64 + c * 16 + r16) * PL_WLD + k0);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const bf16x8 afr = *reinterpret_cast<const bf16x8 *>(in + (r * 16 + r16) * PL_LD + k0);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[c], acc[r][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int col = wv * 64 + c * 16 + r16;
        const float bias = b[col];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[(r * 16 + kq * 4 + j) * PL_LD + col] = f2bf(elu_fast(acc[r][c][j] + bias));
    }
}

template <int TM>
__global__ __launch_bounds__(256) void k_policy_lds(const float *__restrict__ obs, int N,
                                                    const uint16_t *__restrict__ W1, const float *__restrict__ b1,
                                                    const uint16_t *__restrict__ W2, const float *__restrict__ b2,
                                                    const uint16_t *__restrict__ W3, const float *__restrict__ b3,
                                                    float steer_max, float *__restrict__ act) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint16_t *s_w = reinterpret_cast<uint16_t *>(smem);      // [256][PL_WLD]
    uint16_t *s_a = s_w + PL_HID * PL_WLD;                   // [TM][PL_LD]
    uint16_t *s_b = s_a + TM * PL_LD;                        // [TM][PL_LD]
    __shared__ uint16_t s_w3[2 * PL_HID];
    const int r0 = blockIdx.x * TM;
    for (int e = threadIdx.x; e < 2 * PL_HID; e += 256) s_w3[e] = W3[e];
    stage_weights(W1, s_w);
    for (int e = threadIdx.x; e < TM * (PL_IN / 4); e += 256) {
        const int row = e / (PL_IN / 4), c4 = e % (PL_IN / 4);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r0 + row < N) v = reinterpret_cast<const float4 *>(obs + (size_t)(r0 + row) * PL_IN)[c4];
        uint16_t *d = s_a + row * PL_LD + 4 * c4;
        d[0] = f2bf(v.x); d[1] = f2bf(v.y); d[2] = f2bf(v.z); d[3] = f2bf(v.w);
    }
    __syncthreads();
    dense_layer_lds<TM>(s_a, s_b, s_w, b1);
    __syncthreads();
    stage_weights(W2, s_w);
    __syncthreads();
    dense_layer_lds<TM>(s_b, s_a, s_w, b2);
    __syncthreads();
    policy_head<TM>(s_a, s_w3, b3, steer_max, r0, N, act);
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, int n) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = f2bf(src[k]);
}

void launch_to_bf16(const float *src, uint16_t *dst, int n, hipStream_t s) {
    if (n > 0) k_to_bf16<<<(n + 255) / 256, 256, 0, s>>>(src, dst, n);
}

template <int TM>
static size_t policy_lds_bytes() {
    return sizeof(uint16_t) * ((size_t)PL_HID * PL_WLD + 2 * (size_t)TM * PL_LD);
}

static_assert(sizeof(uint16_t) * (PL_HID * PL_WLD + 2 * 16 * PL_LD + 2 * PL_HID) <= 160 * 1024,
              "16-row tile exceeds LDS");

static bool g_policy_attr = false;

// tm 16: weights staged in LDS (the copy and two 16-row tiles take
// 149 KB); 32 and 64: weight fragments from L2
void launch_policy(const float *obs, int N, const uint16_t *W1, const float *b1, const uint16_t *W2,
                   const float *b2, const uint16_t *W3, const float *b3, float steer_max, float *act,
                   int tm, hipStream_t s) {
    if (N == 0) return;
    if (!g_policy_attr) {
        (void)hipFuncSetAttribute((const void *)k_policy_lds<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)policy_lds_bytes<16>());
        g_policy_attr = true;
    }
    if (tm <= 16)
        sf_launch(k_policy_lds<16>, dim3((N + 15) / 16), dim3(256), policy_lds_bytes<16>(), s, obs, N, W1, b1, W2, b2,
                  W3, b3, steer_max, act);
    else if (tm <= 32)
        sf_launch(k_policy<32>, dim3((N + 31) / 32), dim3(256), 0, s, obs, N, W1, b1, W2, b2, W3, b3, steer_max, act);
    else
        sf_launch(k_policy<64>, dim3((N + 63) / 64), dim3(256), 0, s, obs, N, W1, b1, W2, b2, W3, b3, steer_max, act);
}
