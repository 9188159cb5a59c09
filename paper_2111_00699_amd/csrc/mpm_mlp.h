// MLP device code shared by the surrogate's training kernels and P2G:
// BF16/FP32 MFMA fragments, the network staged in LDS, and the forward pass
// of a 16-sample tile (layers in transposed form Z^T = W A^T, so the
// output fragment of one layer is the B fragment of the next).
#pragma once

#include "mpm_internal.h"
#include "mpm_surrogate.h"

namespace mpm {
namespace mlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// tanh(x) = 1 - 2 / (1 + exp(2x)): one exponential and one division, exact
// to ~1e-7 absolute, well inside the BF16 operands it feeds (and -> +-1 for
// large |x| without overflow trouble: exp -> inf gives 1, exp -> 0 gives -1).
__device__ __forceinline__ float act_tanh(float x) { return 1.0f - 2.0f / (1.0f + __expf(2.0f * x)); }

// Round to nearest even (finite inputs; the network's values are bounded).
__device__ __forceinline__ short to_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (short)(r >> 16);
}

// The weights of one layer as the A operand, staged in LDS row-major
// [rows][ld] (FP32; BF16 fragments are rounded at load).  acc += W_tile(mt, kt) * B.
template <bool BF16>
__device__ __forceinline__ f32x4 mma_w(f32x4 acc, const float* W, int ld, int mt, int kt, const float b[4]) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const float* row = W + (16 * mt + i) * ld + 16 * kt + 4 * g;
    if constexpr (BF16) {
        bf16x4 a, bb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = to_bf16(row[j]);
            bb[j] = to_bf16(b[j]);
        }
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(row[r], b[r], acc, 0, 0, 0);
        return acc;
    }
}

// acc += A * B where both operands come from LDS: A[i][k] = a[(16*mt + i) * lda + 16*kt + k]
// and B[k][j] = bmat[(16*kt + k) * ldb + 16*nt + j] (row-major K x N).
template <bool BF16>
__device__ __forceinline__ f32x4 mma_ll(f32x4 acc, const float* a, int lda, int mt, int kt, const float* bm, int ldb,
                                        int nt) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    float av[4], bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        av[j] = a[(16 * mt + i) * lda + 16 * kt + 4 * g + j];
        bv[j] = bm[(16 * kt + 4 * g + j) * ldb + 16 * nt + i];
    }
    if constexpr (BF16) {
        bf16x4 x, y;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            x[j] = to_bf16(av[j]);
            y[j] = to_bf16(bv[j]);
        }
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv[r], acc, 0, 0, 0);
        return acc;
    }
}

// The network staged in LDS for the forward pass (FP32, zero padded):
// W1 [64][16], W2 [64][64], W3 [16][64], biases and the normalisation.
struct NetLds {
    float W1[64 * 16], b1[64], W2[64 * 64], b2[64], W3[16 * 64], b3[16];
    float imu[16], isd[16], omu[16], osd[16];
};

// Transposed weights for backpropagation: W2T [64][64], W3T [64][16].
struct NetLdsT {
    float W2T[64 * 64], W3T[64 * 16];
};

__device__ inline void load_net(NetLds& L, const float* __restrict__ th, const float* __restrict__ norm) {
    for (int t = threadIdx.x; t < 64 * 16; t += blockDim.x) {
        const int o = t >> 4, i = t & 15;
        L.W1[t] = i < SUR_IN ? th[SUR_W1 + o * SUR_IN + i] : 0.0f;
        const int o3 = t >> 6, i3 = t & 63;  // W3 padded to 16 outputs
        L.W3[t] = o3 < SUR_OUT ? th[SUR_W3 + o3 * SUR_H + i3] : 0.0f;
    }
    for (int t = threadIdx.x; t < 64 * 64; t += blockDim.x) L.W2[t] = th[SUR_W2 + t];
    for (int t = threadIdx.x; t < 64; t += blockDim.x) {
        L.b1[t] = th[SUR_B1 + t];
        L.b2[t] = th[SUR_B2 + t];
    }
    for (int t = threadIdx.x; t < 16; t += blockDim.x) {
        L.b3[t] = t < SUR_OUT ? th[SUR_B3 + t] : 0.0f;
        L.imu[t] = t < SUR_IN ? norm[t] : 0.0f;
        L.isd[t] = t < SUR_IN ? norm[SUR_IN + t] : 1.0f;
        L.omu[t] = t < SUR_OUT ? norm[2 * SUR_IN + t] : 0.0f;
        L.osd[t] = t < SUR_OUT ? norm[2 * SUR_IN + SUR_OUT + t] : 1.0f;
    }
}

__device__ inline void load_net_t(NetLdsT& L, const float* __restrict__ th) {
    for (int t = threadIdx.x; t < 64 * 16; t += blockDim.x) {
        const int o3 = t >> 6, i3 = t & 63;
        L.W3T[i3 * 16 + o3] = o3 < SUR_OUT ? th[SUR_W3 + o3 * SUR_H + i3] : 0.0f;
    }
    for (int t = threadIdx.x; t < 64 * 64; t += blockDim.x) L.W2T[(t & 63) * 64 + (t >> 6)] = th[SUR_W2 + t];
}

// Forward pass of one 16-sample tile held by a wave.  xin: the tile's
// normalised inputs in LDS [16 samples][16].  Outputs h1, h2 (tanh
// activations, D layout: per hidden tile mt, lane holds units 16mt+4g+r of
// sample l%16) and y (normalised outputs, D layout over 16 output rows).
template <bool BF16>
__device__ __forceinline__ void forward_tile(const NetLds& L, const float* xin, float h1[4][4], float h2[4][4],
                                             float y[4]) {
    const int lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
    float xb[4];  // B fragment of X^T: features 4g..4g+3 of sample s
#pragma unroll
    for (int j = 0; j < 4; ++j) xb[j] = xin[s * 16 + 4 * g + j];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_w<BF16>(acc, L.W1, 16, mt, 0, xb);
#pragma unroll
        for (int r = 0; r < 4; ++r) h1[mt][r] = act_tanh(acc[r] + L.b1[16 * mt + 4 * g + r]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) acc = mma_w<BF16>(acc, L.W2, 64, mt, kt, h1[kt]);
#pragma unroll
        for (int r = 0; r < 4; ++r) h2[mt][r] = act_tanh(acc[r] + L.b2[16 * mt + 4 * g + r]);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) acc = mma_w<BF16>(acc, L.W3, 64, 0, kt, h2[kt]);
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = acc[r] + L.b3[4 * g + r];
}

// Normalised input row of sample `row` into LDS (zero padded to 16).
__device__ __forceinline__ void stage_input(const NetLds& L, const float* __restrict__ X, int64_t row, bool valid,
                                            float* xin, int s) {
    // 4 lanes per sample: lane group g writes features 4g..4g+3
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int f = 4 * g + j;
        float v = 0.0f;
        if (valid && f < SUR_IN) v = (X[row * SUR_IN + f] - L.imu[f]) / L.isd[f];
        xin[s * 16 + f] = v;
    }
}

// Inference copy of the network for P2G: the weights rounded to BF16 once
// as they are staged, biases and normalisation FP32.  The hidden layers run
// on gfx950's 16x16x32 BF16 MFMA: a K = 32 fragment of lane (i, g) holds the
// eight k' = 8g..8g+7, and k' is a permutation of the 32 hidden units of the
// block chosen so that the B fragment is the D output of the previous layer
// as it lies in the registers (units 4g..4g+3 of two consecutive 16-unit
// tiles); the weight rows are stored in that k' order, so an A fragment is
// one 16-byte LDS read.  Rows are padded to W16_LD so the 16 rows one read
// instruction touches start in different banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4h __attribute__((ext_vector_type(4)));
constexpr int W16_LD = 72;

struct __attribute__((aligned(16))) NetLds16 {
    __bf16 W1[64 * 16];      // [unit][feature], the K = 16 first layer
    __bf16 W2[64 * W16_LD];  // [unit][k'] of the two K = 32 blocks
    __bf16 W3[16 * W16_LD];  // [output][k'] (outputs padded to 16)
    float b1[64], b2[64], b3[16];
    float imu[16], isd[16], omu[16], osd[16];
};

// Position k' of hidden unit u in its K = 32 block: unit 32 kb + 16 h + 4 g + r
// sits at 32 kb + 8 g + 4 h + r.
__device__ __forceinline__ int kperm(int u) {
    const int w = u & 31;
    return (u & 32) + 8 * ((w & 15) >> 2) + 4 * (w >> 4) + (w & 3);
}

__device__ inline void load_net16(NetLds16& L, const float* __restrict__ th, const float* __restrict__ norm) {
    for (int t = threadIdx.x; t < 64 * 16; t += blockDim.x) {
        const int o = t >> 4, i = t & 15;
        L.W1[t] = (__bf16)(i < SUR_IN ? th[SUR_W1 + o * SUR_IN + i] : 0.0f);
        const int o3 = t >> 6, u = t & 63;
        L.W3[o3 * W16_LD + kperm(u)] = (__bf16)(o3 < SUR_OUT ? th[SUR_W3 + o3 * SUR_H + u] : 0.0f);
    }
    for (int t = threadIdx.x; t < 64 * 64; t += blockDim.x)
        L.W2[(t >> 6) * W16_LD + kperm(t & 63)] = (__bf16)th[SUR_W2 + t];
    for (int t = threadIdx.x; t < 64; t += blockDim.x) {
        L.b1[t] = th[SUR_B1 + t];
        L.b2[t] = th[SUR_B2 + t];
    }
    for (int t = threadIdx.x; t < 16; t += blockDim.x) {
        L.b3[t] = t < SUR_OUT ? th[SUR_B3 + t] : 0.0f;
        L.imu[t] = t < SUR_IN ? norm[t] : 0.0f;
        L.isd[t] = t < SUR_IN ? norm[SUR_IN + t] : 1.0f;
        L.omu[t] = t < SUR_OUT ? norm[2 * SUR_IN + t] : 0.0f;
        L.osd[t] = t < SUR_OUT ? norm[2 * SUR_IN + SUR_OUT + t] : 1.0f;
    }
}

// tanh of the four accumulators and their BF16 B-fragment halves
__device__ __forceinline__ void act_pack(f32x4 a0, f32x4 a1, bf16x8& b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        b[r] = (__bf16)act_tanh(a0[r]);
        b[4 + r] = (__bf16)act_tanh(a1[r]);
    }
}

// Forward pass of the wave's 64 samples, one per lane: xn the lane's
// normalised inputs, yn its normalised outputs.  stage: FWD_STAGE floats of
// LDS owned by the wave, 16-byte aligned (the rows move as 16-byte vectors),
// the inputs as BF16 rows [64][16] in the first 512
// and the outputs [64][12] after them.  The four 16-sample tiles run one
// after the other with no barrier between them (the four output tiles of a
// layer are independent MFMA chains).
constexpr int FWD_STAGE = 512 + 64 * SUR_OUT;

__device__ __forceinline__ void forward_wave16(const NetLds16& L, float* stage, const float xn[SUR_IN],
                                               float yn[SUR_OUT]) {
    static_assert(SUR_OUT == 12, "the output rows are three float4");
    const int lane = threadIdx.x & 63, g = lane >> 4, i = lane & 15;
    __bf16* xs = reinterpret_cast<__bf16*>(stage);
    float* ys = stage + 512;
    {
        bf16x8 r0, r1;
#pragma unroll
        for (int j = 0; j < 8; ++j) r0[j] = (__bf16)xn[j];
#pragma unroll
        for (int j = 0; j < 8; ++j) r1[j] = (__bf16)(8 + j < SUR_IN ? xn[8 + j] : 0.0f);
        *reinterpret_cast<bf16x8*>(xs + lane * 16) = r0;
        *reinterpret_cast<bf16x8*>(xs + lane * 16 + 8) = r1;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        // the weights are read again for every tile rather than held in registers
        // across the four (they would take some 80 VGPRs from the caller)
        asm volatile("" ::: "memory");
        // B fragment of the first layer: features 4g..4g+3 of sample 16t + i
        const bf16x4h xb = *reinterpret_cast<const bf16x4h*>(xs + (16 * t + i) * 16 + 4 * g);
        f32x4 h[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4h a = *reinterpret_cast<const bf16x4h*>(L.W1 + (16 * mt + i) * 16 + 4 * g);
            h[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, a),
                                                               __builtin_bit_cast(bf16x4, xb),
                                                               *reinterpret_cast<const f32x4*>(L.b1 + 16 * mt + 4 * g),
                                                               0, 0, 0);
        }
        bf16x8 hb[2];
        act_pack(h[0], h[1], hb[0]);
        act_pack(h[2], h[3], hb[1]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = *reinterpret_cast<const f32x4*>(L.b2 + 16 * mt + 4 * g);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(L.W2 + (16 * mt + i) * W16_LD + 32 * kb + 8 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[kb], acc, 0, 0, 0);
            }
            h[mt] = acc;
        }
        act_pack(h[0], h[1], hb[0]);
        act_pack(h[2], h[3], hb[1]);
        f32x4 acc = *reinterpret_cast<const f32x4*>(L.b3 + 4 * g);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(L.W3 + i * W16_LD + 32 * kb + 8 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[kb], acc, 0, 0, 0);
        }
        // outputs 4g..4g+3 of sample 16t + i (g = 3 holds the padding outputs)
        if (g < 3) *reinterpret_cast<f32x4*>(ys + (16 * t + i) * SUR_OUT + 4 * g) = acc;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int o = 0; o < SUR_OUT; ++o) yn[o] = ys[lane * SUR_OUT + o];
    __builtin_amdgcn_wave_barrier();
}

}  // namespace mlp
}  // namespace mpm
