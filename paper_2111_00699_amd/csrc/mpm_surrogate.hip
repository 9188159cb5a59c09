// Learned constitutive surrogate on gfx950: an MLP 12 -> 64 -> 64 -> 12
// (tanh hidden layers, linear output) that maps the trial elastic singular
// values, the plastic volume and the hardening state of a snow particle to
// the projected singular values and principal Kirchhoff stress.  This file
// holds the network's forward pass, its loss gradient by backpropagation,
// Adam, the normalisation statistics and the generation of training pairs
// from a running simulation with the exact return map.
//
// MI355X design:
//  * Every layer runs on MFMA in transposed form, Z^T = W A^T: the weight
//    tile is the A operand and the activations the B operand.  The 16x16
//    output fragment of v_mfma_f32_16x16x16_bf16 (lane l: rows 4(l/16)+r,
//    column l%16) is then exactly the B fragment the next layer needs, so
//    hidden activations never leave registers in the forward pass.
//  * Precision: BF16 operands with FP32 accumulation (the product path), or
//    FP32 operands on v_mfma_f32_16x16x4_f32 for checking gradients.  The
//    FP32 form splits each K=16 step into four K=4 steps over the K rows
//    {4g + r}, g = 0..3, so it consumes the same register fragments.
//  * Training: a wave takes 16 samples at a time; the weight gradients of
//    its samples accumulate in MFMA accumulators (samples as the K
//    dimension, activations and deltas staged in LDS for the transposes)
//    and reach the global gradient with one atomic add per parameter per
//    wave.
#include "mpm_mlp.h"

namespace mpm {

namespace {

constexpr int SW = 256;  // threads per workgroup (4 waves)
using namespace mlp;

template <bool BF16>
__global__ __launch_bounds__(SW) void k_sur_forward(const float* __restrict__ th, const float* __restrict__ norm,
                                                    const float* __restrict__ X, int64_t count,
                                                    float* __restrict__ Y) {
    __shared__ NetLds L;
    __shared__ float xin[SW / 64][16 * 16];
    load_net(L, th, norm);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
    const int64_t tiles = (count + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * (SW / 64) + w; t < tiles; t += (int64_t)gridDim.x * (SW / 64)) {
        const int64_t row = 16 * t + s;
        const bool valid = row < count;
        stage_input(L, X, row, valid, xin[w], s);
        __builtin_amdgcn_wave_barrier();
        float h1[4][4], h2[4][4], y[4];
        forward_tile<BF16>(L, xin[w], h1, h2, y);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * g + r;
            if (valid && o < SUR_OUT) Y[row * SUR_OUT + o] = y[r] * L.osd[o] + L.omu[o];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Y = network(X) with the BF16 inference copy of the network: the weights
// rounded to BF16 once as they are staged (NetLds16) and the wave-wide
// forward pass P2G runs (forward_wave16, 64 samples a wave), with P2G's
// input normalisation.
__global__ __launch_bounds__(SW) void k_sur_forward16(const float* __restrict__ th, const float* __restrict__ norm,
                                                      const float* __restrict__ X, int64_t count,
                                                      float* __restrict__ Y) {
    __shared__ NetLds16 L;
    __shared__ __attribute__((aligned(16))) float stage[SW / 64][FWD_STAGE];
    load_net16(L, th, norm);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t groups = (count + 63) / 64;
    for (int64_t t = (int64_t)blockIdx.x * (SW / 64) + w; t < groups; t += (int64_t)gridDim.x * (SW / 64)) {
        const int64_t row = 64 * t + lane;
        const bool valid = row < count;
        float xn[SUR_IN], yn[SUR_OUT];
#pragma unroll
        for (int f = 0; f < SUR_IN; ++f) xn[f] = valid ? (X[row * SUR_IN + f] - L.imu[f]) / L.isd[f] : 0.0f;
        forward_wave16(L, stage[w], xn, yn);
        if (valid) {
#pragma unroll
            for (int o = 0; o < SUR_OUT; ++o) Y[row * SUR_OUT + o] = yn[o] * L.osd[o] + L.omu[o];
        }
    }
}

// Loss 1/2 |y~ - t~|^2 averaged over `count` samples (normalised space) and
// its gradient, accumulated into grad[SUR_PARAMS] and *loss (both zeroed by
// the caller).
template <bool BF16>
__global__ __launch_bounds__(SW) void k_sur_grad(const float* __restrict__ th, const float* __restrict__ norm,
                                                 const float* __restrict__ X, const float* __restrict__ T,
                                                 int64_t count, const int* __restrict__ idx, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
    __shared__ NetLds L;
    __shared__ NetLdsT LT;
    // per wave: inputs [16][16], a1 [16][64], a2 [16][64] (sample-major), deltas d3^T [16][16],
    // d2^T [64][16], d1^T [64][16] (unit-major)
    __shared__ float st_x[SW / 64][16 * 16], st_a1[SW / 64][16 * 64], st_a2[SW / 64][16 * 64];
    __shared__ float st_d3[SW / 64][16 * 16], st_d2[SW / 64][64 * 16], st_d1[SW / 64][64 * 16];
    load_net(L, th, norm);
    load_net_t(LT, th);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
    const float inv_n = 1.0f / (float)count;
    // gradient accumulators (D layout): gW1 4 tiles [64x16], gW2 16 tiles, gW3 4 tiles [16x64]
    f32x4 gW1[4], gW2[4][4], gW3[4];
    float gb1[4][4], gb2[4][4], gb3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        gW3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        gb3[a] = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            gb1[a][b] = gb2[a][b] = 0.0f;
        }
    }
    float lsum = 0.0f;
    const int64_t tiles = (count + 15) / 16;
    float* xs = st_x[w];
    float* a1 = st_a1[w];
    float* a2 = st_a2[w];
    float* d3 = st_d3[w];
    float* d2 = st_d2[w];
    float* d1 = st_d1[w];
    for (int64_t t = (int64_t)blockIdx.x * (SW / 64) + w; t < tiles; t += (int64_t)gridDim.x * (SW / 64)) {
        const int64_t pos = 16 * t + s;
        const bool valid = pos < count;
        const int64_t row = valid ? (idx ? (int64_t)idx[pos] : pos) : 0;
        stage_input(L, X, row, valid, xs, s);
        __builtin_amdgcn_wave_barrier();
        float h1[4][4], h2[4][4], y[4];
        forward_tile<BF16>(L, xs, h1, h2, y);
        // output delta (normalised targets), D layout rows 4g+r of sample s
        float dy[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * g + r;
            float e = 0.0f;
            if (valid && o < SUR_OUT) {
                e = y[r] - (T[row * SUR_OUT + o] - L.omu[o]) / L.osd[o];
                lsum += 0.5f * e * e;
            }
            dy[r] = e * inv_n;
            d3[o * 16 + s] = dy[r];  // [out][sample]: the gW3 A operand
        }
        // activations staged [sample][unit] for the weight-gradient B operands
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a1[s * 64 + 16 * mt + 4 * g + r] = h1[mt][r];
                a2[s * 64 + 16 * mt + 4 * g + r] = h2[mt][r];
            }
        // delta2^T = (W3^T dy^T) * (1 - a2^2): A = W3T tile (hidden x out), B = dy^T fragment
        float e2[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma_w<BF16>(acc, LT.W3T, 16, mt, 0, dy);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                e2[mt][r] = acc[r] * (1.0f - h2[mt][r] * h2[mt][r]);
                d2[(16 * mt + 4 * g + r) * 16 + s] = e2[mt][r];  // [unit][sample]
            }
        }
        // delta1^T = (W2^T delta2^T) * (1 - a1^2)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) acc = mma_w<BF16>(acc, LT.W2T, 64, mt, kt, e2[kt]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float e1 = acc[r] * (1.0f - h1[mt][r] * h1[mt][r]);
                d1[(16 * mt + 4 * g + r) * 16 + s] = e1;
                gb1[mt][r] += e1;
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) gb2[mt][r] += e2[mt][r];
#pragma unroll
        for (int r = 0; r < 4; ++r) gb3[r] += dy[r];
        __builtin_amdgcn_wave_barrier();
        // weight gradients, samples as K: gW3 (16 x 64) += d3^T (16 x 16s) * a2 (16s x 64)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gW3[nt] = mma_ll<BF16>(gW3[nt], d3, 16, 0, 0, a2, 64, nt);
        // gW2 (64 x 64) += d2^T (64 x 16s) * a1 (16s x 64)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mma_ll<BF16>(gW2[mt][nt], d2, 16, mt, 0, a1, 64, nt);
        // gW1 (64 x 16) += d1^T (64 x 16s) * x (16s x 16)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) gW1[mt] = mma_ll<BF16>(gW1[mt], d1, 16, mt, 0, xs, 16, 0);
        __builtin_amdgcn_wave_barrier();
    }
    // one atomic per parameter per wave (D layout: lane holds rows 4g+r, column s)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * mt + 4 * g + r;
            if (s < SUR_IN) atomicAdd(&grad[SUR_W1 + o * SUR_IN + s], gW1[mt][r]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) atomicAdd(&grad[SUR_W2 + o * SUR_H + 16 * nt + s], gW2[mt][nt][r]);
        }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * g + r;
            if (o < SUR_OUT) atomicAdd(&grad[SUR_W3 + o * SUR_H + 16 * nt + s], gW3[nt][r]);
        }
    // bias gradients: sums over the wave's samples (lanes with equal g hold the same units)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v1 = gb1[mt][r], v2 = gb2[mt][r];
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                v1 += __shfl_xor(v1, d, 64);
                v2 += __shfl_xor(v2, d, 64);
            }
            if (s == 0) {
                atomicAdd(&grad[SUR_B1 + 16 * mt + 4 * g + r], v1);
                atomicAdd(&grad[SUR_B2 + 16 * mt + 4 * g + r], v2);
            }
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v3 = gb3[r];
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) v3 += __shfl_xor(v3, d, 64);
        if (s == 0 && 4 * g + r < SUR_OUT) atomicAdd(&grad[SUR_B3 + 4 * g + r], v3);
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) lsum += __shfl_xor(lsum, d, 64);
    if (lane == 0) atomicAdd(loss, lsum * inv_n);
}

// Adam (bias-corrected moments); also clears the gradient for the next step.
__global__ __launch_bounds__(SW) void k_sur_adam(float* __restrict__ th, float* __restrict__ grad,
                                                 float* __restrict__ m, float* __restrict__ v, int step, float lr,
                                                 float b1, float b2, float eps) {
    const int i = blockIdx.x * SW + threadIdx.x;
    if (i >= SUR_PARAMS) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)step));
    const float vh = vi / (1.0f - powf(b2, (float)step));
    th[i] -= lr * mh / (sqrtf(vh) + eps);
    grad[i] = 0.0f;
}

__global__ __launch_bounds__(SW) void k_sur_zero(float* __restrict__ p, int n) {
    const int i = blockIdx.x * SW + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Column means and standard deviations (floored) of X [count][SUR_IN] and
// T [count][SUR_OUT]: one workgroup per column, FP64 sums.
__global__ __launch_bounds__(SW) void k_sur_norm(const float* __restrict__ X, const float* __restrict__ T,
                                                 int64_t count, float floor_sd, float* __restrict__ norm) {
    const int col = blockIdx.x;  // 0..11 inputs, 12..23 outputs
    const float* A = col < SUR_IN ? X : T;
    const int ld = col < SUR_IN ? SUR_IN : SUR_OUT;
    const int c = col < SUR_IN ? col : col - SUR_IN;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += SW) {
        const double a = A[i * ld + c];
        s1 += a;
        s2 += a * a;
    }
    __shared__ double r1[SW], r2[SW];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int d = SW / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            r1[threadIdx.x] += r1[threadIdx.x + d];
            r2[threadIdx.x] += r2[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = r1[0] / (double)count;
        double var = r2[0] / (double)count - mean * mean;
        if (var < 0.0) var = 0.0;
        const float sd = fmaxf((float)sqrt(var), floor_sd);
        if (col < SUR_IN) {
            norm[c] = (float)mean;
            norm[SUR_IN + c] = sd;
        } else {
            norm[2 * SUR_IN + c] = (float)mean;
            norm[2 * SUR_IN + SUR_OUT + c] = sd;
        }
    }
}

// Minibatch rows: idx[i] = splitmix64(seed + (step * 2^32 + i) * golden) mod count
// (splitmix64 as published by Steele, Lea and Flood: add the golden gamma,
// then two xor-shift-multiply rounds and a final xor-shift).
__global__ __launch_bounds__(SW) void k_sur_indices(uint64_t seed, int step, int batch, int64_t count,
                                                    int* __restrict__ idx) {
    const int i = blockIdx.x * SW + threadIdx.x;
    if (i >= batch) return;
    uint64_t z = seed + (((uint64_t)step << 32) + (uint64_t)i) * 0x9E3779B97F4A7C15ull + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    idx[i] = (int)(z % (uint64_t)count);
}

// Training pairs: the trial state of each particle of `scene` (the deferred
// update applied when `pending`) through the exact snow return map, written
// as feature and target rows (compacted with a counter, one atomic add per
// wave for the wave's rows; rows of inverted particles are skipped).
__global__ __launch_bounds__(SW) void k_sur_sample(const float* __restrict__ S, int64_t cap, int N, Scenes T,
                                                   int scene, int pending, float E, float dt_ref, int64_t max_rows,
                                                   float* __restrict__ X, float* __restrict__ Y,
                                                   unsigned long long* __restrict__ counter) {
    const int j0 = blockIdx.x * SW + threadIdx.x;
    bool ok = j0 < N && fsid_scene(S[sidx(FSID, j0 < N ? j0 : 0, cap)]) == scene;
    const int j = ok ? j0 : 0;
    const Scene& sc = T.scene[scene];
    const Mat& M = sc.M;
    float C[9], F[9], Fh[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        C[k] = S[sidx(FC + k, j, cap)];
        F[k] = S[sidx(FF + k, j, cap)];
    }
    const float Jp = S[sidx(FS, j, cap)];
    if (pending)
        advance_gradient(C, sc.P.dt, F, Fh);
    else
#pragma unroll
        for (int k = 0; k < 9; ++k) Fh[k] = F[k];
    float U[9], sig[3], J;
    left_svd(Fh, U, sig, J);
    // descending order
    float a = sig[0], b = sig[1], c = sig[2], t;
    if (a < b) { t = a; a = b; b = t; }
    if (b < c) { t = b; b = c; c = t; }
    if (a < b) { t = a; a = b; b = t; }
    ok = ok && c > 0.0f && Jp > 0.0f;
    // the wave's rows take consecutive slots from one add to the counter
    const unsigned long long m = __ballot(ok);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63, first = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == first) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(base >> 32), first) << 32) |
           (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, first);
    if (!ok) return;
    const float s[3] = {a, b, c};
    float sn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sn[k] = fminf(fmaxf(s[k], M.lo), M.hi);
    const float Js = s[0] * s[1] * s[2], Jn = sn[0] * sn[1] * sn[2];
    const float Jpn = Jp * Js / Jn;
    const float hn = expf(M.xi * (1.0f - Jpn));
    const unsigned long long r = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
    if ((int64_t)r >= max_rows) return;
    float* x = X + r * SUR_IN;
    float* y = Y + r * SUR_OUT;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        x[k] = s[k];
        x[3 + k] = logf(s[k]);
        y[k] = sn[k];
        y[3 + k] = logf(sn[k] / s[k]);
        y[6 + k] = (2.0f * M.mu * hn * (sn[k] - 1.0f) * sn[k] + M.la * hn * (Jn - 1.0f) * Jn) / E;
    }
    x[6] = Jp;
    x[7] = logf(Jp);
    x[8] = expf(M.xi * (1.0f - Jp));
    x[9] = div_refined(sc.P.dt, dt_ref);  // as P2G computes it (exactly 1 at dt_ref)
    x[10] = Js;
    x[11] = 1.0f;
    y[9] = Jpn / Jp;
    y[10] = hn;
    y[11] = Jn;
}

}  // namespace

void sur_indices(hipStream_t st, uint64_t seed, int step, int batch, int64_t count, int* idx) {
    hipLaunchKernelGGL(k_sur_indices, dim3((batch + SW - 1) / SW), dim3(SW), 0, st, seed, step, batch, count, idx);
}

void sur_sample(hipStream_t st, const float* S, int64_t cap, int N, const Scenes& T, int scene, int pending, float E,
                float dt_ref, int64_t max_rows, float* X, float* Y, unsigned long long* counter) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_sur_sample, dim3((N + SW - 1) / SW), dim3(SW), 0, st, S, cap, N, T, scene, pending, E, dt_ref,
                       max_rows, X, Y, counter);
}

void sur_forward(hipStream_t st, int bf16, const float* th, const float* norm, const float* X, int64_t count,
                 float* Y) {
    if (count <= 0) return;
    const int64_t tiles = (count + 15) / 16;
    const int grid = (int)((tiles + 3) / 4 < 4096 ? (tiles + 3) / 4 : 4096);
    if (bf16) {  // the inference path P2G runs
        const int64_t groups = (count + 63) / 64;
        const int g16 = (int)((groups + 3) / 4 < 4096 ? (groups + 3) / 4 : 4096);
        hipLaunchKernelGGL(k_sur_forward16, dim3(g16), dim3(SW), 0, st, th, norm, X, count, Y);
    } else {
        hipLaunchKernelGGL(k_sur_forward<false>, dim3(grid), dim3(SW), 0, st, th, norm, X, count, Y);
    }
}

void sur_grad(hipStream_t st, int bf16, const float* th, const float* norm, const float* X, const float* T,
              int64_t count, const int* idx, float* grad, float* loss, bool zero) {
    if (zero) {
        hipLaunchKernelGGL(k_sur_zero, dim3((SUR_PARAMS + SW - 1) / SW), dim3(SW), 0, st, grad, SUR_PARAMS);
        hipLaunchKernelGGL(k_sur_zero, dim3(1), dim3(SW), 0, st, loss, 1);
    }
    if (count <= 0) return;
    const int64_t tiles = (count + 15) / 16;
    const int grid = (int)((tiles + 3) / 4 < 1024 ? (tiles + 3) / 4 : 1024);
    if (bf16)
        hipLaunchKernelGGL(k_sur_grad<true>, dim3(grid), dim3(SW), 0, st, th, norm, X, T, count, idx, grad, loss);
    else
        hipLaunchKernelGGL(k_sur_grad<false>, dim3(grid), dim3(SW), 0, st, th, norm, X, T, count, idx, grad, loss);
}

void sur_adam(hipStream_t st, float* th, float* grad, float* m, float* v, int step, float lr) {
    hipLaunchKernelGGL(k_sur_adam, dim3((SUR_PARAMS + SW - 1) / SW), dim3(SW), 0, st, th, grad, m, v, step, lr, 0.9f,
                       0.999f, 1e-8f);
}

void sur_zero(hipStream_t st, float* p, int n) {
    if (n > 0) hipLaunchKernelGGL(k_sur_zero, dim3((n + SW - 1) / SW), dim3(SW), 0, st, p, n);
}

void sur_norm(hipStream_t st, const float* X, const float* T, int64_t count, float* norm) {
    hipLaunchKernelGGL(k_sur_norm, dim3(SUR_IN + SUR_OUT), dim3(SW), 0, st, X, T, count, 1e-6f, norm);
}

}  // namespace mpm
