// Layout of the constitutive surrogate's parameters and normalisation, and
// the launchers of its kernels (mpm_surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

// MLP 12 -> 64 -> 64 -> 12.  Flat FP32 parameters, weights row-major
// (output, input): W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [12][64], b3 [12].
constexpr int SUR_IN = 12, SUR_H = 64, SUR_OUT = 12;
constexpr int SUR_W1 = 0;
constexpr int SUR_B1 = SUR_W1 + SUR_H * SUR_IN;
constexpr int SUR_W2 = SUR_B1 + SUR_H;
constexpr int SUR_B2 = SUR_W2 + SUR_H * SUR_H;
constexpr int SUR_W3 = SUR_B2 + SUR_H;
constexpr int SUR_B3 = SUR_W3 + SUR_OUT * SUR_H;
constexpr int SUR_PARAMS = SUR_B3 + SUR_OUT;  // 5772
// Normalisation: input means [12], input sds [12], output means [12], output sds [12].
constexpr int SUR_NORM = 2 * (SUR_IN + SUR_OUT);

// Features of a trial state (descending singular values s, plastic volume
// J_P): [s1..s3, ln s1..s3, J_P, ln J_P, exp(xi (1 - J_P)), dt/dt_ref, s1 s2 s3, 1].
// Targets: [s'1..s'3, ln(s'/s)1..3, tau1..3 / E, J_P'/J_P, exp(xi (1 - J_P')), s'1 s'2 s'3].

void sur_forward(hipStream_t st, int bf16, const float* th, const float* norm, const float* X, int64_t count,
                 float* Y);
// Zeroes grad and loss first when `zero`; idx (may be NULL) selects the rows of X and T.
void sur_grad(hipStream_t st, int bf16, const float* th, const float* norm, const float* X, const float* T,
              int64_t count, const int* idx, float* grad, float* loss, bool zero);
void sur_adam(hipStream_t st, float* th, float* grad, float* m, float* v, int step, float lr);
void sur_zero(hipStream_t st, float* p, int n);
void sur_norm(hipStream_t st, const float* X, const float* T, int64_t count, float* norm);
void sur_indices(hipStream_t st, uint64_t seed, int step, int batch, int64_t count, int* idx);
struct Scenes;
void sur_sample(hipStream_t st, const float* S, int64_t cap, int N, const Scenes& T, int scene, int pending, float E,
                float dt_ref, int64_t max_rows, float* X, float* Y, unsigned long long* counter);

}  // namespace mpm
