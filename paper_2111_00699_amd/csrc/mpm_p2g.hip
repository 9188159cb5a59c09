// P2G on gfx950: particle-to-grid transfer with the deferred deformation
// update, the snow return map and the Kirchhoff stress fused in (paper,
// "Merge Kernels": plasticity, SVD and stress computed inside P2G).
//
// Avoiding non-native intrinsics ("Avoid non-native intrinsics"): on V100
// the paper drops shared-memory float atomics because they are emulated.
// On gfx950 ds_add_f32 exists but runs at about 0.3 lane-ops per clock per
// CU, while ds_add_f64 runs at about 6.6 and ds_add_u64 at 9.1 (and far
// better under bank and address conflicts), and global float atomics (about
// 0.4, executed memory-side) move a full write per update.  The same
// principle -- use only the fast native operations -- leads here to:
//   * a workgroup takes one chunk (<= 256 or 512 particles of one particle
//     block), one particle per thread, loads coalesced;
//   * phase 1 computes every particle's contribution and the bounding box of
//     the stencils of the chunk's in-zone particles (block reduction);
//   * the tile is that box (at most 1024 padded nodes; a particle block's
//     stencils cover 6^3 = 216 nodes right after a rebuild), four 64-bit
//     fixed-point channels (weight sum and three momentum components, the
//     latter scaled per chunk) accumulated with ds_add_u64: exact, so the
//     sums do not depend on the order of the adds;
//   * the tile is then STORED (plain, coalesced float4 stores) to the
//     staging buffer; the rebuild registered each chunk with every physical
//     block its in-zone stencils can reach, and the grid update gathers each
//     node from the registered tiles whose box holds it, in chunk order --
//     no global atomics, and the transfer of in-zone particles is
//     deterministic.  Each workgroup owns an
//     equal slice of the staging buffer and packs its chunks' tiles there
//     (offset recorded per chunk), so no allocation is shared.
// The rebuild stores each chunk dealt over its 16-lane LDS passes by the
// bank pair of each particle's cell in this tile layout, so the 16 lanes of
// one LDS access meet each bank pair about as rarely as the chunk's cells
// allow and rarely share an address (conflicting lanes of a pass
// serialize; lanes in different passes do not conflict).
// Particles outside their free zone (before a late rebuild) scatter straight
// to global atomics and activate the blocks they touch.
#include <type_traits>

#include "mpm_kernels.h"
#include "mpm_mlp.h"

namespace mpm {

namespace {

constexpr int CT = 1024;  // LDS tile capacity in nodes (padded layout, below)

// LDS tile layout: the padded node-box layout (pitch_row, pitch_plane in
// mpm_kernels.h), four 64-bit fixed-point channels: the weight sum in units
// of 2^-51 and the three momentum components in units of 2^-FRAC_M of the
// chunk's momentum scale (below).  Integer adds are exact and
// order-independent, and ds_add_u64 meets far fewer conflict cycles than
// ds_add_f64 (a replay of late-frame snow stencils: 14 against 22 cycles per
// wave instruction).
constexpr float W_SCALE = 0x1p51f;  // weight units per 1: w <= 27/64, so w W_SCALE < 2^50
constexpr int FRAC_M = 50;          // momentum: |w m| scaled below 2^50 per contribution
// A contribution below this weight goes to the global FP32 accumulator
// instead: a node that only such contributions reach would be resolved to
// too few fixed-point units for its velocity (momentum / mass).
constexpr float TINY_W = 0x1p-32f;

// Round-to-nearest integer of y (|y| < 2^51) as a 64-bit two's-complement
// word: adding 1.5 2^52 in FP64 leaves the integer in the low mantissa bits.
__device__ __forceinline__ unsigned long long fixed64(float y) {
    return (unsigned long long)(__double_as_longlong((double)y + 0x1.8p52) - 0x4338000000000000LL);
}

// ------------------------------------------------ snow return map without SVD
// Eigenvalues of the symmetric b = [b0 b1 b2; . b3 b4; . . b5] as
// q + p mu_k, mu descending, by the trigonometric solution of the
// characteristic cubic of the normalised deviator Bn = (b - q I)/p (whose
// eigenvalues mu satisfy mu^3 - 3 mu - det Bn = 0).  Returns false when b is
// too close to a multiple of the identity for the deviator to be resolved.
__device__ __forceinline__ bool eig_closed(const float b[6], float& q, float& p, float mu[3], float Bn[6]) {
    q = (b[0] + b[3] + b[5]) * (1.0f / 3.0f);
    const float d0 = b[0] - q, d1 = b[3] - q, d2 = b[5] - q;
    const float p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0f * (b[1] * b[1] + b[2] * b[2] + b[4] * b[4]);
    p = sqrtf(p2 * (1.0f / 6.0f));
    if (!(p > 2e-5f * fabsf(q))) return false;
    const float ip = 1.0f / p;
    Bn[0] = d0 * ip; Bn[1] = b[1] * ip; Bn[2] = b[2] * ip;
    Bn[3] = d1 * ip; Bn[4] = b[4] * ip; Bn[5] = d2 * ip;
    const float det = Bn[0] * (Bn[3] * Bn[5] - Bn[4] * Bn[4]) - Bn[1] * (Bn[1] * Bn[5] - Bn[4] * Bn[2]) +
                      Bn[2] * (Bn[1] * Bn[4] - Bn[3] * Bn[2]);
    const float phi = acosf(fminf(fmaxf(0.5f * det, -1.0f), 1.0f)) * (1.0f / 3.0f);
    mu[0] = 2.0f * cosf(phi);
    mu[2] = 2.0f * cosf(phi + 2.09439510f);  // + 2 pi / 3
    mu[1] = -mu[0] - mu[2];
    return true;
}

// sum_k c_k L_k(Bn) = A2 Bn^2 + A1 Bn + A0 I, with L_k the Lagrange
// polynomials on the (distinct) eigenvalues mu: each L_k(Bn) is the
// projector on eigenvector k (Sylvester's formula), so isotropic functions
// of b are built without eigenvectors.
__device__ __forceinline__ void lagrange(const float mu[3], const float c[3], float& A2, float& A1, float& A0) {
    A2 = A1 = A0 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = (k + 1) % 3, j = (k + 2) % 3;
        const float w = c[k] / ((mu[k] - mu[i]) * (mu[k] - mu[j]));
        A2 += w;
        A1 += w * mu[k];  // -(mu_i + mu_j) = mu_k since the mu sum to zero
        A0 += w * mu[i] * mu[j];
    }
}

// The snow return map and Kirchhoff stress of every lane's particle from the
// eigenvalues of b = F^ F^T alone: F_E' = (I + sum_k delta_k L_k) F^ and
// tau = tau_bar I + sum_k (tau_k - tau_bar) L_k, with delta_k = s'_k/s_k - 1.
// The projected values come from the exact clamp (ret = 2) or from the
// network (ret = 1; all lanes of the wave run it on MFMA).  A lane falls
// back to the exact (Jacobi) map when its eigenvalues are too close, its
// particle is inverted, or (network) the prediction leaves the yield
// surface or changes the total volume by more than the tolerance.
template <bool NET>
__device__ void snow_without_svd(const mlp::NetLds16* net, float* stage, const Scenes& T, const Scene& sc, float dt,
                                 int pending, bool have, const float C[9], float F[9], float& s, float tau[6],
                                 bool& fell_back) {
    const Mat& M = sc.M;
    float Fh[9];
    if (pending) {
        advance_gradient(C, dt, F, Fh);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Fh[k] = F[k];
    }
    float b[6];
    b[0] = Fh[0] * Fh[0] + Fh[1] * Fh[1] + Fh[2] * Fh[2];
    b[1] = Fh[0] * Fh[3] + Fh[1] * Fh[4] + Fh[2] * Fh[5];
    b[2] = Fh[0] * Fh[6] + Fh[1] * Fh[7] + Fh[2] * Fh[8];
    b[3] = Fh[3] * Fh[3] + Fh[4] * Fh[4] + Fh[5] * Fh[5];
    b[4] = Fh[3] * Fh[6] + Fh[4] * Fh[7] + Fh[5] * Fh[8];
    b[5] = Fh[6] * Fh[6] + Fh[7] * Fh[7] + Fh[8] * Fh[8];
    float q, p, mu[3], Bn[6];
    bool use = have && eig_closed(b, q, p, mu, Bn) && det3(Fh) > 0.0f;
    use = use && (mu[0] - mu[1]) >= T.sur_gap && (mu[1] - mu[2]) >= T.sur_gap;
    float sh[3], sn[3], tk[3], Jpn;
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k] = use ? sqrtf(fmaxf(q + p * mu[k], 1e-30f)) : 1.0f;
    const float Jp = use ? s : 1.0f;
    if (NET && pending && __ballot(use) != 0ull) {  // a wave with no eligible lane skips the network
        // features [s, ln s, J_P, ln J_P, h, dt/dt_ref, s1 s2 s3, 1], the wave's 64 samples at once.
        // dt/dt_ref is exactly 1 at the training step (a refined division): a feature that was
        // constant in training has a floored spread (1e-6), so one ulp off would move its
        // normalised value by 0.06 and the J_P output by about 4e-4.
        const float dtr = div_refined(dt, T.sur_dt_ref);
        const float xf[SUR_IN] = {sh[0], sh[1], sh[2], logf(sh[0]), logf(sh[1]), logf(sh[2]), Jp, logf(Jp),
                                  expf(M.xi * (1.0f - Jp)), dtr, sh[0] * sh[1] * sh[2], 1.0f};
        float xn[SUR_IN], yv[SUR_OUT];
#pragma unroll
        for (int f = 0; f < SUR_IN; ++f) xn[f] = (xf[f] - net->imu[f]) / net->isd[f];
        mlp::forward_wave16(*net, stage, xn, yv);
#pragma unroll
        for (int o = 0; o < SUR_OUT; ++o) yv[o] = yv[o] * net->osd[o] + net->omu[o];
        // outputs [s', ln(s'/s), tau/E, J_P'/J_P, h', s1's2's3']: the projected state comes from
        // ln(s'/s) and J_P'/J_P; the stress is evaluated from that state, and the network's own
        // stress outputs serve as a consistency check
        float res_t = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) sn[k] = sh[k] * expf(yv[3 + k]);
        Jpn = Jp * yv[9];
        {
            const float h = expf(M.xi * (1.0f - Jpn));
            const float Jn = sn[0] * sn[1] * sn[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                tk[k] = 2.0f * M.mu * h * (sn[k] - 1.0f) * sn[k] + M.la * h * (Jn - 1.0f) * Jn;
                res_t = fmaxf(res_t, fabsf(yv[6 + k] - tk[k] / sc.E));
            }
        }
        float res_y = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) res_y = fmaxf(res_y, fmaxf(M.lo - sn[k], sn[k] - M.hi));
        const float res_v = fabsf(logf(sn[0] * sn[1] * sn[2] * Jpn) - logf(sh[0] * sh[1] * sh[2] * Jp));
        const bool fin = isfinite(tk[0] + tk[1] + tk[2] + Jpn + sn[0] + sn[1] + sn[2]);
        use = use && fin && res_y <= T.sur_tol && res_v <= T.sur_tol && res_t <= T.sur_tol;
    } else {
        // exact clamp; with nothing pending the stored state is already projected
        // (as in the exact path), so only the stress is evaluated
#pragma unroll
        for (int k = 0; k < 3; ++k) sn[k] = pending ? fminf(fmaxf(sh[k], M.lo), M.hi) : sh[k];
        Jpn = Jp * (sh[0] * sh[1] * sh[2]) / (sn[0] * sn[1] * sn[2]);
        const float h = expf(M.xi * (1.0f - Jpn));
        const float Jn = sn[0] * sn[1] * sn[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) tk[k] = 2.0f * M.mu * h * (sn[k] - 1.0f) * sn[k] + M.la * h * (Jn - 1.0f) * Jn;
    }
    fell_back = have && !use;
    if (!have) return;
    if (!use) {
        material_step(M, dt, pending, C, F, s, tau);
        return;
    }
    float B2[6];
    B2[0] = Bn[0] * Bn[0] + Bn[1] * Bn[1] + Bn[2] * Bn[2];
    B2[1] = Bn[0] * Bn[1] + Bn[1] * Bn[3] + Bn[2] * Bn[4];
    B2[2] = Bn[0] * Bn[2] + Bn[1] * Bn[4] + Bn[2] * Bn[5];
    B2[3] = Bn[1] * Bn[1] + Bn[3] * Bn[3] + Bn[4] * Bn[4];
    B2[4] = Bn[1] * Bn[2] + Bn[3] * Bn[4] + Bn[4] * Bn[5];
    B2[5] = Bn[2] * Bn[2] + Bn[4] * Bn[4] + Bn[5] * Bn[5];
    // F_E' = G F^ with G = I + sum_k delta_k L_k
    float dl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dl[k] = sn[k] / sh[k] - 1.0f;
    float A2, A1, A0;
    lagrange(mu, dl, A2, A1, A0);
    float G[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) G[e] = A2 * B2[e] + A1 * Bn[e];
    G[0] += 1.0f + A0;
    G[3] += 1.0f + A0;
    G[5] += 1.0f + A0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float f0 = Fh[0 * 3 + c], f1 = Fh[1 * 3 + c], f2 = Fh[2 * 3 + c];
        F[0 * 3 + c] = G[0] * f0 + G[1] * f1 + G[2] * f2;
        F[1 * 3 + c] = G[1] * f0 + G[3] * f1 + G[4] * f2;
        F[2 * 3 + c] = G[2] * f0 + G[4] * f1 + G[5] * f2;
    }
    s = Jpn;
    // tau = tau_bar I + sum_k (tau_k - tau_bar) L_k
    const float tb = (tk[0] + tk[1] + tk[2]) * (1.0f / 3.0f);
    const float dt3[3] = {tk[0] - tb, tk[1] - tb, tk[2] - tb};
    lagrange(mu, dt3, A2, A1, A0);
#pragma unroll
    for (int e = 0; e < 6; ++e) tau[e] = A2 * B2[e] + A1 * Bn[e];
    tau[0] += tb + A0;
    tau[3] += tb + A0;
    tau[5] += tb + A0;
}

// NT threads per workgroup = the largest chunk it takes (128, 256 or 512).
// SURM: 0 every snow scene takes the exact map; 1 some scene takes the
// closed form without SVD; 2 some scene takes the network (staged in LDS).
// FUSED (with the tile path and the exact map only): each chunk first does
// the previous substep's G2P -- gathered from the node box of that
// substep's tile, staged in the tile's LDS -- and scatters with the fresh
// v, C and x; the particle's v and C are not stored (the G2P that brings the
// state up to date before a read recomputes them).  vel, host_flag and
// fb_limit serve that G2P.
template <bool GLOBAL_ONLY, int NT, int SURM, bool FUSED>
__device__ __forceinline__ void p2g_body(float* __restrict__ S, int64_t cap, const Chunk* __restrict__ chunks,
                                         int* __restrict__ ctl, float* __restrict__ acc,
                                         int* __restrict__ acc_dirty, float4* __restrict__ stage,
                                         int stage_nodes, int4* __restrict__ box, int* __restrict__ brick_state,
                                         int* __restrict__ ovf, int parity, const Scenes& T, int pending,
                                         int nbricks, int act, const float4* __restrict__ vel,
                                         int* __restrict__ host_flag, int fb_limit) {
    static_assert(!FUSED || (!GLOBAL_ONLY && SURM == 0), "the fused G2P needs the LDS tile and the exact map");
    __shared__ __align__(16) double tq[GLOBAL_ONLY ? 1 : 4 * CT];
    __shared__ int red_i[7][NT / 64];
#ifndef MPM_WEIGHTS_IN_LDS
#define MPM_WEIGHTS_IN_LDS 0
#endif
#if MPM_WEIGHTS_IN_LDS
    __shared__ float wpark[9 * NT];
#endif
    struct Empty {};
    __shared__ typename std::conditional<SURM == 2, mlp::NetLds16, Empty>::type net;
    __shared__ __attribute__((aligned(16))) float sur_stage[SURM == 2 ? NT / 64 * mlp::FWD_STAGE : 1];
    if constexpr (SURM == 2) {
        if (T.sur_theta) mlp::load_net16(net, T.sur_theta, T.sur_norm);
        __syncthreads();
    }
    int begin, end, stride;
    xcd_split(rank_limit(T, ctl, act, RE_CHUNK, CTL_NCHUNK), begin, end, stride);
    if constexpr (!GLOBAL_ONLY) {  // (workgroup-uniform: skipped by a workgroup without chunks)
        if (begin < end) {
            for (int t = threadIdx.x; t < 4 * CT; t += NT) tq[t] = 0.0;
            __syncthreads();
        }
    }
    unsigned err = 0;
    unsigned n_sur = 0, n_fb = 0;
    // fused G2P: the free-zone request, as the G2P kernel makes it (the
    // previous substep's P2G counted its tile fallbacks in the other slot)
    bool left = FUSED && blockIdx.x == 0 && threadIdx.x == 0 && ctl[CTL_FB + (parity ^ 1)] > fb_limit;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // this workgroup's slice of the staging buffer, filled front to back
    const int slice = (int)((int64_t)stage_nodes / gridDim.x);
    const int slice0 = slice * (int)blockIdx.x;
    int used = 0;
    for (int c = begin; c < end; c += stride) {
        const Chunk ch = chunks[c];
        const Scene& sc = T.scene[ch.scene];
        const Step P = sc.P;
        const Mat M = sc.M;
        const float dx = P.dx, dt = P.dt;
        const int count = ch.count;
        const bool have = tid < count;
        const int p = ch.start + (have ? tid : 0);

        // ---- phase 1: material update, stress and this particle's payload
        Stencil st;
        float q[3] = {0.f, 0.f, 0.f}, Ad[9];
        bool ok = false, in_zone = false;
        float x[3] = {0.5f, 0.5f, 0.5f}, v[3] = {0.f, 0.f, 0.f}, C[9], F[9], s = 1.0f, tau[6];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            C[k] = 0.0f;
            F[k] = (k % 4 == 0) ? 1.0f : 0.0f;
        }
        if (have) {
#pragma unroll
            for (int a = 0; a < 3; ++a) x[a] = S[sidx(FX + a, p, cap)];
            if (!FUSED) {
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a] = S[sidx(FV + a, p, cap)];
#pragma unroll
                for (int k = 0; k < 9; ++k) C[k] = S[sidx(FC + k, p, cap)];
            }
            s = S[sidx(FS, p, cap)];
            if (M.kind != MPM_WATER) {
#pragma unroll
                for (int k = 0; k < 9; ++k) F[k] = S[sidx(FF + k, p, cap)];
            }
        }
        int B[3] = {0, 0, 0};  // the particle's block at the last rebuild (its free zone)
        if (have) fsid_block(S[sidx(FSID, p, cap)], B);
        int ng = 0, ngs = 0;  // fused G2P: nodes of the previous box, and the LDS float4 they span
        if constexpr (FUSED) {
            const int4 bb = box[c];  // this chunk's tile box of the previous substep
            const int lg[3] = {bb.x & 1023, (bb.x >> 10) & 1023, bb.x >> 20};
            const int eg[3] = {bb.y & 255, (bb.y >> 8) & 255, bb.y >> 16};
            ng = eg[0] * eg[1] * eg[2];
            const int Rg = pitch_row(eg[0]), Qg = pitch_plane(Rg, eg[1]);  // padded: no bank conflicts
            ngs = ng > 0 ? Qg * eg[2] : 0;
            if (ngs > 2 * CT) ng = ngs = 0;  // the tile holds 2 CT float4
            float4* tv = reinterpret_cast<float4*>(tq);
            const float4* vels = vel + (int64_t)sc.brick_base * BLOCK_NODES;
            load_node_box(tv, vels, P.NB, lg, eg, ng, Rg, Qg, tid, NT);
            __syncthreads();
            Stencil sg;
            if (have && make_stencil(x, P, sg, err)) {
                g2p_gather(sg, tv, vels, P.NB, lg, eg, ng, Rg, Qg, 4.0f * P.fn, v, C);
                bool fin = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    x[a] += dt * v[a];
                    S[sidx(FX + a, p, cap)] = x[a];
                    fin = fin && (fabsf(x[a]) < 1e30f) && (fabsf(v[a]) < 1e30f);
                }
                left = left || left_free_zone(x, P.fn, B);
                if (!fin) err |= MPM_ERR_NONFINITE;
            }
        }
        bool sur_chunk = false;
        if constexpr (SURM != 0) {
            sur_chunk = sc.ret != 0 && M.kind == MPM_SNOW;  // uniform over the workgroup
            if (sur_chunk) {
                bool fb = false;
                if constexpr (SURM == 2) {
                    if (sc.ret == 1)
                        snow_without_svd<true>(&net, sur_stage + wv * mlp::FWD_STAGE, T, sc, dt, pending, have, C, F, s, tau, fb);
                    else
                        snow_without_svd<false>(&net, sur_stage, T, sc, dt, pending, have, C, F, s, tau, fb);
                } else {  // no network in this variant
                    snow_without_svd<false>(nullptr, nullptr, T, sc, dt, pending, have, C, F, s, tau, fb);
                }
                n_sur += __popcll(__ballot(have && !fb));
                n_fb += __popcll(__ballot(fb));
            }
        }
        if (!sur_chunk && have) material_step(M, dt, pending, C, F, s, tau);
        if (have) {
            if (pending) {  // the deferred update of the last G2P lands here
                if (M.kind != MPM_WATER) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) S[sidx(FF + k, p, cap)] = F[k];
                }
                if (M.kind != MPM_JELLY) S[sidx(FS, p, cap)] = s;
            }
            ok = make_stencil(x, P, st, err);
#if MPM_WEIGHTS_IN_LDS  // the register-pressure ablation: weights parked in LDS until the scatter
#pragma unroll
            for (int k = 0; k < 9; ++k) wpark[k * NT + tid] = st.w[k / 3][k % 3];
#endif
            // A = m C - (4 dt V0 / dx^2) tau;  Ad = dx A;  q = m v - Ad f, so the
            // momentum sent to stencil node o is w_o (q + Ad o).
            const float Tf[9] = {tau[0], tau[1], tau[2], tau[1], tau[3], tau[4], tau[2], tau[4], tau[5]};
#pragma unroll
            for (int k = 0; k < 9; ++k) Ad[k] = dx * (M.mp * C[k] - M.scale * Tf[k]);
#pragma unroll
            for (int a = 0; a < 3; ++a)
                q[a] = M.mp * v[a] - (Ad[a * 3 + 0] * st.f[0] + Ad[a * 3 + 1] * st.f[1] + Ad[a * 3 + 2] * st.f[2]);
            in_zone = ok;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int l = st.base[a] - (4 * B[a] - 4);
                in_zone = in_zone && l >= 0 && l <= TILE - 3;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) Ad[k] = 0.0f;
        }

        // ---- the box of the in-zone stencils of the chunk
        int lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
        int nt = 0, off = 0, R = 4, Q = 8;  // tight node count, staging offset, LDS pitches
        float m_scale = 1.0f, m_unit = 1.0f;  // momentum fixed-point scale of the chunk and its inverse
        if (GLOBAL_ONLY && tid == 0) box[c] = make_int4(0, 0, 0, 0);
        if (!GLOBAL_ONLY) {
            const bool tiled = have && in_zone;
            int mn[3], mx[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = wave_min(tiled ? st.base[a] : INT_MAX);
                mx[a] = wave_max(tiled ? st.base[a] + 2 : INT_MIN);
            }
            // bound on |q_a + Ad_a . o| over the stencil (o in {0,1,2}^3), the momentum a tiled
            // particle sends to a node before its weight (non-negative: ordered as an int)
            float mb = 0.0f;
            if (tiled) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    mb = fmaxf(mb, fabsf(q[a]) + 2.0f * (fabsf(Ad[3 * a]) + fabsf(Ad[3 * a + 1]) + fabsf(Ad[3 * a + 2])));
            }
            const int mbw = wave_max(__float_as_int(mb));
            if (lane == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    red_i[a][wv] = mn[a];
                    red_i[3 + a][wv] = mx[a];
                }
                red_i[6][wv] = mbw;
            }
            __syncthreads();
            if constexpr (FUSED) {  // every gather is done: clear the staged node box, keeping the tile zero
                for (int t = tid; t < 2 * ngs; t += NT) tq[t] = 0.0;
                __syncthreads();
            }
            int hi[3], mbk = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = INT_MAX;
                hi[a] = INT_MIN;
            }
#pragma unroll
            for (int k = 0; k < NT / 64; ++k) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lo[a] = min(lo[a], red_i[a][k]);
                    hi[a] = max(hi[a], red_i[3 + a][k]);
                }
                mbk = max(mbk, red_i[6][k]);
            }
            // the chunk's momentum scale 2^(FRAC_M - em): every contribution |w m| < 27/64 * bound
            // < 2^em stays below 2^FRAC_M units
            {
                int em = 0;
                (void)frexpf(0.421875f * __int_as_float(mbk), &em);
                em = min(max(em, -70), 77);
                m_scale = ldexpf(1.0f, FRAC_M - em);
                m_unit = ldexpf(1.0f, em - FRAC_M);
            }
            if (hi[0] >= lo[0]) {
#pragma unroll
                for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a] + 1;
                nt = ext[0] * ext[1] * ext[2];
                R = pitch_row(ext[0]);
                Q = pitch_plane(R, ext[1]);
            }
            // no room in the tile or in this workgroup's staging slice: the chunk goes to global atomics
            if (Q * ext[2] > CT || used + nt > slice) nt = -1;
            if (!ch.tile) nt = -1;  // a registration list was full at the rebuild
            if (nt < 0 && tid == 0) atomicAdd(&ctl64(ctl, blockIdx.x)[CTL64_FALLBACK_CHUNKS], 1ull);
            off = slice0 + used;
            if (nt > 0) used += nt;
            // (the tile is all zero here: cleared at the start, and every node a chunk touched is
            // zeroed again as it is stored)
            if (tid == 0)
                box[c] = nt > 0 ? make_int4(lo[0] | (lo[1] << 10) | (lo[2] << 20), ext[0] | (ext[1] << 8) | (ext[2] << 16),
                                            off, 0)
                                : make_int4(0, 0, 0, 0);
        }

        // ---- phase 2: scatter
        {
            const unsigned long long g = __ballot(have && ok && (GLOBAL_ONLY || !in_zone || nt <= 0));
            if (g && lane == 0)
                atomicAdd(&ctl64(ctl, blockIdx.x * (NT / 64) + wv)[CTL64_GLOBAL_PARTICLES], (unsigned long long)__popcll(g));
            // in-zone particles that lost the tile: a rebuild would shrink their chunk's box again
            const unsigned long long fb = __ballot(have && ok && !GLOBAL_ONLY && in_zone && nt <= 0);
            if (fb && lane == 0) atomicAdd(&ctl[CTL_FB + parity], (int)__popcll(fb));
        }
#if MPM_WEIGHTS_IN_LDS  // (a barrier separates the store from this load)
        if (have) {
#pragma unroll
            for (int k = 0; k < 9; ++k) st.w[k / 3][k % 3] = wpark[k * NT + tid];
        }
#endif
        // Tile lanes whose stencil holds a weight below TINY_W send those
        // contributions to the global accumulators instead; the smallest of a
        // stencil's 27 weights is the product of its per-axis minima.  The
        // per-node test is only compiled into the pass of waves that have
        // such a lane (rare: a coordinate within 2^-11 dx of a cell edge).
        bool any_tiny = false;
        if (!GLOBAL_ONLY) {
            float wmin = 1.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) wmin *= fminf(fminf(st.w[a][0], st.w[a][1]), st.w[a][2]);
            any_tiny = __any(have && ok && in_zone && nt > 0 && wmin < TINY_W);
        }
        if (have && ok) {
            if (!GLOBAL_ONLY && in_zone && nt > 0) {
                const int tb = (st.base[0] - lo[0]) + R * (st.base[1] - lo[1]) + Q * (st.base[2] - lo[2]);
                unsigned long long* tu = reinterpret_cast<unsigned long long*>(tq);
                float qs[3], As[9];  // in momentum units (exact: a power-of-two scale)
#pragma unroll
                for (int a = 0; a < 3; ++a) qs[a] = q[a] * m_scale;
#pragma unroll
                for (int k = 0; k < 9; ++k) As[k] = Ad[k] * m_scale;
                auto scatter = [&](auto check) {
                    constexpr bool CHECK = decltype(check)::value;
#pragma unroll
                    for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                        for (int o1 = 0; o1 < 3; ++o1) {
                            const float wyz = st.w[1][o1] * st.w[2][o2];
                            float m0 = qs[0] + o1 * As[1] + o2 * As[2];
                            float m1 = qs[1] + o1 * As[4] + o2 * As[5];
                            float m2 = qs[2] + o1 * As[7] + o2 * As[8];
                            const int row = tb + R * o1 + Q * o2;
#pragma unroll
                            for (int o0 = 0; o0 < 3; ++o0) {
                                const float w = wyz * st.w[0][o0];
                                const int t = row + o0;
                                if (!CHECK || w >= TINY_W) {
                                    atomicAdd(&tu[t], fixed64(w * W_SCALE));
                                    atomicAdd(&tu[CT + t], fixed64(w * m0));
                                    atomicAdd(&tu[2 * CT + t], fixed64(w * m1));
                                    atomicAdd(&tu[3 * CT + t], fixed64(w * m2));
                                } else {  // rare: to the node's global accumulator, in FP32
                                    const int gx = st.base[0] + o0, gy = st.base[1] + o1, gz = st.base[2] + o2;
                                    const int bk = (((gz >> 2) + 1) * P.NB + ((gy >> 2) + 1)) * P.NB + ((gx >> 2) + 1);
                                    float* a = acc + 4 * ((int64_t)(sc.brick_base + bk) * BLOCK_NODES + (gx & 3) +
                                                          ((gy & 3) << 2) + ((gz & 3) << 4));
                                    unsafeAtomicAdd(a + 0, w * M.mp);
                                    unsafeAtomicAdd(a + 1, w * m0 * m_unit);
                                    unsafeAtomicAdd(a + 2, w * m1 * m_unit);
                                    unsafeAtomicAdd(a + 3, w * m2 * m_unit);
                                    acc_dirty[sc.brick_base + bk] = 1;
                                }
                                m0 += As[0];
                                m1 += As[3];
                                m2 += As[6];
                            }
                        }
                };
                if (any_tiny)
                    scatter(std::true_type{});
                else
                    scatter(std::false_type{});
            } else {
                if (!in_zone)
                    activate_blocks(st, P.NB, sc.brick_base, brick_state, ovf, &ctl[CTL_OVF + parity], nbricks, err);
                int xo[3], yo[3], zo[3];
                axis_offsets(st.base[0], 1, 0, xo);
                axis_offsets(st.base[1], P.NB, 2, yo);
                axis_offsets(st.base[2], P.NB * P.NB, 4, zo);
                float* accs = acc + 4 * (int64_t)sc.brick_base * BLOCK_NODES;
                {  // the stencil's nodes lie in blocks (base >> 2) + 1 and ((base + 2) >> 2) + 1 per axis
                    int* dirty = acc_dirty + sc.brick_base;
                    const int bl[3] = {(st.base[0] >> 2) + 1, (st.base[1] >> 2) + 1, (st.base[2] >> 2) + 1};
                    const int bh[3] = {((st.base[0] + 2) >> 2) + 1, ((st.base[1] + 2) >> 2) + 1,
                                       ((st.base[2] + 2) >> 2) + 1};
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        dirty[((k & 4 ? bh[2] : bl[2]) * P.NB + (k & 2 ? bh[1] : bl[1])) * P.NB + (k & 1 ? bh[0] : bl[0])] = 1;
                }
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 3; ++o1) {
                        const float wyz = st.w[1][o1] * st.w[2][o2];
                        float m0 = q[0] + o1 * Ad[1] + o2 * Ad[2];
                        float m1 = q[1] + o1 * Ad[4] + o2 * Ad[5];
                        float m2 = q[2] + o1 * Ad[7] + o2 * Ad[8];
#pragma unroll
                        for (int o0 = 0; o0 < 3; ++o0) {
                            const float w = wyz * st.w[0][o0];
                            float* a = accs + 4 * (xo[o0] + yo[o1] + zo[o2]);
                            unsafeAtomicAdd(a + 0, w * M.mp);
                            unsafeAtomicAdd(a + 1, w * m0);
                            unsafeAtomicAdd(a + 2, w * m1);
                            unsafeAtomicAdd(a + 3, w * m2);
                            m0 += Ad[0];
                            m1 += Ad[3];
                            m2 += Ad[6];
                        }
                    }
            }
        }

        // ---- store the tile to the chunk's staging slot
        if (!GLOBAL_ONLY) {
            __syncthreads();
            float4* slot = stage + off;
            const int e01 = ext[0] * ext[1];
            const float r01 = 1.0f / (float)(e01 > 0 ? e01 : 1), r0 = 1.0f / (float)(ext[0] > 0 ? ext[0] : 1);
            for (int u = tid; u < nt; u += NT) {  // staged in the tight box layout
                const int z = div_small(u, r01), u01 = u - z * e01;
                const int y = div_small(u01, r0), xx = u01 - y * ext[0];
                const int t = xx + R * y + Q * z;
                const long long* ti = reinterpret_cast<const long long*>(tq);
                const double mu = (double)m_unit;
                slot[u] = make_float4((float)((double)ti[t] * (0x1p-51 * (double)M.mp)), (float)((double)ti[CT + t] * mu),
                                      (float)((double)ti[2 * CT + t] * mu), (float)((double)ti[3 * CT + t] * mu));
#pragma unroll
                for (int ch4 = 0; ch4 < 4; ++ch4) tq[ch4 * CT + t] = 0.0;  // ready for the next chunk
            }
            __syncthreads();
        }
    }
    if constexpr (FUSED) {
        if (__ballot(left) != 0ull && (threadIdx.x & 63) == 0) {
            if (__hip_atomic_load(&ctl[CTL_REBUILD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                atomicExch(&ctl[CTL_REBUILD], 1) == 0 && host_flag)
                __hip_atomic_store(host_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl[CTL_STEP] += 1;  // the G2P part completed a substep
    }
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
    if (SURM != 0 && (threadIdx.x & 63) == 0) {
        unsigned long long* c64 = ctl64(ctl, blockIdx.x * (NT / 64) + (threadIdx.x >> 6));
        if (n_sur) atomicAdd(&c64[CTL64_SUR_PARTICLES], (unsigned long long)n_sur);
        if (n_fb) atomicAdd(&c64[CTL64_SUR_FALLBACKS], (unsigned long long)n_fb);
    }
}


// Land the deferred deformation update of every particle with its scene's
// snow map -- exact, closed form (no SVD) or the network -- the way P2G
// applies it, for contexts where some snow scene takes a map without SVD.
// One chunk per workgroup pass (a chunk holds one scene, so the network runs
// on whole waves of one scene).
template <int SURM, int NT>
__global__ __launch_bounds__(NT) void k_materialize_map(float* __restrict__ S, int64_t cap,
                                                        const Chunk* __restrict__ chunks, const int* __restrict__ ctl,
                                                        Scenes T) {
    struct Empty {};
    __shared__ typename std::conditional<SURM == 2, mlp::NetLds16, Empty>::type net;
    __shared__ __attribute__((aligned(16))) float sur_stage[SURM == 2 ? NT / 64 * mlp::FWD_STAGE : 1];
    if constexpr (SURM == 2) {
        if (T.sur_theta) mlp::load_net16(net, T.sur_theta, T.sur_norm);
        __syncthreads();
    }
    const int nchunk = ctl[CTL_NCHUNK];
    const int tid = threadIdx.x, wv = tid >> 6;
    for (int c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const Chunk ch = chunks[c];
        const Scene& sc = T.scene[ch.scene];
        const Mat M = sc.M;
        const bool have = tid < ch.count;
        const int p = ch.start + (have ? tid : 0);
        float C[9], F[9], s = 1.0f, tau[6];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            C[k] = have ? S[sidx(FC + k, p, cap)] : 0.0f;
            F[k] = have ? S[sidx(FF + k, p, cap)] : ((k % 4 == 0) ? 1.0f : 0.0f);
        }
        if (have) s = S[sidx(FS, p, cap)];
        bool fb = false;
        if (sc.ret != 0 && M.kind == MPM_SNOW) {  // uniform over the workgroup
            if constexpr (SURM == 2) {
                if (sc.ret == 1)
                    snow_without_svd<true>(&net, sur_stage + wv * mlp::FWD_STAGE, T, sc, sc.P.dt, 1, have, C, F, s, tau, fb);
                else
                    snow_without_svd<false>(&net, sur_stage, T, sc, sc.P.dt, 1, have, C, F, s, tau, fb);
            } else {
                snow_without_svd<false>(nullptr, nullptr, T, sc, sc.P.dt, 1, have, C, F, s, tau, fb);
            }
        } else if (have) {
            material_step(M, sc.P.dt, 1, C, F, s, tau);
        }
        if (have) {
            if (M.kind != MPM_WATER) {
#pragma unroll
                for (int k = 0; k < 9; ++k) S[sidx(FF + k, p, cap)] = F[k];
            }
            if (M.kind != MPM_JELLY) S[sidx(FS, p, cap)] = s;
        }
    }
}

#define MPM_P2G_PARAMS                                                                                          \
    float *__restrict__ S, int64_t cap, const Chunk *__restrict__ chunks, int *__restrict__ ctl,               \
        float *__restrict__ acc, int *__restrict__ acc_dirty, float4 *__restrict__ stage, int stage_nodes,     \
        int4 *__restrict__ box,                                                                                 \
        int *__restrict__ brick_state, int *__restrict__ ovf, int parity, Scenes T, int pending, int nbricks, \
        int act, const float4 *__restrict__ vel, int *__restrict__ host_flag, int fb_limit
#define MPM_P2G_ARGS \
    S, cap, chunks, ctl, acc, acc_dirty, stage, stage_nodes, box, brick_state, ovf, parity, T, pending, nbricks, act, vel, \
        host_flag, fb_limit

template <bool GLOBAL_ONLY, int NT, int SURM>
__global__ __launch_bounds__(NT) void k_p2g(MPM_P2G_PARAMS) {
    p2g_body<GLOBAL_ONLY, NT, SURM, false>(MPM_P2G_ARGS);
}

// The fused form holds the gathered v and C beside the P2G state; four
// waves per SIMD (at most 128 VGPRs) keep it as resident as the plain form.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_p2g_fused(MPM_P2G_PARAMS) {
    p2g_body<false, NT, 0, true>(MPM_P2G_ARGS);
}

#undef MPM_P2G_PARAMS
#undef MPM_P2G_ARGS

}  // namespace

int p2g_grid_size(int cus, int chunk) {
    const int nt = chunk_threads(chunk);
    const void* fn = nt == 128   ? reinterpret_cast<const void*>(k_p2g<false, 128, 0>)
                     : nt == 256 ? reinterpret_cast<const void*>(k_p2g<false, 256, 0>)
                                 : reinterpret_cast<const void*>(k_p2g<false, 512, 0>);
    // Four times the resident workgroups (at most 4096 threads per CU): the
    // chunks of the block-sorted list differ in cost (fill, box size), and
    // with each workgroup taking every stride-th chunk of its XCD's slice,
    // more and shorter-lived workgroups even the load out (twice the
    // resident count: 146.6 us, four times: 140.9 us per launch on the
    // 1.28M-particle snow scene, frames 2-40).
    int occ = 4 * wgs_per_cu(fn, nt);
    if (occ > 4096 / nt) occ = 4096 / nt;
    const int g = cus * occ;
    return g < 8 ? 8 : (g / 8) * 8;
}

void enqueue_p2g(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap, const Chunk* chunks,
                 int* ctl, GridBuffers& G, int* brick_state, int pending, int parity, int global_atomics,
                 int nbricks, int chunk, int act, int fused, int* host_flag, int fb_limit) {
    const int nt = chunk_threads(chunk);
    const int surm = T.sur_any;  // 0, 1 (closed form) or 2 (network)
    auto launch = [&](auto kernel, int threads) {
        hipLaunchKernelGGL(kernel, dim3(L.p2g_grid), dim3(threads), 0, st, S, cap, chunks, ctl, G.acc, G.acc_dirty, G.stage,
                           G.stage_nodes, G.box, brick_state, G.ovf[parity], parity, T, pending, nbricks, act, G.vel,
                           host_flag, fb_limit);
    };
#define MPM_LAUNCH_P2G_NT(GO, SU)                                                              \
    do {                                                                                       \
        if (nt == 128) launch(k_p2g<GO, 128, SU>, 128);                                        \
        else if (nt == 256) launch(k_p2g<GO, 256, SU>, 256);                                   \
        else launch(k_p2g<GO, 512, SU>, 512);                                                  \
    } while (0)
    if (fused) {  // callers check: tile path, exact map
        if (nt == 128) launch(k_p2g_fused<128>, 128); else if (nt == 256) launch(k_p2g_fused<256>, 256); else launch(k_p2g_fused<512>, 512);
    } else if (global_atomics) {
        if (surm == 2) MPM_LAUNCH_P2G_NT(true, 2); else if (surm == 1) MPM_LAUNCH_P2G_NT(true, 1); else MPM_LAUNCH_P2G_NT(true, 0);
    } else {
        if (surm == 2) MPM_LAUNCH_P2G_NT(false, 2); else if (surm == 1) MPM_LAUNCH_P2G_NT(false, 1); else MPM_LAUNCH_P2G_NT(false, 0);
    }
#undef MPM_LAUNCH_P2G_NT
}

void enqueue_materialize_map(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap,
                             const Chunk* chunks, const int* ctl, int chunk) {
    const int nt = chunk_threads(chunk);
    const int grid = L.p2g_grid;
#define MPM_LAUNCH_MAT(SU)                                                                                        \
    do {                                                                                                          \
        if (nt == 128) hipLaunchKernelGGL((k_materialize_map<SU, 128>), dim3(grid), dim3(128), 0, st, S, cap, chunks, ctl, T); \
        else if (nt == 256) hipLaunchKernelGGL((k_materialize_map<SU, 256>), dim3(grid), dim3(256), 0, st, S, cap, chunks, ctl, T); \
        else hipLaunchKernelGGL((k_materialize_map<SU, 512>), dim3(grid), dim3(512), 0, st, S, cap, chunks, ctl, T); \
    } while (0)
    if (T.sur_any == 2) MPM_LAUNCH_MAT(2); else MPM_LAUNCH_MAT(1);
#undef MPM_LAUNCH_MAT
}

}  // namespace mpm
