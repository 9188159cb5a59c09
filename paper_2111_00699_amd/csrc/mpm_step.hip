// Grid update (boundary conditions and clearing of the accumulators fused
// in) and G2P (with the free-zone test fused in) of an explicit MPM substep
// on gfx950, plus the particle insert/read/materialize utilities.  Paper,
// "Material Point Method on a Single GPU" and "Merge Kernels".  P2G lives in
// mpm_p2g.hip.
//
// MI355X design:
//  * Particles are processed in chunks that share one particle block, so
//    every particle of a chunk inside its free zone scatters into the same
//    12^3-node tile (the 3x3x3 physical blocks of the "Rebuild-Mapping"
//    subsection).  The tile lives in LDS and takes native ds_add_f32
//    atomics; only its non-empty nodes are flushed with native
//    global_atomic_add_f32.  (The paper drops shared memory on V100 because
//    float atomics there are emulated with CAS loops; on gfx950 both LDS and
//    global float adds are native, so the same principle -- use only native
//    atomics -- leads to an LDS tile.)
//  * Chunks are dealt to the eight XCDs in contiguous ranges of the
//    block-sorted order so each XCD's L2 sees a compact region of the grid.
//  * The grid is a dense array of 4^3-node blocks over the padded domain; a
//    particle that has left its free zone before the next rebuild scatters
//    straight to global atomics and activates the blocks it touches, so a
//    late rebuild never costs correctness.
#include "mpm_kernels.h"

namespace mpm {

namespace {

// ----------------------------------------------------------- grid update
// One wave64 per 4^3 block: v = p/m + dt g where m > 0 (else 0), then the
// wall condition; writes (v, m), clears the accumulators, and stamps the block.
__global__ __launch_bounds__(WG) void k_grid(float* __restrict__ acc, float4* __restrict__ vel,
                                             const int* __restrict__ active, int* __restrict__ ctl,
                                             const int* __restrict__ ovf, int* __restrict__ brick_state,
                                             int* __restrict__ stamp, int parity, int step, int nbricks, Step P) {
    const int nact = ctl[CTL_NACTIVE];
    const int total = nact + min(ctl[CTL_OVF + parity], nbricks - nact);
    const int lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int nwaves = gridDim.x * (WG / 64);
    float4* acc4 = reinterpret_cast<float4*>(acc);
    for (int it = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); it < total; it += nwaves) {
        const int b = it < nact ? active[it] : ovf[it - nact];
        const int bx = b % P.NB, by = (b / P.NB) % P.NB, bz = b / (P.NB * P.NB);
        const int g[3] = {4 * (bx - 1) + lx, 4 * (by - 1) + ly, 4 * (bz - 1) + lz};
        const float4 a = acc4[b * 64 + lane];
        float v[3] = {0.0f, 0.0f, 0.0f};
        if (a.x > 0.0f) {
            const float inv = 1.0f / a.x;
            v[0] = a.y * inv + P.dt * P.g0;
            v[1] = a.z * inv + P.dt * P.g1;
            v[2] = a.w * inv + P.dt * P.g2;
        }
        bool any = false;
        bool lowside[3], highside[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lowside[k] = g[k] < P.bc_cells;
            highside[k] = g[k] > P.n - P.bc_cells;
            any = any || lowside[k] || highside[k];
        }
        if (any) {
            if (P.bc == MPM_BC_STICKY) {
                v[0] = v[1] = v[2] = 0.0f;
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (P.bc == MPM_BC_SLIP) {
                        if (lowside[k] || highside[k]) v[k] = 0.0f;
                    } else {
                        if (lowside[k] && v[k] < 0.0f) v[k] = 0.0f;
                        if (highside[k] && v[k] > 0.0f) v[k] = 0.0f;
                    }
                }
            }
        }
        vel[b * 64 + lane] = make_float4(v[0], v[1], v[2], a.x);
        acc4[b * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane == 0) {
            stamp[b] = step;
            if (it >= nact) brick_state[b] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[CTL_OVF + (parity ^ 1)] = 0;
}

// -------------------------------------------------------------------- G2P
__global__ __launch_bounds__(WG) void k_g2p(float* __restrict__ S, int64_t cap, const Chunk* __restrict__ chunks,
                                            int* __restrict__ ctl, const float4* __restrict__ vel,
                                            int* __restrict__ host_flag, Step P) {
    unsigned err = 0;
    bool left = false;
    int begin, end, stride;
    xcd_split(ctl[CTL_NCHUNK], begin, end, stride);
    const float c4 = 4.0f * P.fn;  // (4/dx^2) * dx
    for (int c = begin; c < end; c += stride) {
        const Chunk ch = chunks[c];
        const int B[3] = {ch.block & 1023, (ch.block >> 10) & 1023, ch.block >> 20};
        for (int i = threadIdx.x; i < ch.count; i += WG) {
            const int p = ch.start + i;
            float x[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) x[a] = S[(FX + a) * cap + p];
            Stencil st;
            if (!make_stencil(x, P, st, err)) continue;
            int xo[3], yo[3], zo[3];
            axis_offsets(st.base[0], 1, 0, xo);
            axis_offsets(st.base[1], P.NB, 2, yo);
            axis_offsets(st.base[2], P.NB * P.NB, 4, zo);
            float vp[3] = {0, 0, 0};
            float Mo[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // sum w v_a o_b
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                for (int o1 = 0; o1 < 3; ++o1) {
                    const float wyz = st.w[1][o1] * st.w[2][o2];
#pragma unroll
                    for (int o0 = 0; o0 < 3; ++o0) {
                        const float w = wyz * st.w[0][o0];
                        const float4 g = vel[xo[o0] + yo[o1] + zo[o2]];
                        const float wv[3] = {w * g.x, w * g.y, w * g.z};
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            vp[a] += wv[a];
                            Mo[a * 3 + 0] += o0 * wv[a];
                            Mo[a * 3 + 1] += o1 * wv[a];
                            Mo[a * 3 + 2] += o2 * wv[a];
                        }
                    }
                }
            // C' = 4/dx^2 sum w v (x_i - x_p)^T = (4/dx) (Mo - v' f^T)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) S[(FC + a * 3 + b) * cap + p] = c4 * (Mo[a * 3 + b] - vp[a] * st.f[b]);
            bool fin = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float xn = x[a] + P.dt * vp[a];
                S[(FV + a) * cap + p] = vp[a];
                S[(FX + a) * cap + p] = xn;
                fin = fin && (fabsf(xn) < 1e30f) && (fabsf(vp[a]) < 1e30f);
                // free zone: the cell code must stay within [4B-3, 4B+6]
                const float cc = floorf(xn * P.fn - 0.5f) + 1.0f;
                left = left || !(cc >= (float)(4 * B[a] - 3) && cc <= (float)(4 * B[a] + 6));
            }
            if (!fin) err |= MPM_ERR_NONFINITE;
        }
    }
    if (__ballot(left) != 0ull && (threadIdx.x & 63) == 0) {
        if (__hip_atomic_load(&ctl[CTL_REBUILD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
            atomicExch(&ctl[CTL_REBUILD], 1) == 0)
            __hip_atomic_store(host_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
}

// ------------------------------------------------------------- utilities
__global__ __launch_bounds__(WG) void k_materialize(float* __restrict__ S, int64_t cap, int N, Step P, Mat M) {
    const int p = blockIdx.x * WG + threadIdx.x;
    if (p >= N) return;
    float C[9], F[9], s, tau[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        C[k] = S[(FC + k) * cap + p];
        F[k] = S[(FF + k) * cap + p];
    }
    s = S[FS * cap + p];
    material_step(M, P.dt, 1, C, F, s, tau);
#pragma unroll
    for (int k = 0; k < 9; ++k) S[(FF + k) * cap + p] = F[k];
    S[FS * cap + p] = s;
}

__global__ __launch_bounds__(WG) void k_insert(float* __restrict__ S, int* __restrict__ ids, int64_t cap, int N0,
                                               int count, const float* __restrict__ x, const float* __restrict__ v,
                                               const float* __restrict__ C, const float* __restrict__ F,
                                               const float* __restrict__ s, int* __restrict__ ctl) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= count) return;
    const int j = N0 + i;
    unsigned err = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float xa = x[a * (int64_t)count + i];
        if (!(fabsf(xa) < 1e30f)) err |= MPM_ERR_NONFINITE;
        else if (!(xa >= 0.0f && xa <= 1.0f)) err |= MPM_ERR_DOMAIN;
        S[(FX + a) * cap + j] = xa;
        S[(FV + a) * cap + j] = v ? v[a * (int64_t)count + i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        S[(FC + k) * cap + j] = C ? C[k * (int64_t)count + i] : 0.0f;
        S[(FF + k) * cap + j] = F ? F[k * (int64_t)count + i] : ((k % 4 == 0) ? 1.0f : 0.0f);
    }
    S[FS * cap + j] = s ? s[i] : 1.0f;
    ids[j] = j;
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
}

__global__ __launch_bounds__(WG) void k_read(const float* __restrict__ S, const int* __restrict__ ids, int64_t cap,
                                             int N, int pending, Step P, Mat M, float* __restrict__ x,
                                             float* __restrict__ v, float* __restrict__ C, float* __restrict__ F,
                                             float* __restrict__ s) {
    const int j = blockIdx.x * WG + threadIdx.x;
    if (j >= N) return;
    const int64_t id = ids[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (x) x[a * (int64_t)N + id] = S[(FX + a) * cap + j];
        if (v) v[a * (int64_t)N + id] = S[(FV + a) * cap + j];
    }
    float Cp[9], Fp[9], sp = S[FS * cap + j], tau[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Cp[k] = S[(FC + k) * cap + j];
        Fp[k] = S[(FF + k) * cap + j];
        if (C) C[k * (int64_t)N + id] = Cp[k];
    }
    if (pending && (F || s)) material_step(M, P.dt, 1, Cp, Fp, sp, tau);
    if (F)
#pragma unroll
        for (int k = 0; k < 9; ++k) F[k * (int64_t)N + id] = Fp[k];
    if (s) s[id] = sp;
}

__global__ __launch_bounds__(WG) void k_read_grid(const float4* __restrict__ vel, const int* __restrict__ stamp,
                                                  int step, Step P, float* __restrict__ m, float* __restrict__ v) {
    const int n1 = P.n + 1;
    const int64_t NN = (int64_t)n1 * n1 * n1;
    const int64_t id = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (id >= NN) return;
    const int i = (int)(id / ((int64_t)n1 * n1)), j = (int)((id / n1) % n1), k = (int)(id % n1);
    const int b = (((k >> 2) + 1) * P.NB + ((j >> 2) + 1)) * P.NB + ((i >> 2) + 1);
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (stamp[b] == step) g = vel[b * 64 + (i & 3) + ((j & 3) << 2) + ((k & 3) << 4)];
    if (m) m[id] = g.w;
    if (v) {
        v[id] = g.x;
        v[NN + id] = g.y;
        v[2 * NN + id] = g.z;
    }
}

}  // namespace

void query_launch(Launch& L) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&L.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (L.cus <= 0) L.cus = 256;
    auto grid_for = [&](const void* fn, int cap_per_cu) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, WG, 0) != hipSuccess || occ <= 0) occ = 2;
        occ = occ > cap_per_cu ? cap_per_cu : occ;
        int g = L.cus * occ;
        return g < 8 ? 8 : (g / 8) * 8;
    };
    L.p2g_grid = p2g_grid_size(L.cus);
    L.g2p_grid = grid_for(reinterpret_cast<const void*>(k_g2p), 8);
    L.grid_grid = grid_for(reinterpret_cast<const void*>(k_grid), 8);
}

void enqueue_grid(hipStream_t st, const Launch& L, const Step& P, const int* active, int* ctl, GridBuffers& G,
                  int* brick_state, int parity, int step) {
    hipLaunchKernelGGL(k_grid, dim3(L.grid_grid), dim3(WG), 0, st, G.acc, G.vel, active, ctl, G.ovf[parity],
                       brick_state, G.stamp, parity, step, P.NB * P.NB * P.NB, P);
}

void enqueue_g2p(hipStream_t st, const Launch& L, const Step& P, float* S, int64_t cap, const Chunk* chunks, int* ctl,
                 const GridBuffers& G, int* host_flag) {
    hipLaunchKernelGGL(k_g2p, dim3(L.g2p_grid), dim3(WG), 0, st, S, cap, chunks, ctl, G.vel, host_flag, P);
}

void enqueue_materialize(hipStream_t st, const Step& P, const Mat& M, float* S, int64_t cap, int N) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_materialize, dim3(cdiv(N, WG)), dim3(WG), 0, st, S, cap, N, P, M);
}

void enqueue_insert(hipStream_t st, float* S, int* ids, int64_t cap, int N0, int count, const float* x, const float* v,
                    const float* C, const float* F, const float* s, int* ctl) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_insert, dim3(cdiv(count, WG)), dim3(WG), 0, st, S, ids, cap, N0, count, x, v, C, F, s, ctl);
}

void enqueue_read(hipStream_t st, const Step& P, const Mat& M, const float* S, const int* ids, int64_t cap, int N,
                  int pending, float* x, float* v, float* C, float* F, float* s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_read, dim3(cdiv(N, WG)), dim3(WG), 0, st, S, ids, cap, N, pending, P, M, x, v, C, F, s);
}

void enqueue_read_grid(hipStream_t st, const Step& P, const GridBuffers& G, int step, float* m, float* v) {
    const int64_t n1 = P.n + 1;
    hipLaunchKernelGGL(k_read_grid, dim3(cdiv(n1 * n1 * n1, WG)), dim3(WG), 0, st, G.vel, G.stamp, step, P, m, v);
}

}  // namespace mpm
