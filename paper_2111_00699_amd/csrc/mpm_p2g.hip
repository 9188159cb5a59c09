// P2G on gfx950: particle-to-grid transfer with the deferred deformation
// update, the snow return map and the Kirchhoff stress fused in (paper,
// "Merge Kernels": plasticity, SVD and stress computed inside P2G).
//
// Avoiding non-native intrinsics ("Avoid non-native intrinsics"): on V100
// the paper drops shared-memory float atomics because they are emulated.
// On gfx950 ds_add_f32 exists but runs at about 0.3 lane-ops per clock per
// CU, while ds_add_f64 runs at about 6.6, and global float atomics (about
// 0.4, executed memory-side) move a full write per update.  The same
// principle -- use only the fast native operations -- leads here to:
//   * a workgroup takes one chunk (<= 256 or 512 particles of one particle
//     block), one particle per thread, loads coalesced;
//   * phase 1 computes every particle's contribution and the bounding box of
//     the stencils of the chunk's in-zone particles (block reduction);
//   * the tile is that box (at most 512 nodes; a particle block's stencils
//     cover 6^3 = 216 nodes right after a rebuild), four FP64 channels
//     (weight sum and three momentum components) accumulated with
//     ds_add_f64;
//   * the tile is then STORED (plain, coalesced float4 stores) to the
//     staging buffer, and the grid update gathers each node from the tiles
//     of the particle blocks around it -- no global atomics, and the
//     transfer of in-zone particles is deterministic.  Each workgroup owns an
//     equal slice of the staging buffer and packs its chunks' tiles there
//     (offset recorded per chunk), so no allocation is shared.
// The rebuild stores each chunk with its sorted order spread by a stride
// coprime to the count, so the 64 lanes of a wave sit in different cells
// and rarely hit one LDS address (same-address atomics serialize).
// Particles outside their free zone (before a late rebuild) scatter straight
// to global atomics and activate the blocks they touch.
#include "mpm_kernels.h"

namespace mpm {

namespace {

constexpr int CT = 512;  // compact tile capacity in nodes

// NT threads per workgroup = the largest chunk it takes (256 or 512).
template <bool GLOBAL_ONLY, int NT>
__global__ __launch_bounds__(NT) void k_p2g(float* __restrict__ S, int64_t cap, const Chunk* __restrict__ chunks,
                                            int* __restrict__ ctl, float* __restrict__ acc,
                                            float4* __restrict__ stage, int stage_nodes, int4* __restrict__ box,
                                            int* __restrict__ brick_state, int* __restrict__ ovf, int parity, Step P,
                                            Mat M, int pending, int nbricks) {
    __shared__ double tq[GLOBAL_ONLY ? 1 : 4 * CT];
    __shared__ int red_i[6][NT / 64];
    unsigned err = 0;
    int begin, end, stride;
    xcd_split(ctl[CTL_NCHUNK], begin, end, stride);
    const float dx = P.dx, dt = P.dt;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // this workgroup's slice of the staging buffer, filled front to back
    const int slice = (int)((int64_t)stage_nodes / gridDim.x);
    const int slice0 = slice * (int)blockIdx.x;
    int used = 0;
    for (int c = begin; c < end; c += stride) {
        const Chunk ch = chunks[c];
        const int count = ch.count;
        const int B[3] = {ch.block & 1023, (ch.block >> 10) & 1023, ch.block >> 20};
        const bool have = tid < count;
        const int p = ch.start + (have ? tid : 0);

        // ---- phase 1: material update, stress and this particle's payload
        Stencil st;
        float q[3] = {0.f, 0.f, 0.f}, Ad[9];
        bool ok = false, in_zone = false;
        if (have) {
            float x[3], v[3], C[9], F[9], s;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                x[a] = S[(FX + a) * cap + p];
                v[a] = S[(FV + a) * cap + p];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) C[k] = S[(FC + k) * cap + p];
            s = S[FS * cap + p];
            if (M.kind != MPM_WATER) {
#pragma unroll
                for (int k = 0; k < 9; ++k) F[k] = S[(FF + k) * cap + p];
            }
            float tau[6];
            material_step(M, dt, pending, C, F, s, tau);
            if (pending) {  // the deferred update of the last G2P lands here
                if (M.kind != MPM_WATER) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) S[(FF + k) * cap + p] = F[k];
                }
                if (M.kind != MPM_JELLY) S[FS * cap + p] = s;
            }
            ok = make_stencil(x, P, st, err);
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
        int nt = 0, off = 0;
        if (GLOBAL_ONLY && tid == 0) box[c] = make_int4(0, 0, 0, 0);
        if (!GLOBAL_ONLY) {
            const bool tiled = have && in_zone;
            int mn[3], mx[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = wave_min(tiled ? st.base[a] : INT_MAX);
                mx[a] = wave_max(tiled ? st.base[a] + 2 : INT_MIN);
            }
            if (lane == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    red_i[a][wv] = mn[a];
                    red_i[3 + a][wv] = mx[a];
                }
            }
            __syncthreads();
            int hi[3];
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
            }
            if (hi[0] >= lo[0]) {
#pragma unroll
                for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a] + 1;
                nt = ext[0] * ext[1] * ext[2];
            }
            // no room in the tile or in this workgroup's staging slice: the chunk goes to global atomics
            if (nt > CT || used + nt > slice) nt = -1;
            if (nt < 0 && tid == 0) atomicAdd(&ctl64(ctl)[CTL64_FALLBACK_CHUNKS], 1ull);
            off = slice0 + used;
            if (nt > 0) used += nt;
            for (int t = tid; t < nt; t += NT) {
#pragma unroll
                for (int ch4 = 0; ch4 < 4; ++ch4) tq[ch4 * CT + t] = 0.0;
            }
            if (tid == 0)
                box[c] = nt > 0 ? make_int4(lo[0] | (lo[1] << 10) | (lo[2] << 20), ext[0] | (ext[1] << 8) | (ext[2] << 16),
                                            off, 0)
                                : make_int4(0, 0, 0, 0);
            __syncthreads();
        }

        // ---- phase 2: scatter
        {
            const unsigned long long g = __ballot(have && ok && (GLOBAL_ONLY || !in_zone || nt <= 0));
            if (g && lane == 0) atomicAdd(&ctl64(ctl)[CTL64_GLOBAL_PARTICLES], (unsigned long long)__popcll(g));
            // in-zone particles that lost the tile: a rebuild would shrink their chunk's box again
            const unsigned long long fb = __ballot(have && ok && !GLOBAL_ONLY && in_zone && nt <= 0);
            if (fb && lane == 0) atomicAdd(&ctl[CTL_FB + parity], (int)__popcll(fb));
        }
        if (have && ok) {
            if (!GLOBAL_ONLY && in_zone && nt > 0) {
                const int tb = (st.base[0] - lo[0]) + ext[0] * ((st.base[1] - lo[1]) + ext[1] * (st.base[2] - lo[2]));
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 3; ++o1) {
                        const float wyz = st.w[1][o1] * st.w[2][o2];
                        float m0 = q[0] + o1 * Ad[1] + o2 * Ad[2];
                        float m1 = q[1] + o1 * Ad[4] + o2 * Ad[5];
                        float m2 = q[2] + o1 * Ad[7] + o2 * Ad[8];
                        const int row = tb + ext[0] * (o1 + ext[1] * o2);
#pragma unroll
                        for (int o0 = 0; o0 < 3; ++o0) {
                            const float w = wyz * st.w[0][o0];
                            const int t = row + o0;
                            atomicAdd(&tq[t], (double)w);
                            atomicAdd(&tq[CT + t], (double)(w * m0));
                            atomicAdd(&tq[2 * CT + t], (double)(w * m1));
                            atomicAdd(&tq[3 * CT + t], (double)(w * m2));
                            m0 += Ad[0];
                            m1 += Ad[3];
                            m2 += Ad[6];
                        }
                    }
            } else {
                if (!in_zone) activate_blocks(st, P, brick_state, ovf, &ctl[CTL_OVF + parity], nbricks, err);
                int xo[3], yo[3], zo[3];
                axis_offsets(st.base[0], 1, 0, xo);
                axis_offsets(st.base[1], P.NB, 2, yo);
                axis_offsets(st.base[2], P.NB * P.NB, 4, zo);
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
                            float* a = acc + 4 * (xo[o0] + yo[o1] + zo[o2]);
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
            for (int t = tid; t < nt; t += NT)
                slot[t] = make_float4((float)(tq[t] * (double)M.mp), (float)tq[CT + t], (float)tq[2 * CT + t],
                                      (float)tq[3 * CT + t]);
            __syncthreads();
        }
    }
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
}

}  // namespace

int p2g_grid_size(int cus, int chunk) {
    const int nt = chunk_threads(chunk);
    const void* fn = nt == 128   ? reinterpret_cast<const void*>(k_p2g<false, 128>)
                     : nt == 256 ? reinterpret_cast<const void*>(k_p2g<false, 256>)
                                 : reinterpret_cast<const void*>(k_p2g<false, 512>);
    // Twice the resident workgroups: chunks differ in size, and a second wave
    // of workgroups evens out the per-XCD work split.
    int occ = 2 * wgs_per_cu(fn, nt);
    if (occ > 4096 / nt) occ = 4096 / nt;
    const int g = cus * occ;
    return g < 8 ? 8 : (g / 8) * 8;
}

void enqueue_p2g(hipStream_t st, const Launch& L, const Step& P, const Mat& M, float* S, int64_t cap,
                 const Chunk* chunks, int* ctl, GridBuffers& G, int* brick_state, int pending, int parity,
                 int global_atomics, int nbricks, int chunk) {
#define MPM_LAUNCH_P2G(GO, T)                                                                                \
    hipLaunchKernelGGL((k_p2g<GO, T>), dim3(L.p2g_grid), dim3(T), 0, st, S, cap, chunks, ctl, G.acc, G.stage, \
                       G.stage_nodes, G.box, brick_state, G.ovf[parity], parity, P, M, pending, nbricks)
    const int nt = chunk_threads(chunk);
    if (nt == 128) {
        if (global_atomics) MPM_LAUNCH_P2G(true, 128); else MPM_LAUNCH_P2G(false, 128);
    } else if (nt == 256) {
        if (global_atomics) MPM_LAUNCH_P2G(true, 256); else MPM_LAUNCH_P2G(false, 256);
    } else {
        if (global_atomics) MPM_LAUNCH_P2G(true, 512); else MPM_LAUNCH_P2G(false, 512);
    }
#undef MPM_LAUNCH_P2G
}

}  // namespace mpm
