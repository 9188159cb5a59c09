// Grid update (boundary conditions and clearing of the accumulators fused
// in) and G2P (with the free-zone test fused in) of an explicit MPM substep
// on gfx950, plus the particle insert/read/materialize utilities.  Paper,
// "Material Point Method on a Single GPU" and "Merge Kernels".  P2G lives in
// mpm_p2g.hip.
//
// MI355X design:
//  * The grid update is one wave64 per 4^3 block of the physical (and
//    overflow) block lists.  It gathers each node from the tiles (exact
//    fixed-point sums, stored as FP32) that P2G staged for the chunks of the
//    27 particle blocks around it (no global atomics on the tiled path), adds
//    the global-path accumulator, then applies gravity and the wall
//    condition and clears the accumulator.  A wave's blocks are pipelined:
//    the next block's registrations and tile boxes load while the current
//    block gathers.
//  * G2P takes one chunk per workgroup and loads the chunk's node box (the
//    box its P2G tile used) into LDS, so the 27-node gathers read LDS.
//  * Work lists are dealt to the eight XCDs in contiguous ranges of the
//    block-sorted order so each XCD's L2 sees a compact region of the grid.
//  * The grid is a dense array of 4^3-node blocks per scene; a particle
//    that has left its free zone before the next rebuild scatters straight
//    to global atomics and activates the blocks it touches, so a late
//    rebuild never costs correctness.
//  * Every kernel reads its scene's grid, time step and material from the
//    scene table, and a substep may run only the first `act` ranks.
#include "mpm_kernels.h"

namespace mpm {

namespace {

// ----------------------------------------------------------- grid update
// One wave64 per 4^3 block.  Each node sums the global-path accumulator and
// the staged P2G tiles of the chunks registered with its block at the
// rebuild whose box (this substep's) holds the node, in chunk order, then
// v = p/m + dt g where m > 0 (else 0) and the wall condition; writes (v, m),
// clears the accumulator, and stamps the block.
// The wall condition on a node's velocity (lowside/highside: the node lies
// in the low/high wall layer of each axis).
__device__ __forceinline__ void wall_condition(const Step& P, const bool lowside[3], const bool highside[3],
                                               float v[3]) {
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

// The grid update's block list: the physical blocks of the last rebuild and
// this substep's overflow blocks; f(b, it, node coordinates, scene) per wave
// and block.
template <class Fn>
__device__ __forceinline__ void for_grid_blocks(const int* active, const int* ctl, const int* ovf, int parity,
                                                int nbricks, const Scenes& T, int act, Fn f) {
    const int nact = rank_limit(T, ctl, act, RE_ACTIVE, CTL_NACTIVE);
    const int total = nact + min(ctl[CTL_OVF + parity], nbricks - ctl[CTL_NACTIVE]);
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (WG / 64);
    for (int it = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); it < total; it += nwaves) {
        const int b = __builtin_amdgcn_readfirstlane(it < nact ? active[it] : ovf[it - nact]);
        const Scene& sc = T.scene[T.rank_scene[rank_of_brick(T, b)]];
        const int NB = sc.P.NB, lb = b - sc.brick_base;
        const int bx = lb % NB, by = (lb / NB) % NB, bz = lb / (NB * NB);
        const int g[3] = {4 * (bx - 1) + (lane & 3), 4 * (by - 1) + ((lane >> 2) & 3), 4 * (bz - 1) + (lane >> 4)};
        f(b, it < nact, g, sc);
    }
}

// The wall condition as a launch of its own, after k_grid<false, ...>.
__global__ __launch_bounds__(WG) void k_grid_walls(float4* __restrict__ vel, float4* __restrict__ dvel,
                                                   const int* __restrict__ active, const int* __restrict__ ctl,
                                                   const int* __restrict__ ovf, int parity, int nbricks, Scenes T,
                                                   int act) {
    const int lane = threadIdx.x & 63;
    for_grid_blocks(active, ctl, ovf, parity, nbricks, T, act, [&](int b, bool, const int g[3], const Scene& sc) {
        const Step P = sc.P;
        bool any = false, lowside[3], highside[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lowside[k] = g[k] < P.bc_cells;
            highside[k] = g[k] > P.n - P.bc_cells;
            any = any || lowside[k] || highside[k];
        }
        if (!any) return;
        float4 u = vel[(int64_t)b * 64 + lane];
        float v[3] = {u.x, u.y, u.z};
        wall_condition(P, lowside, highside, v);
        vel[(int64_t)b * 64 + lane] = make_float4(v[0], v[1], v[2], u.w);
        if (P.flip > 0.0f) {  // keep the ASFLIP grid change consistent with the walls
            float4 d = dvel[(int64_t)b * 64 + lane];
            d.x += v[0] - u.x;
            d.y += v[1] - u.y;
            d.z += v[2] - u.z;
            if (u.w > 0.0f) dvel[(int64_t)b * 64 + lane] = d;
        }
    });
}

// The clearing of the global accumulators as a launch of its own, after
// k_grid<..., false>.
__global__ __launch_bounds__(WG) void k_grid_clear(float* __restrict__ acc, int* __restrict__ acc_dirty,
                                                   const int* __restrict__ active, const int* __restrict__ ctl,
                                                   const int* __restrict__ ovf, int* __restrict__ brick_state,
                                                   int parity, int nbricks, Scenes T, int act) {
    const int lane = threadIdx.x & 63;
    float4* acc4 = reinterpret_cast<float4*>(acc);
    for_grid_blocks(active, ctl, ovf, parity, nbricks, T, act, [&](int b, bool physical, const int*, const Scene&) {
        if (__builtin_amdgcn_readfirstlane(acc_dirty[b]) != 0) {
            acc4[(int64_t)b * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (lane == 0) acc_dirty[b] = 0;
        }
        if (lane == 0 && !physical) brick_state[b] = 0;
    });
}

// BC and CLEAR false (the kernel-merging ablations): the wall condition, or
// the clearing of the global accumulators, is left to a launch of its own
// (k_grid_walls, k_grid_clear).
template <bool BC, bool CLEAR>
__global__ __launch_bounds__(WG) void k_grid(float* __restrict__ acc, int* __restrict__ acc_dirty,
                                             float4* __restrict__ vel, float4* __restrict__ dvel,
                                             const int* __restrict__ active, int* __restrict__ ctl,
                                             const int* __restrict__ ovf, int* __restrict__ brick_state,
                                             int* __restrict__ stamp, const int* __restrict__ reg_n,
                                             const int* __restrict__ reg, const float4* __restrict__ stage,
                                             int zero_node, const int4* __restrict__ box, int parity, int nbricks,
                                             Scenes T, int act) {
    const int nact = rank_limit(T, ctl, act, RE_ACTIVE, CTL_NACTIVE);
    const int total = nact + min(ctl[CTL_OVF + parity], nbricks - ctl[CTL_NACTIVE]);
    const int step = ctl[CTL_STEP];
    const int lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int nwaves = gridDim.x * (WG / 64);
    float4* acc4 = reinterpret_cast<float4*>(acc);
    // The blocks of a wave are a software pipeline: the block index, the registration count
    // and this lane's first registration of the next block are loaded as the current block
    // starts, and that registration's tile box and the block's global-path flag once the
    // current block's tiles are in, so the chain block -> registrations -> boxes -> staged
    // tiles is not paid in full per block.  (Every read is in bounds: reg holds REG_MAX
    // entries per block index, and box is read only for a registration that exists.)
    const bool one = T.S == 1;
    int it = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    int b_nx = 0, m_nx = 0, r_nx = 0, dirty_nx = 0;
    int4 bb_nx = make_int4(0, 0, 0, 0);
    if (it < total) {
        b_nx = it < nact ? active[it] : ovf[it - nact];
        m_nx = it < nact ? reg_n[it] : 0;
        r_nx = reg[(int64_t)it * REG_MAX + lane];
        if (lane < m_nx) bb_nx = box[r_nx];
        dirty_nx = acc_dirty[__builtin_amdgcn_readfirstlane(b_nx)];
    }
    for (; it < total; it += nwaves) {
        const int b = __builtin_amdgcn_readfirstlane(b_nx);
        const int m = min(__builtin_amdgcn_readfirstlane(m_nx), REG_MAX);
        const int nx = it + nwaves;
        if (nx < total) {
            b_nx = nx < nact ? active[nx] : ovf[nx - nact];
            m_nx = nx < nact ? reg_n[nx] : 0;
            r_nx = reg[(int64_t)nx * REG_MAX + lane];
        } else {
            m_nx = 0;
        }
        // one scene: no lookup (the record's address does not depend on the block)
        const Scene& sc = T.scene[one ? 0 : T.rank_scene[rank_of_brick(T, b)]];
        const Step P = sc.P;
        const int NB = P.NB, base = sc.brick_base;
        const int lb = b - base;
        const int bx = lb % NB, by = (lb / NB) % NB, bz = lb / (NB * NB);
        const int n0 = 4 * (bx - 1), n1 = 4 * (by - 1), n2 = 4 * (bz - 1);  // first node of the block
        const int g[3] = {n0 + lx, n1 + ly, n2 + lz};
        // the block's global-atomic sums, if P2G sent any here this substep
        const bool dirty = __builtin_amdgcn_readfirstlane(dirty_nx) != 0;
        float4 a = dirty ? acc4[(int64_t)b * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (it < nact) {  // a physical block: gather the tiles registered with it (at most REG_MAX)
            int4 bb = bb_nx;  // this lane's registration of the round (the first round's was prefetched)
            for (int rb = 0; rb < m; rb += 64) {  // 64 registrations a round, one per lane
                // Each lane prepares its registration's tile for the whole wave: the lanes of
                // this block whose node lies in the tile's box (a 64-bit mask, lane = x + 4 y +
                // 16 z) and the staged index of the block's first node, so that node (x, y, z)
                // of the block sits at base + x + e0 y + e0 e1 z of the tight box layout.
                bool ov = false;  // does tile `lane` still exist and reach into this block?
                uint64_t lm = 0;
                int base = 0, s1 = 0, s2 = 0;
                if (rb > 0 && rb + lane < m) bb = box[reg[(int64_t)it * REG_MAX + rb + lane]];
                if (rb + lane < m) {
                    const int e0 = bb.y & 255, e1 = (bb.y >> 8) & 255, e2 = bb.y >> 16;
                    const int l0 = bb.x & 1023, l1 = (bb.x >> 10) & 1023, l2 = bb.x >> 20;
                    // block-local node range [x0, x1) x [y0, y1) x [z0, z1) inside the box
                    const int x0 = max(l0 - n0, 0), x1 = min(l0 + e0 - n0, 4);
                    const int y0 = max(l1 - n1, 0), y1 = min(l1 + e1 - n1, 4);
                    const int z0 = max(l2 - n2, 0), z1 = min(l2 + e2 - n2, 4);
                    ov = e0 > 0 && x0 < x1 && y0 < y1 && z0 < z1;
                    if (ov) {
                        const unsigned xm = ((1u << x1) - 1u) & ~((1u << x0) - 1u);
                        const unsigned ry = (0x1111u >> (4 * (4 - (y1 - y0)))) << (4 * y0);
                        const uint64_t rz = (0x0001000100010001ull >> (16 * (4 - (z1 - z0)))) << (16 * z0);
                        lm = (uint64_t)(xm * ry) * rz;  // the factors' set bits never overlap: no carries
                        base = bb.z + (n0 - l0) + e0 * ((n1 - l1) + e1 * (n2 - l2));
                        s1 = e0;
                        s2 = e0 * e1;
                    }
                }
                // the overlapping tiles in registration order, eight loads in flight at a time
                // (summed in the same order as one at a time)
                for (uint64_t mask = __ballot(ov); mask;) {
                    float4 sv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (mask) {  // wave-uniform
                            const int i = __builtin_ctzll(mask);
                            mask &= mask - 1;
                            const uint64_t lmi =
                                ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(lm >> 32), i) << 32) |
                                (unsigned)__builtin_amdgcn_readlane((int)(unsigned)lm, i);
                            const int bi = __builtin_amdgcn_readlane(base, i), s1i = __builtin_amdgcn_readlane(s1, i),
                                      s2i = __builtin_amdgcn_readlane(s2, i);
                            // every lane loads: those outside the tile's box read the zero node
                            const int ri = bi + lx + (int)__umul24(s1i, ly) + (int)__umul24(s2i, lz);
                            const int idx = ((lmi >> lane) & 1ull) ? ri : zero_node;
                            sv[u] = stage[idx];
                        } else {
                            sv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        a.x += sv[u].x;
                        a.y += sv[u].y;
                        a.z += sv[u].z;
                        a.w += sv[u].w;
                    }
                }
            }
        }
        // the next block's first-round tile boxes and global-path flag (its index and
        // registrations have arrived by now)
        if (lane < m_nx) bb_nx = box[r_nx];
        if (nx < total) dirty_nx = acc_dirty[__builtin_amdgcn_readfirstlane(b_nx)];
        float v[3] = {0.0f, 0.0f, 0.0f};
        if (a.x > 0.0f) {
            const float inv = __frcp_rn(a.x);
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
        if (BC && any) wall_condition(P, lowside, highside, v);
        // A block that took no mass this substep keeps its old contents and stamp: no
        // particle's stencil reaches it (every node of a stencil takes mass from its own
        // particle, or a weight of exactly zero, which multiplies the old finite value),
        // and reads of the grid show a block with an old stamp as empty.
        const bool took_mass = __ballot(a.x > 0.0f) != 0ull;
        if (took_mass) {
            vel[(int64_t)b * 64 + lane] = make_float4(v[0], v[1], v[2], a.x);
            if (P.flip > 0.0f) {  // ASFLIP: the change from the transferred velocity p/m
                float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
                if (a.x > 0.0f) {
                    const float inv = __frcp_rn(a.x);
                    d = make_float4(v[0] - a.y * inv, v[1] - a.z * inv, v[2] - a.w * inv, 0.0f);
                }
                dvel[(int64_t)b * 64 + lane] = d;
            }
        }
        if (CLEAR && dirty) acc4[(int64_t)b * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane == 0) {
            if (took_mass) stamp[b] = step;
            if (CLEAR && dirty) acc_dirty[b] = 0;
            if (CLEAR && it >= nact) brick_state[b] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl[CTL_OVF + (parity ^ 1)] = 0;
        ctl[CTL_FB + (parity ^ 1)] = 0;
    }
}

// -------------------------------------------------------------------- G2P
// A chunk's in-zone stencils lie in the node box its P2G tile used this
// substep (box[c]); the grid velocities of that box are loaded once, coalesced,
// into LDS and the 27-node gathers read LDS.  Particles whose stencil leaves
// the box gather from the dense grid.
// The free-zone test sets the rebuild request; so does a P2G that had to
// send more than `fb_limit` in-zone particles to global atomics because
// their chunk's box outgrew the tile (a rebuild shrinks the boxes again).
constexpr int G2P_BOX = 512;

template <bool LDS_BOX, int NT>
__global__ __launch_bounds__(NT) void k_g2p(float* __restrict__ S, int64_t cap, const Chunk* __restrict__ chunks,
                                            int* __restrict__ ctl, const float4* __restrict__ vel,
                                            const int4* __restrict__ box, int* __restrict__ host_flag, int parity,
                                            int fb_limit, int report_zone, Scenes T, int act,
                                            const float4* __restrict__ dvel) {
    __shared__ float4 tv[LDS_BOX ? G2P_BOX : 1];
    unsigned err = 0;
    bool left = report_zone && blockIdx.x == 0 && threadIdx.x == 0 && ctl[CTL_FB + parity] > fb_limit;
    int begin, end, stride;
    xcd_split(rank_limit(T, ctl, act, RE_CHUNK, CTL_NCHUNK), begin, end, stride);
    for (int c = begin; c < end; c += stride) {
        const Chunk ch = chunks[c];
        const Scene& sc = T.scene[ch.scene];
        const Step P = sc.P;
        const float c4 = 4.0f * P.fn;  // (4/dx^2) * dx
        const int NB = P.NB;
        const float4* vels = vel + (int64_t)sc.brick_base * BLOCK_NODES;
        // this thread's particle (a chunk holds at most NT): its position and
        // block word are loaded before the node box, so the two loads overlap
        const bool mine = (int)threadIdx.x < ch.count;
        const int p = ch.start + (mine ? (int)threadIdx.x : 0);
        float x[3] = {0.f, 0.f, 0.f}, fsid = 0.f;
        if (mine) {
#pragma unroll
            for (int a = 0; a < 3; ++a) x[a] = S[sidx(FX + a, p, cap)];
            fsid = S[sidx(FSID, p, cap)];
        }
        int lo[3] = {0, 0, 0}, e[3] = {0, 0, 0}, nt = 0, R = 4, Q = 8;
        if (LDS_BOX) {
            const int4 bb = box[c];
            e[0] = bb.y & 255;
            e[1] = (bb.y >> 8) & 255;
            e[2] = bb.y >> 16;
            lo[0] = bb.x & 1023;
            lo[1] = (bb.x >> 10) & 1023;
            lo[2] = bb.x >> 20;
            nt = e[0] * e[1] * e[2];
            // the P2G tile's padded pitches where they fit (with the rebuild's bank-dealt
            // lane order the lanes of one LDS pass then read different banks), else the
            // tight layout
            R = pitch_row(e[0]);
            Q = pitch_plane(R, e[1]);
            if (Q * e[2] > G2P_BOX) {
                R = e[0];
                Q = e[0] * e[1];
                if (nt > G2P_BOX) nt = 0;
            }
            load_node_box(tv, vels, NB, lo, e, nt, R, Q, threadIdx.x, NT);
            __syncthreads();
        }
        Stencil st;
        if (mine && make_stencil(x, P, st, err)) {
            float vp[3], Cn[9];
            g2p_gather(st, tv, vels, NB, lo, e, nt, R, Q, c4, vp, Cn);
#pragma unroll
            for (int k = 0; k < 9; ++k) S[sidx(FC + k, p, cap)] = Cn[k];
            // APIC: x' = x + dt v', v' the interpolated new grid velocity
            float xv[3] = {vp[0], vp[1], vp[2]};
            if (P.flip > 0.0f) {
                // ASFLIP: the particle's FLIP velocity v + sum w (v_i' - v~_i) (its own
                // velocity plus the interpolated grid change), blended in by `flip`; the
                // position takes a share beta of the FLIP correction, bmax unless the
                // particle's volume is being compressed (J' < 1; J' = J det(I + dt C') for
                // water, det(I + dt C') otherwise)
                const float4* dv = dvel + (int64_t)sc.brick_base * BLOCK_NODES;
                int xo[3], yo[3], zo[3];
                axis_offsets(st.base[0], 1, 0, xo);
                axis_offsets(st.base[1], NB, 2, yo);
                axis_offsets(st.base[2], NB * NB, 4, zo);
                float ds[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 3; ++o1) {
                        const float wyz = st.w[1][o1] * st.w[2][o2];
#pragma unroll
                        for (int o0 = 0; o0 < 3; ++o0) {
                            const float4 d = dv[xo[o0] + yo[o1] + zo[o2]];
                            const float w = wyz * st.w[0][o0];
                            ds[0] += w * d.x;
                            ds[1] += w * d.y;
                            ds[2] += w * d.z;
                        }
                    }
                float G[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) G[k] = P.dt * Cn[k] + ((k % 4 == 0) ? 1.0f : 0.0f);
                float J = det3(G);
                if (sc.M.kind == MPM_WATER) J *= S[sidx(FS, p, cap)];
                const float beta = J < 1.0f ? P.bmin : P.bmax;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float corr = S[sidx(FV + a, p, cap)] + ds[a] - vp[a];  // v_FLIP - v_PIC
                    xv[a] = vp[a] + beta * P.flip * corr;
                    vp[a] += P.flip * corr;
                }
            }
            bool fin = true;
            float xn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xn[a] = x[a] + P.dt * xv[a];
                S[sidx(FV + a, p, cap)] = vp[a];
                S[sidx(FX + a, p, cap)] = xn[a];
                fin = fin && (fabsf(xn[a]) < 1e30f) && (fabsf(vp[a]) < 1e30f);
            }
            int B[3];  // the particle's block at the last rebuild (its free zone)
            fsid_block(fsid, B);
            left = left || (report_zone && left_free_zone(xn, P.fn, B));
            if (!fin) err |= MPM_ERR_NONFINITE;
        }
        if (LDS_BOX) __syncthreads();
    }
    if (__ballot(left) != 0ull && (threadIdx.x & 63) == 0) {
        if (__hip_atomic_load(&ctl[CTL_REBUILD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
            atomicExch(&ctl[CTL_REBUILD], 1) == 0 && host_flag)
            __hip_atomic_store(host_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
    // every workgroup has read what it needs; the grid update of the next
    // substep stamps blocks with the advanced count
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[CTL_STEP] += 1;
}

// ------------------------------------------------------------- utilities
// Land the deferred deformation update of every particle (with the material
// and time step of its scene).
__global__ __launch_bounds__(WG) void k_materialize(float* __restrict__ S, int64_t cap, int N, Scenes T) {
    const int p = blockIdx.x * WG + threadIdx.x;
    if (p >= N) return;
    const Scene& sc = T.scene[fsid_scene(S[sidx(FSID, p, cap)])];
    float C[9], F[9], s, tau[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        C[k] = S[sidx(FC + k, p, cap)];
        F[k] = S[sidx(FF + k, p, cap)];
    }
    s = S[sidx(FS, p, cap)];
    material_step(sc.M, sc.P.dt, 1, C, F, s, tau);
#pragma unroll
    for (int k = 0; k < 9; ++k) S[sidx(FF + k, p, cap)] = F[k];
    S[sidx(FS, p, cap)] = s;
}

// Append `count` particles of `scene` at storage positions N0.., numbered
// id0.. inside their scene.
__global__ __launch_bounds__(WG) void k_insert(float* __restrict__ S, int* __restrict__ ids, int64_t cap, int N0,
                                               int count, int scene, int id0, const float* __restrict__ x,
                                               const float* __restrict__ v, const float* __restrict__ C,
                                               const float* __restrict__ F, const float* __restrict__ s,
                                               int* __restrict__ ctl) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= count) return;
    const int j = N0 + i;
    unsigned err = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float xa = x[a * (int64_t)count + i];
        if (!(fabsf(xa) < 1e30f)) err |= MPM_ERR_NONFINITE;
        else if (!(xa >= 0.0f && xa <= 1.0f)) err |= MPM_ERR_DOMAIN;
        S[sidx(FX + a, j, cap)] = xa;
        S[sidx(FV + a, j, cap)] = v ? v[a * (int64_t)count + i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        S[sidx(FC + k, j, cap)] = C ? C[k * (int64_t)count + i] : 0.0f;
        S[sidx(FF + k, j, cap)] = F ? F[k * (int64_t)count + i] : ((k % 4 == 0) ? 1.0f : 0.0f);
    }
    S[sidx(FS, j, cap)] = s ? s[i] : 1.0f;
    S[sidx(FSID, j, cap)] = __int_as_float(scene);
    ids[j] = id0 + i;
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
}

// Scatter the particles of one scene (Ns of them) to insertion order.
__global__ __launch_bounds__(WG) void k_read(const float* __restrict__ S, const int* __restrict__ ids, int64_t cap,
                                             int N, int scene, int Ns, int pending, Scenes T, float* __restrict__ x,
                                             float* __restrict__ v, float* __restrict__ C, float* __restrict__ F,
                                             float* __restrict__ s) {
    const int j = blockIdx.x * WG + threadIdx.x;
    if (j >= N || fsid_scene(S[sidx(FSID, j, cap)]) != scene) return;
    const Scene& sc = T.scene[scene];
    const int64_t id = ids[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (x) x[a * (int64_t)Ns + id] = S[sidx(FX + a, j, cap)];
        if (v) v[a * (int64_t)Ns + id] = S[sidx(FV + a, j, cap)];
    }
    float Cp[9], Fp[9], sp = S[sidx(FS, j, cap)], tau[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Cp[k] = S[sidx(FC + k, j, cap)];
        Fp[k] = S[sidx(FF + k, j, cap)];
        if (C) C[k * (int64_t)Ns + id] = Cp[k];
    }
    if (pending && (F || s)) material_step(sc.M, sc.P.dt, 1, Cp, Fp, sp, tau);
    if (F)
#pragma unroll
        for (int k = 0; k < 9; ++k) F[k * (int64_t)Ns + id] = Fp[k];
    if (s) s[id] = sp;
}

__global__ __launch_bounds__(WG) void k_read_grid(const float4* __restrict__ vel, const int* __restrict__ stamp,
                                                  int step, Step P, int base, float* __restrict__ m,
                                                  float* __restrict__ v) {
    const int n1 = P.n + 1;
    const int64_t NN = (int64_t)n1 * n1 * n1;
    const int64_t id = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (id >= NN) return;
    const int i = (int)(id / ((int64_t)n1 * n1)), j = (int)((id / n1) % n1), k = (int)(id % n1);
    const int b = base + (((k >> 2) + 1) * P.NB + ((j >> 2) + 1)) * P.NB + ((i >> 2) + 1);
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (stamp[b] == step) g = vel[(int64_t)b * 64 + (i & 3) + ((j & 3) << 2) + ((k & 3) << 4)];
    if (m) m[id] = g.w;
    if (v) {
        v[id] = g.x;
        v[NN + id] = g.y;
        v[2 * NN + id] = g.z;
    }
}

}  // namespace

int wgs_per_cu(const void* fn, int threads) {
    int dev = 0, lds_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
        lds_cu = 160 * 1024;
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) return 2;
    const int waves = (threads + 63) / 64;
    const int vgpr = a.numRegs > 0 ? (a.numRegs + 7) / 8 * 8 : 512;
    int per_simd = 512 / vgpr;
    if (per_simd > 8) per_simd = 8;
    int occ = per_simd * 4 / waves;
    if (a.sharedSizeBytes > 0) {
        const int by_lds = lds_cu / (int)a.sharedSizeBytes;
        if (by_lds < occ) occ = by_lds;
    }
    return occ < 1 ? 1 : occ;
}

namespace {
const void* g2p_fn(bool lds_box, int nt) {
    if (lds_box)
        return nt == 128   ? reinterpret_cast<const void*>(k_g2p<true, 128>)
               : nt == 256 ? reinterpret_cast<const void*>(k_g2p<true, 256>)
                           : reinterpret_cast<const void*>(k_g2p<true, 512>);
    return nt == 128   ? reinterpret_cast<const void*>(k_g2p<false, 128>)
           : nt == 256 ? reinterpret_cast<const void*>(k_g2p<false, 256>)
                       : reinterpret_cast<const void*>(k_g2p<false, 512>);
}
}  // namespace

void query_launch(Launch& L, int chunk) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&L.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (L.cus <= 0) L.cus = 256;
    auto grid_for = [&](const void* fn, int threads, int cap_per_cu) {
        int occ = wgs_per_cu(fn, threads);
        occ = occ > cap_per_cu ? cap_per_cu : occ;
        const int g = L.cus * occ;
        return g < 8 ? 8 : (g / 8) * 8;
    };
    const int nt = chunk_threads(chunk);
    L.p2g_grid = p2g_grid_size(L.cus, chunk);
    L.g2p_grid = grid_for(g2p_fn(true, nt), nt, 8 * 256 / nt);
    L.grid_grid = grid_for(reinterpret_cast<const void*>(k_grid<true, true>), WG, 8);
}

void enqueue_grid(hipStream_t st, const Launch& L, const Scenes& T, const BinBuffers& B, int* ctl, GridBuffers& G,
                  int parity, int nbricks, int act, int separate) {
    const bool bc = !(separate & 1), clear = !(separate & 2);
#define MPM_LAUNCH_GRID(BCV, CLV)                                                                                  \
    hipLaunchKernelGGL((k_grid<BCV, CLV>), dim3(L.grid_grid), dim3(WG), 0, st, G.acc, G.acc_dirty, G.vel, G.dvel, \
                       B.active, ctl, G.ovf[parity], B.brick_state, G.stamp, G.reg_n, G.reg, G.stage,                 \
                       G.stage_nodes, G.box, parity, nbricks, T, act)
    if (bc && clear) MPM_LAUNCH_GRID(true, true);
    else if (bc) MPM_LAUNCH_GRID(true, false);
    else if (clear) MPM_LAUNCH_GRID(false, true);
    else MPM_LAUNCH_GRID(false, false);
#undef MPM_LAUNCH_GRID
    if (!bc)
        hipLaunchKernelGGL(k_grid_walls, dim3(L.grid_grid), dim3(WG), 0, st, G.vel, G.dvel, B.active, ctl,
                           G.ovf[parity], parity, nbricks, T, act);
    if (!clear)
        hipLaunchKernelGGL(k_grid_clear, dim3(L.grid_grid), dim3(WG), 0, st, G.acc, G.acc_dirty, B.active, ctl,
                           G.ovf[parity], B.brick_state, parity, nbricks, T, act);
}

void enqueue_g2p(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap, const Chunk* chunks,
                 int* ctl, const GridBuffers& G, int* host_flag, int lds_box, int parity, int fb_limit, int chunk,
                 int act, int report_zone) {
#define MPM_LAUNCH_G2P(LB, NT)                                                                                    \
    hipLaunchKernelGGL((k_g2p<LB, NT>), dim3(L.g2p_grid), dim3(NT), 0, st, S, cap, chunks, ctl, G.vel, G.box, \
                       host_flag, parity, fb_limit, report_zone, T, act, G.dvel)
    const int nt = chunk_threads(chunk);
    if (lds_box) {
        if (nt == 128) MPM_LAUNCH_G2P(true, 128); else if (nt == 256) MPM_LAUNCH_G2P(true, 256); else MPM_LAUNCH_G2P(true, 512);
    } else {
        if (nt == 128) MPM_LAUNCH_G2P(false, 128); else if (nt == 256) MPM_LAUNCH_G2P(false, 256); else MPM_LAUNCH_G2P(false, 512);
    }
#undef MPM_LAUNCH_G2P
}

// The largest particle speed |v| into *out (zeroed by the caller): a wave
// maximum, then one atomic per wave on the float's bits (non-negative floats
// order like their bit patterns).
// Particle speeds: out[0] the largest (as ordered int bits), out[1] their sum.
// One add of each per workgroup (same-address atomics run one at a time).
__global__ __launch_bounds__(WG) void k_speeds(const float* __restrict__ S, int64_t cap, int N,
                                               float* __restrict__ out) {
    float m = 0.0f, sum = 0.0f;
    for (int p = blockIdx.x * WG + threadIdx.x; p < N; p += gridDim.x * WG) {
        const float a = S[sidx(FV, p, cap)], b = S[sidx(FV + 1, p, cap)], c = S[sidx(FV + 2, p, cap)];
        const float v = sqrtf(a * a + b * b + c * c);
        m = fmaxf(m, v);
        sum += v;
    }
    m = wave_maxf(m);
    sum = wave_sumf(sum);
    __shared__ float wm[WG / 64], ws[WG / 64];
    if ((threadIdx.x & 63) == 0) {
        wm[threadIdx.x >> 6] = m;
        ws[threadIdx.x >> 6] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) {
            m = fmaxf(m, wm[w]);
            sum += ws[w];
        }
        atomicMax(reinterpret_cast<int*>(out), __float_as_int(m));
        atomicAdd(out + 1, sum);
    }
}

// The speeds reduced into word[0..1] (cleared first), published to pinned
// host memory as float bits (host[0] largest, host[1] sum), word cleared again.
__global__ void k_publish_speeds(float* __restrict__ word, int* __restrict__ host) {
    if (threadIdx.x == 0) {
        __hip_atomic_store(host, __float_as_int(word[0]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(host + 1, __float_as_int(word[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        word[0] = 0.0f;
        word[1] = 0.0f;
    }
}

void enqueue_speeds(hipStream_t st, const float* S, int64_t cap, int N, float* out) {
    if (N <= 0) return;
    const int grid = cdiv(N, WG) < 256 ? cdiv(N, WG) : 256;
    hipLaunchKernelGGL(k_speeds, dim3(grid), dim3(WG), 0, st, S, cap, N, out);
}

void enqueue_speeds_to_host(hipStream_t st, const float* S, int64_t cap, int N, float* word, int* host) {
    enqueue_speeds(st, S, cap, N, word);
    hipLaunchKernelGGL(k_publish_speeds, dim3(1), dim3(64), 0, st, word, host);
}

void enqueue_materialize(hipStream_t st, const Scenes& T, float* S, int64_t cap, int N) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_materialize, dim3(cdiv(N, WG)), dim3(WG), 0, st, S, cap, N, T);
}

void enqueue_insert(hipStream_t st, float* S, int* ids, int64_t cap, int N0, int count, int scene, int id0,
                    const float* x, const float* v, const float* C, const float* F, const float* s, int* ctl) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_insert, dim3(cdiv(count, WG)), dim3(WG), 0, st, S, ids, cap, N0, count, scene, id0, x, v, C,
                       F, s, ctl);
}

void enqueue_read(hipStream_t st, const Scenes& T, const float* S, const int* ids, int64_t cap, int N, int scene,
                  int Ns, int pending, float* x, float* v, float* C, float* F, float* s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_read, dim3(cdiv(N, WG)), dim3(WG), 0, st, S, ids, cap, N, scene, Ns, pending, T, x, v, C, F,
                       s);
}

void enqueue_read_grid(hipStream_t st, const Scene& sc, const GridBuffers& G, int step, float* m, float* v) {
    const int64_t n1 = sc.P.n + 1;
    hipLaunchKernelGGL(k_read_grid, dim3(cdiv(n1 * n1 * n1, WG)), dim3(WG), 0, st, G.vel, G.stamp, step, sc.P,
                       sc.brick_base, m, v);
}

}  // namespace mpm
