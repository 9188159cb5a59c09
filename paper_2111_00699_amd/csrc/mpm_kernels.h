// Device helpers shared by the substep kernels: per-XCD work split, the
// quadratic B-spline stencil, dense block addressing, overflow-block
// activation and wave64 reductions.
#pragma once

#include <limits.h>

#include "mpm_internal.h"

namespace mpm {

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Contiguous per-XCD ranges: workgroup w runs on XCD w % 8, so each XCD walks
// its own contiguous slice of the block-sorted work list.
__device__ __forceinline__ void xcd_split(int total, int& begin, int& end, int& stride) {
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    stride = gridDim.x >> 3;
    begin = (int)(((int64_t)total * x) >> 3) + slot;
    end = (int)(((int64_t)total * (x + 1)) >> 3);
}

struct Stencil {
    int base[3];
    float f[3];
    float w[3][3];
};

// Quadratic B-spline stencil: base = floor(x/dx - 1/2), f = x/dx - base,
// weights 1/2 (3/2 - f)^2, 3/4 - (f - 1)^2, 1/2 (f - 1/2)^2.  Returns false
// (and sets an error bit) when x is not finite or the stencil leaves [0, n].
__device__ __forceinline__ bool make_stencil(const float x[3], const Step& P, Stencil& s, unsigned& err) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float t = x[a] * P.fn;
        const float b = floorf(t - 0.5f);
        if (!(b == b)) {
            err |= MPM_ERR_NONFINITE;
            ok = false;
            s.base[a] = 0;
            s.f[a] = 1.0f;
        } else {
            if (!(b >= 0.0f && b <= (float)(P.n - 2))) {
                err |= MPM_ERR_DOMAIN;
                ok = false;
            }
            s.base[a] = (int)b;
            s.f[a] = t - b;
        }
        const float f = s.f[a];
        s.w[a][0] = 0.5f * (1.5f - f) * (1.5f - f);
        s.w[a][1] = 0.75f - (f - 1.0f) * (f - 1.0f);
        s.w[a][2] = 0.5f * (f - 0.5f) * (f - 0.5f);
    }
    return ok;
}

// Offsets (in nodes) into the dense block array for the three stencil nodes
// along one axis: block = (node >> 2) + 1 (padded), local = node & 3.
__device__ __forceinline__ void axis_offsets(int base, int blockstride, int localshift, int off[3]) {
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        const int node = base + o;
        off[o] = ((node >> 2) + 1) * blockstride * BLOCK_NODES + ((node & 3) << localshift);
    }
}

// ------------------------------------------------------------ node boxes
// Padded layout of a node box of ext0 x ext1 x ext2 nodes in LDS: node
// (x, y, z) at x + R y + Q z with the row pitch R the smallest of 4, 12, 20,
// 28, ... that holds a row (so R >= ext0 and R = 4 or 12 mod 16) and the
// plane pitch Q = 8 (mod 16).  With the round-ordered chunks, the 16 lanes an
// LDS access serves together hold cells x in 0..3, y in {y, y+1}, z in
// {z, z+1}; their addresses x + R y' + Q z' are 16 different values mod 16
// for every stencil offset, so 8-byte (FP64) and 16-byte (float4) accesses
// meet no bank conflicts.  (A chunk of several blocks has a box up to 16
// nodes wide.)
__device__ __forceinline__ int pitch_row(int e0) { return e0 <= 4 ? 4 : ((e0 + 3) & ~7) + 4; }
__device__ __forceinline__ int pitch_plane(int R, int e1) {
    const int q = R * e1;
    return q + ((8 - (q & 15)) & 15);
}

// floor(u / d) for 0 <= u < 2^20 and d >= 1, from rcp = 1/d in FP32 (1 ulp):
// (u + 1/2) rcp lies within (u + 1/2) 2^-22 / d of (u + 1/2) / d, which is at
// least 1/(2d) away from every integer, so the truncation is exact while
// (u + 1/2) 2^-22 < 1/2.  Three instructions instead of an integer division.
__device__ __forceinline__ int div_small(int u, float rcp) { return (int)(((float)u + 0.5f) * rcp); }

// ------------------------------------------------------------ G2P pieces
// A chunk's node box (origin lo, extent e per axis, from its P2G tile) as a
// float4 array tv[x + R y + Q z] of grid velocities (R, Q: the row and plane
// pitches), loaded by the workgroup's threads (vels: the scene's node
// velocities; nt = e0 e1 e2 nodes).
__device__ __forceinline__ void load_node_box(float4* tv, const float4* vels, int NB, const int lo[3],
                                              const int e[3], int nt, int R, int Q, int tid, int nthreads) {
    const float r0 = 1.0f / (float)e[0], r01 = 1.0f / (float)(e[0] * e[1]);
    for (int t = tid; t < nt; t += nthreads) {
        const int z = div_small(t, r01), t01 = t - z * e[0] * e[1];
        const int y = div_small(t01, r0), x = t01 - y * e[0];
        const int gx = lo[0] + x, gy = lo[1] + y, gz = lo[2] + z;
        tv[x + R * y + Q * z] = vels[((((gz >> 2) + 1) * NB + ((gy >> 2) + 1)) * NB + ((gx >> 2) + 1)) * 64 +
                                     (gx & 3) + ((gy & 3) << 2) + ((gz & 3) << 4)];
    }
}

// G2P of one particle with stencil st: v' = sum w v_i and
// C' = 4/dx^2 sum w v_i (x_i - x_p)^T, gathered from the node box tv
// (nt > 0 nodes, origin lo, extent e, pitches R, Q) when the stencil lies
// inside it, else from the dense node velocities.  c4 = 4/dx.
__device__ __forceinline__ void g2p_gather(const Stencil& st, const float4* tv, const float4* vels, int NB,
                                           const int lo[3], const int e[3], int nt, int R, int Q, float c4,
                                           float vp[3], float Cn[9]) {
    int r[3];
    bool inbox = nt > 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r[a] = st.base[a] - lo[a];
        inbox = inbox && r[a] >= 0 && r[a] + 2 < e[a];
    }
    // Separable sums: along each x-row (o1, o2) r_a = sum_o0 wx[o0] v_a and
    // rx_a = sum_o0 o0 wx[o0] v_a, then v' += wyz r, Mo_a0 += wyz rx_a,
    // Mo_a1 += o1 wyz r_a, Mo_a2 += o2 wyz r_a (terms with a zero offset are
    // not formed).
    float Mo[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // sum w v_a o_b
#pragma unroll
    for (int a = 0; a < 3; ++a) vp[a] = 0.0f;
    const float wx1 = st.w[0][1], wx2 = st.w[0][2], wx2d = 2.0f * st.w[0][2];
    auto row = [&](int o1, int o2, const float4 g0, const float4 g1, const float4 g2) {
        const float wyz = st.w[1][o1] * st.w[2][o2];
        const float rr[3] = {st.w[0][0] * g0.x + wx1 * g1.x + wx2 * g2.x, st.w[0][0] * g0.y + wx1 * g1.y + wx2 * g2.y,
                             st.w[0][0] * g0.z + wx1 * g1.z + wx2 * g2.z};
        const float rx[3] = {wx1 * g1.x + wx2d * g2.x, wx1 * g1.y + wx2d * g2.y, wx1 * g1.z + wx2d * g2.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float t = wyz * rr[a];
            vp[a] += t;
            Mo[a * 3 + 0] += wyz * rx[a];
            if (o1 == 1) Mo[a * 3 + 1] += t;
            if (o1 == 2) Mo[a * 3 + 1] += 2.0f * t;
            if (o2 == 1) Mo[a * 3 + 2] += t;
            if (o2 == 2) Mo[a * 3 + 2] += 2.0f * t;
        }
    };
    if (inbox) {
        const int tb = r[0] + R * r[1] + Q * r[2];
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1) {
                const int t = tb + R * o1 + Q * o2;
                row(o1, o2, tv[t], tv[t + 1], tv[t + 2]);
            }
    } else {
        int xo[3], yo[3], zo[3];
        axis_offsets(st.base[0], 1, 0, xo);
        axis_offsets(st.base[1], NB, 2, yo);
        axis_offsets(st.base[2], NB * NB, 4, zo);
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1) {
                const int t = yo[o1] + zo[o2];
                row(o1, o2, vels[xo[0] + t], vels[xo[1] + t], vels[xo[2] + t]);
            }
    }
    // C' = 4/dx^2 sum w v (x_i - x_p)^T = (4/dx) (Mo - v' f^T)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2) Cn[a * 3 + b2] = c4 * (Mo[a * 3 + b2] - vp[a] * st.f[b2]);
}

// The particle's cell code after the move must stay within [4B-3, 4B+6] per
// axis (its free zone, B its block at the last rebuild).
__device__ __forceinline__ bool left_free_zone(const float xn[3], float fn, const int B[3]) {
    bool left = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float cc = floorf(xn[a] * fn - 0.5f) + 1.0f;
        left = left || !(cc >= (float)(4 * B[a] - 3) && cc <= (float)(4 * B[a] + 6));
    }
    return left;
}

// Mark the (at most 2x2x2) blocks of a stencil in the block grid of its
// scene (NB padded blocks per axis, first brick `base`); blocks outside the
// physical set of the last rebuild are appended once to the overflow list.
__device__ __forceinline__ void activate_blocks(const Stencil& s, int NB, int base, int* brick_state, int* ovf,
                                                int* ovf_count, int nbricks, unsigned& err) {
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = (s.base[a] >> 2) + 1;
        hi[a] = ((s.base[a] + 2) >> 2) + 1;
    }
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
        for (int by = lo[1]; by <= hi[1]; ++by)
            for (int bx = lo[0]; bx <= hi[0]; ++bx) {
                const int b = base + (bz * NB + by) * NB + bx;
                if (__hip_atomic_load(&brick_state[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                    atomicCAS(&brick_state[b], 0, 2) == 0) {
                    const int k = atomicAdd(ovf_count, 1);
                    if (k < nbricks)
                        ovf[k] = b;
                    else
                        err |= MPM_ERR_CAPACITY;
                }
            }
}

// Wave-wide min / max of an int, in DPP steps (no LDS): row_shr 1, 2, 4, 8
// leaves each 16-lane row's result in its lane 15, row_bcast 15 and 31 carry
// it across the rows, lane 63 ends with the wave's result.  All lanes active.
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

}  // namespace mpm
