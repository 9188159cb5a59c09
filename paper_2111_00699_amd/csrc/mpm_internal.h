// Internal declarations of the gfx950 MLS-MPM library: buffer layout,
// per-substep constants, launchers and the per-particle device math.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpm.h"

namespace mpm {

// ----------------------------------------------------------------- layout
// Particle state: FP32 scalar fields.  The default build stores them as a
// structure of arrays, field f of particle j at S[f * cap + j].  Built with
// MPM_AOSOA=1 (the layout ablation) it stores an array of structures of
// arrays: particles in groups of AOSOA_B = 64 (one wave), each group holding
// its fields one after another, 64 values each.  FSID holds integer bits:
// the particle's scene (bits 0-7) and the block it was binned to at the last
// rebuild (x, y, z in bits 8-15, 16-23, 24-31), which fixes its free zone; it
// moves with the particle through the rebuild permutation.
enum Field : int { FX = 0, FV = 3, FC = 6, FF = 15, FS = 24, FSID = 25, NF = 26 };

#ifndef MPM_AOSOA
#define MPM_AOSOA 0
#endif
constexpr int AOSOA_SHIFT = 6;
constexpr int AOSOA_B = 1 << AOSOA_SHIFT;

// Index of field f of particle j (cap: the buffer's particle capacity, a
// multiple of AOSOA_B), as a part common to all particles (the field's
// start) plus a 32-bit part per particle, so that loads address a uniform
// base plus a 32-bit offset.
__host__ __device__ __forceinline__ int64_t sidx(int f, int64_t j, int64_t cap) {
#if MPM_AOSOA
    (void)cap;
    const uint32_t jj = (uint32_t)j;
    return (int64_t)f * AOSOA_B + (int64_t)((jj >> AOSOA_SHIFT) * (uint32_t)(NF * AOSOA_B) + (jj & (AOSOA_B - 1)));
#else
    return (int64_t)f * cap + (int64_t)(uint32_t)j;
#endif
}

__device__ __forceinline__ int fsid_scene(float f) { return __float_as_int(f) & 255; }
__device__ __forceinline__ void fsid_block(float f, int B[3]) {
    const uint32_t u = (uint32_t)__float_as_int(f);
    B[0] = (int)((u >> 8) & 255u);
    B[1] = (int)((u >> 16) & 255u);
    B[2] = (int)(u >> 24);
}

constexpr int WG = 256;       // threads per workgroup (four wave64s)
constexpr int TILE = 12;      // nodes per axis reachable from one particle block (3 blocks)
constexpr int TILE3 = TILE * TILE * TILE;
constexpr int BLOCK_NODES = 64;  // 4^3 nodes per grid block

// Small device-side control words.
enum Ctl : int {
    CTL_NGB = 0,       // geometric (particle) blocks of the last rebuild
    CTL_NCHUNK = 1,    // work chunks of the last rebuild
    CTL_NACTIVE = 2,   // physical blocks of the last rebuild
    CTL_REBUILD = 3,   // a particle left its free zone since the last rebuild
    CTL_ERROR = 4,     // sticky MPM_ERR_* bits
    CTL_OVF = 5,       // overflow-block counts, two slots by substep parity
    CTL_SCAN = 8,      // scratch total of a device scan
    CTL_FB = 9,        // in-zone particles of chunks whose tile did not fit, two slots by substep parity
    CTL_STEP = 11,     // substeps completed (advanced by G2P; stamps the blocks the grid update touched)
    CTL_NGROUP = 12,   // merge groups (2x2x1 block slabs) of the last rebuild
    CTL_WORDS = 16,
    // 64-bit running counters, kept in CTL64_STRIPES copies a 128-byte line
    // apart (from byte offset 128): device-scope atomics on one address are
    // executed one after another (about 9 ns each on MI355X), so the many
    // waves that count spread their adds over the stripes, and a reader sums
    // the stripes.
    CTL64_FALLBACK_CHUNKS = 0,     // P2G chunks whose node box did not fit the LDS tile
    CTL64_GLOBAL_PARTICLES = 1,    // particles P2G scattered with global atomics
    CTL64_SUR_PARTICLES = 2,       // snow return maps done by the surrogate / closed-form path
    CTL64_SUR_FALLBACKS = 3,       // ... that fell back to the exact path
    CTL64_WORDS = 4,
    CTL64_BASE = 32,               // int offset of stripe 0
    CTL64_STRIDE = 16,             // 64-bit words per stripe (128 bytes)
    CTL64_STRIPES = 64,
    CTL_ALLOC_WORDS = CTL64_BASE + 2 * CTL64_STRIDE * CTL64_STRIPES
};

// Stripe s of the 64-bit counters (s taken modulo the stripe count).
__host__ __device__ inline unsigned long long* ctl64(int* ctl, int s = 0) {
    return reinterpret_cast<unsigned long long*>(ctl + CTL64_BASE) + (s & (CTL64_STRIPES - 1)) * CTL64_STRIDE;
}

// Derived material constants.
struct Mat {
    int kind;
    float mu, la;      // Lame parameters
    float mp;          // particle mass rho * V0
    float scale;       // 4 dt V0 / dx^2 (stress term of the APIC affine matrix)
    float lo, hi;      // snow singular-value bounds 1 - theta_c, 1 + theta_s
    float xi, bulk;
    float h0, h1, h2, h3;  // sand friction angle phi(q) = h0 + (h1 q - h3) exp(-h2 q), radians
    float kdp;             // sand (3 lambda + 2 mu) / (2 mu)
};

// Per-substep constants.
struct Step {
    int n;          // cells per axis
    int NB;         // padded blocks per axis, n/4 + 2
    float fn;       // float(n) = 1/dx
    float dx, dt;
    float g0, g1, g2;
    int bc, bc_cells;
    // ASFLIP transfer (flip = 0: APIC): the particle velocity blends the
    // interpolated new grid velocity with its own FLIP update by `flip`, and
    // the position moves with a share beta of that FLIP correction (bmax
    // where the particle's volume is not compressed, bmin elsewhere)
    float flip, bmin, bmax;
};

// A run of at most `chunk` sorted particles: a piece of one particle block,
// or several whole blocks of one 2x2x1 slab of blocks (sparse regions).
struct Chunk {
    int start, count;
    int tile;  // 1: registered with every physical block its in-zone stencils can reach (P2G may stage
               // a tile); 0: a registration list was full, the chunk scatters to global atomics
    int scene;
};

// Tile registrations per physical block, made by the rebuild: every chunk
// whose in-zone stencils can reach a block (the 3x3x3 neighbourhoods of the
// chunk's particle blocks) is listed under that block's position in the
// active list, in ascending chunk order.
constexpr int REG_MAX = 256;

// One scene of a context: its grid and time step, its material, where its
// dense block grid starts in the shared brick space, and its rank (position
// in the particle-code order; scenes are ranked by increasing dt, so the
// scenes still running late in a frame form a prefix of the ranks).
struct Scene {
    Step P;
    Mat M;
    int brick_base;
    int rank;
    int ret;  // snow return map: 0 exact (Jacobi), 1 learned surrogate, 2 closed form without the network
    float E;  // Young's modulus (scales the surrogate's stress outputs)
};

// Device tables of a context's scenes.  `rank_end` is filled at every
// rebuild: for rank r, rank_end[k*S + r] is the end (exclusive) of the
// entries of ranks <= r in the sorted particles (k = 0), geometric blocks
// (k = 1), chunks (k = 2) and physical blocks (k = 3).
struct Scenes {
    const Scene* scene;     // [S] by scene index
    const int* rank_scene;  // [S] scene index of each rank
    const int* rank_brick;  // [S + 1] first brick of each rank's grid; the brick space is laid out in rank order
    int* rank_end;          // [4 * S]
    int S;                  // number of scenes
    int shift;              // the rank sits at bit `shift` of a particle code (shift = 3 log2(max n))
    const float* sur_theta;  // surrogate parameters and normalisation (NULL when no scene uses it)
    const float* sur_norm;
    float sur_tol;           // residual tolerance of the learned map
    float sur_gap;           // smallest eigenvalue separation (units of the spread) for the closed form
    float sur_dt_ref;        // time step the surrogate was trained at
    int sur_any;             // 2: some scene runs the network; 1: some the closed form only; 0: none
};

enum RankEnd : int { RE_PART = 0, RE_GBLOCK = 1, RE_CHUNK = 2, RE_ACTIVE = 3 };

// Entries of kind k that belong to the first `act` ranks (act = S: all).
__device__ __forceinline__ int rank_limit(const Scenes& T, const int* ctl, int act, int k, int ctl_word) {
    return act >= T.S ? ctl[ctl_word] : T.rank_end[k * T.S + act - 1];
}

// Rank whose brick range holds brick b (binary search over S + 1 bases).
__device__ __forceinline__ int rank_of_brick(const Scenes& T, int b) {
    int lo = 0, hi = T.S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T.rank_brick[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------ launchers
// Binning and sorting (mpm_bin.hip).
struct BinBuffers {
    uint32_t *keys[2], *vals[2];
    int* hist;         // radix digit histograms [256][tiles]
    int* scan_tiles;   // per-tile sums of the generic scan
    int* gstart;       // [cap + 1]
    uint32_t* gcode;   // [cap]
    Chunk* chunks;     // [cap]
    int* brick_state;  // [bricks] 0 idle, 2 overflow this substep, 3 + i physical block at active[i]
    int* active;       // [bricks]
    int* group_start;  // [cap + 1] first geometric block of each merge group
    int* sorted_ids;   // [cap] insertion id of each particle in particle-code order
    int sorted;        // which keys/vals slot holds the last sorted codes (host side)
};

// Codes, stable radix sort, blocks, chunks and the gather into sorted order
// for all scenes at once; `key_bits` is the width of the particle codes.
void enqueue_rebuild(hipStream_t st, const Scenes& T, float* S_cur, float* S_alt, int* id_cur, int* id_alt,
                     int64_t cap, int N, int chunk, int spread, int pack, BinBuffers& B, int* ctl, int nbricks,
                     int key_bits,
                     int* reg_n, int* reg);
// dst[i] = src[i] & mask (particle codes without the rank bits).
void enqueue_copy_codes(hipStream_t st, uint32_t* dst, const uint32_t* src, int count, uint32_t mask);

// Substep kernels (mpm_step.hip).
struct GridBuffers {
    float* acc;     // [NB^3 * 64 * 4] (m, px, py, pz) accumulators, zero between substeps
    int* acc_dirty; // [NB^3] 1 where P2G's global atomics wrote the block's accumulators this
                    // substep; the grid update reads and clears only those blocks' accumulators
    float4* vel;    // [NB^3 * 64] (vx, vy, vz, m) after the grid update
    float4* dvel;   // [NB^3 * 64] (v - p/m, 0): the grid velocity change of the update, for ASFLIP
                    // scenes (allocated when a scene first takes ASFLIP; NULL before)
    int* stamp;     // [NB^3] substep index of the last update of each block
    int* ovf[2];    // overflow block lists, by substep parity
    float4* stage;  // [stage_nodes + 1] P2G tiles, (m, px, py, pz) per node; each P2G workgroup owns an
                    // equal slice of the first stage_nodes and packs the tiles of its chunks there; node
                    // stage_nodes stays zero (the grid update's loads outside a tile read it)
    int4* box;      // [cap] per chunk: x = tile origin packed 10 bits/axis, y = extent packed 8 bits/axis
                    // (0 = no tile), z = offset of the tile in `stage` (nodes)
    int stage_nodes;
    int* reg_n;     // [bricks] chunks registered with physical block i at the last rebuild (may exceed
                    // REG_MAX: those chunks have no tile)
    int* reg;       // [bricks * REG_MAX] their chunk indices, ascending
};

struct Launch {
    int p2g_grid, g2p_grid, grid_grid, cus;
};

// Threads per P2G/G2P workgroup for a chunk size: one particle per thread.
inline int chunk_threads(int chunk) { return chunk <= 128 ? 128 : chunk <= 256 ? 256 : 512; }

// `act`: the substep advances the scenes of the first `act` ranks only.
// fused: the previous substep's G2P runs inside P2G (see k_p2g); host_flag
// and fb_limit serve its free-zone request.  Only with the tile path and the
// exact return map (T.sur_any == 0, global_atomics == 0).
void enqueue_p2g(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap, const Chunk* chunks,
                 int* ctl, GridBuffers& G, int* brick_state, int pending, int parity, int global_atomics,
                 int nbricks, int chunk, int act, int fused, int* host_flag, int fb_limit);
int p2g_grid_size(int cus, int chunk);
// Workgroups of `threads` threads that fit on one compute unit at once, from
// the kernel's register and LDS use (gfx950: 512 VGPRs per lane and SIMD,
// 8 waves per SIMD, 4 SIMDs, `lds_per_cu` bytes of LDS).
int wgs_per_cu(const void* fn, int threads);
void enqueue_grid(hipStream_t st, const Launch& L, const Scenes& T, const BinBuffers& B, int* ctl, GridBuffers& G,
                  int parity, int nbricks, int act, int separate = 0);
// host_flag may be NULL (graph-recorded frames read no flag); report_zone 0
// leaves the free-zone request alone (a G2P that only brings the state up to
// date before it is read; the next substep's G2P reports the same exits).
void enqueue_g2p(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap, const Chunk* chunks,
                 int* ctl, const GridBuffers& G, int* host_flag, int lds_box, int parity, int fb_limit, int chunk,
                 int act, int report_zone);
void enqueue_materialize(hipStream_t st, const Scenes& T, float* S, int64_t cap, int N);
// Particle speeds of the whole state: out[0] the largest, out[1] the sum (out zeroed by the caller).
void enqueue_speeds(hipStream_t st, const float* S, int64_t cap, int N, float* out);
// ... reduced into word[0..1] (zero on entry), published to pinned host[0..1] as float bits, and
// word cleared again (graph frames)
void enqueue_speeds_to_host(hipStream_t st, const float* S, int64_t cap, int N, float* word, int* host);
void enqueue_clear_overflow(hipStream_t st, int* ctl);
// The same with each snow scene's own map (exact, closed form or network), over the chunk list of the
// last rebuild; for contexts with T.sur_any != 0.
void enqueue_materialize_map(hipStream_t st, const Launch& L, const Scenes& T, float* S, int64_t cap,
                             const Chunk* chunks, const int* ctl, int chunk);
void enqueue_insert(hipStream_t st, float* S, int* ids, int64_t cap, int N0, int count, int scene, int id0,
                    const float* x, const float* v, const float* C, const float* F, const float* s, int* ctl);
void enqueue_read(hipStream_t st, const Scenes& T, const float* S, const int* ids, int64_t cap, int N, int scene,
                  int Ns, int pending, float* x, float* v, float* C, float* F, float* s);
void enqueue_read_grid(hipStream_t st, const Scene& sc, const GridBuffers& G, int step, float* m, float* v);
void query_launch(Launch& L, int chunk);

// ----------------------------------------------------------- device math
__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 low bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {  // inverse of spread3
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0x030000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

// One Jacobi rotation of a symmetric 3x3 in the (p,q) plane that zeroes a_pq;
// r is the remaining index.  The rotation is accumulated into columns p, q of U.
__device__ __forceinline__ void jacobi_rotate(float& app, float& aqq, float& apq, float& arp, float& arq, float& u0p,
                                              float& u0q, float& u1p, float& u1q, float& u2p, float& u2q) {
    const float d = aqq - app;
    const float den = fabsf(d) + sqrtf(d * d + 4.0f * apq * apq);
    const float t = den > 0.0f ? __fdividef(d >= 0.0f ? 2.0f * apq : -2.0f * apq, den) : 0.0f;
    const float c = rsqrtf(1.0f + t * t);
    const float s = t * c;
    app -= t * apq;
    aqq += t * apq;
    apq = 0.0f;
    const float rp = arp, rq = arq;
    arp = c * rp - s * rq;
    arq = s * rp + c * rq;
    float a, b;
    a = u0p; b = u0q; u0p = c * a - s * b; u0q = s * a + c * b;
    a = u1p; b = u1q; u1p = c * a - s * b; u1q = s * a + c * b;
    a = u2p; b = u2q; u2p = c * a - s * b; u2q = s * a + c * b;
}

// Eigen-decomposition of the symmetric b = [b00 b01 b02; . b11 b12; . . b22]
// by cyclic Jacobi sweeps.  On return lam[k] are the eigenvalues and column k
// of U (U[i*3+k]) the matching unit eigenvector.
__device__ __forceinline__ void eig_sym3(float b00, float b01, float b02, float b11, float b12, float b22, float U[9],
                                         float lam[3]) {
    float u00 = 1, u01 = 0, u02 = 0, u10 = 0, u11 = 1, u12 = 0, u20 = 0, u21 = 0, u22 = 1;
#pragma unroll
    for (int sweep = 0; sweep < 3; ++sweep) {  // quadratic convergence: 3 sweeps reach FP32 rounding
        // the third sweep only if some lane of the wave still has off-diagonal mass above
        // FP32 rounding (|offdiag| > 1e-7 |diag|)
        if (sweep == 2 && __all(b01 * b01 + b02 * b02 + b12 * b12 <= 1e-14f * (b00 * b00 + b11 * b11 + b22 * b22)))
            break;
        jacobi_rotate(b00, b11, b01, b02, b12, u00, u01, u10, u11, u20, u21);  // (0,1), r = 2
        jacobi_rotate(b00, b22, b02, b01, b12, u00, u02, u10, u12, u20, u22);  // (0,2), r = 1
        jacobi_rotate(b11, b22, b12, b01, b02, u01, u02, u11, u12, u21, u22);  // (1,2), r = 0
    }
    lam[0] = b00; lam[1] = b11; lam[2] = b22;
    U[0] = u00; U[1] = u01; U[2] = u02;
    U[3] = u10; U[4] = u11; U[5] = u12;
    U[6] = u20; U[7] = u21; U[8] = u22;
}

// a / b refined by one Newton step on the reciprocal quotient: the library
// divides by hardware reciprocals (1 ulp), and where the quotient feeds a
// quantity that must be exact (a = b gives exactly 1) the residual
// a - q b, exact in an FMA, corrects it.
__device__ __forceinline__ float div_refined(float a, float b) {
    const float r = 1.0f / b;
    const float q = a * r;
    return fmaf(fmaf(-q, b, a), r, q);
}

__device__ __forceinline__ float det3(const float A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// out = (I + dt C) A
__device__ __forceinline__ void advance_gradient(const float C[9], float dt, const float A[9], float out[9]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            out[a * 3 + b] = A[a * 3 + b] +
                             dt * (C[a * 3 + 0] * A[0 * 3 + b] + C[a * 3 + 1] * A[1 * 3 + b] + C[a * 3 + 2] * A[2 * 3 + b]);
}

// U diag(d) U^T as the 6 entries (00, 01, 02, 11, 12, 22)
__device__ __forceinline__ void sym_from_eig(const float U[9], float d0, float d1, float d2, float T[6]) {
    T[0] = U[0] * U[0] * d0 + U[1] * U[1] * d1 + U[2] * U[2] * d2;
    T[1] = U[0] * U[3] * d0 + U[1] * U[4] * d1 + U[2] * U[5] * d2;
    T[2] = U[0] * U[6] * d0 + U[1] * U[7] * d1 + U[2] * U[8] * d2;
    T[3] = U[3] * U[3] * d0 + U[4] * U[4] * d1 + U[5] * U[5] * d2;
    T[4] = U[3] * U[6] * d0 + U[4] * U[7] * d1 + U[5] * U[8] * d2;
    T[5] = U[6] * U[6] * d0 + U[7] * U[7] * d1 + U[8] * U[8] * d2;
}

// Singular values of F from the eigen-decomposition of b = F F^T, with the
// sign of det F carried by the smallest one; U holds the left singular vectors.
__device__ __forceinline__ void left_svd(const float F[9], float U[9], float sig[3], float& J) {
    const float b00 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const float b01 = F[0] * F[3] + F[1] * F[4] + F[2] * F[5];
    const float b02 = F[0] * F[6] + F[1] * F[7] + F[2] * F[8];
    const float b11 = F[3] * F[3] + F[4] * F[4] + F[5] * F[5];
    const float b12 = F[3] * F[6] + F[4] * F[7] + F[5] * F[8];
    const float b22 = F[6] * F[6] + F[7] * F[7] + F[8] * F[8];
    float lam[3];
    eig_sym3(b00, b01, b02, b11, b12, b22, U, lam);
    sig[0] = sqrtf(fmaxf(lam[0], 0.0f));
    sig[1] = sqrtf(fmaxf(lam[1], 0.0f));
    sig[2] = sqrtf(fmaxf(lam[2], 0.0f));
    J = det3(F);
    if (J < 0.0f) {  // negate the smallest singular value
        const int k = (sig[0] <= sig[1]) ? (sig[0] <= sig[2] ? 0 : 2) : (sig[1] <= sig[2] ? 1 : 2);
        sig[k] = -sig[k];
    }
}

// Sand: Hencky elasticity in the logarithmic strain eps = log |sig| and the
// Drucker-Prager return map of Klar et al. 2016 (a stand-in for the sand model
// the paper cites).  When `pending`, the trial gradient Fh = U diag(sig) V^T
// is mapped: expansion (tr eps > 0) releases all elastic strain; otherwise
// dg = |dev eps| + kdp tr(eps) alpha(q) > 0 scales the deviator down by dg.
// The new gradient U diag(exp eps') V^T is Fh + U diag(exp(eps')/sig - 1) U^T Fh,
// and s = 1 + q grows by the log strain removed.  sig and J come back as those
// of the stored gradient; e its log strain.
__device__ __forceinline__ void sand_return_map(const Mat& M, int pending, const float U[9], const float Fh[9],
                                                float F[9], float sig[3], float& s, float e[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = __logf(fmaxf(fabsf(sig[k]), 1e-6f));
    if (!pending) return;
    const float t = e[0] + e[1] + e[2];
    float d[3];
    float nd = 0.0f, ne = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k] = e[k] - t * (1.0f / 3.0f);
        nd += d[k] * d[k];
        ne += e[k] * e[k];
    }
    nd = sqrtf(nd);
    float en[3] = {e[0], e[1], e[2]};
    float dq = 0.0f;
    if (t > 0.0f) {
        en[0] = en[1] = en[2] = 0.0f;
        dq = sqrtf(ne);
    } else {
        const float q = s - 1.0f;
        const float phi = M.h0 + (M.h1 * q - M.h3) * __expf(-M.h2 * q);
        const float sp = __sinf(phi);
        const float alpha = 0.81649658f * 2.0f * sp / (3.0f - sp);  // sqrt(2/3) 2 sin / (3 - sin)
        const float dg = nd + M.kdp * t * alpha;
        if (dg > 0.0f) {
            const float r = dg / nd;
#pragma unroll
            for (int k = 0; k < 3; ++k) en[k] = e[k] - r * d[k];
            dq = dg;
        }
    }
    if (dq > 0.0f) {
        float r[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float sn = __expf(en[k]);
            r[k] = sn / copysignf(fmaxf(fabsf(sig[k]), 1e-6f), sig[k]) - 1.0f;
            sig[k] = sn;
            e[k] = en[k];
        }
        float R[6];
        sym_from_eig(U, r[0], r[1], r[2], R);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const float f0 = Fh[0 * 3 + b], f1 = Fh[1 * 3 + b], f2 = Fh[2 * 3 + b];
            F[0 * 3 + b] = f0 + (R[0] * f0 + R[1] * f1 + R[2] * f2);
            F[1 * 3 + b] = f1 + (R[1] * f0 + R[3] * f1 + R[4] * f2);
            F[2 * 3 + b] = f2 + (R[2] * f0 + R[4] * f1 + R[5] * f2);
        }
        s += dq;
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) F[i] = Fh[i];
    }
}

// Apply the deferred deformation update of the last G2P (when `pending`),
// the snow return map, and produce the Kirchhoff stress tau (6 entries).
// F (9) and s are updated in place.
__device__ __forceinline__ void material_step(const Mat& M, float dt, int pending, const float C[9], float F[9],
                                              float& s, float tau[6]) {
    if (M.kind == MPM_WATER) {
        if (pending) {
            float G[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) G[i] = dt * C[i] + ((i % 4 == 0) ? 1.0f : 0.0f);
            s *= det3(G);
        }
        const float p = M.bulk * (s - 1.0f) * s;
        tau[0] = p; tau[1] = 0.0f; tau[2] = 0.0f; tau[3] = p; tau[4] = 0.0f; tau[5] = p;
        return;
    }
    float Fh[9];
    if (pending) {
        advance_gradient(C, dt, F, Fh);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) Fh[i] = F[i];
    }
    float U[9], sig[3], J;
    left_svd(Fh, U, sig, J);
    float mu = M.mu, la = M.la;
    if (M.kind == MPM_SAND) {
        float e[3];
        sand_return_map(M, pending, U, Fh, F, sig, s, e);
        const float tr = la * (e[0] + e[1] + e[2]);
        sym_from_eig(U, 2.0f * mu * e[0] + tr, 2.0f * mu * e[1] + tr, 2.0f * mu * e[2] + tr, tau);
        return;
    }
    if (M.kind == MPM_SNOW) {
        if (pending) {
            float sc[3], r[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sc[k] = fminf(fmaxf(sig[k], M.lo), M.hi);
                r[k] = __fdividef(sc[k], sig[k]) - 1.0f;  // zero inside the yield surface
            }
            // F_E' = U diag(sc/sig) U^T Fhat = Fhat + U diag(sc/sig - 1) U^T Fhat: the
            // rounding of U (orthogonal only to FP32 precision) then scales with the
            // plastic correction instead of adding strain noise to elastic states.
            float R[6];
            sym_from_eig(U, r[0], r[1], r[2], R);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float f0 = Fh[0 * 3 + b], f1 = Fh[1 * 3 + b], f2 = Fh[2 * 3 + b];
                F[0 * 3 + b] = f0 + (R[0] * f0 + R[1] * f1 + R[2] * f2);
                F[1 * 3 + b] = f1 + (R[1] * f0 + R[3] * f1 + R[4] * f2);
                F[2 * 3 + b] = f2 + (R[2] * f0 + R[4] * f1 + R[5] * f2);
            }
            const float Jc = sc[0] * sc[1] * sc[2];
            s = s * J / Jc;
            J = Jc;
            sig[0] = sc[0]; sig[1] = sc[1]; sig[2] = sc[2];
        }
        const float h = __expf(M.xi * (1.0f - s));
        mu *= h;
        la *= h;
    } else if (pending) {
#pragma unroll
        for (int i = 0; i < 9; ++i) F[i] = Fh[i];
    }
    const float vol = la * (J - 1.0f) * J;
    sym_from_eig(U, 2.0f * mu * (sig[0] - 1.0f) * sig[0] + vol, 2.0f * mu * (sig[1] - 1.0f) * sig[1] + vol,
                 2.0f * mu * (sig[2] - 1.0f) * sig[2] + vol, tau);
}

}  // namespace mpm
