// Rebuild-mapping and particle sorting on gfx950.
//
// Paper, "Material Point Method on a Single GPU": particle codes interleave
// the 3-D cell index with the block code in the high bits and the cell code
// in the low bits; the blocks holding particles (gblocks) and their 3x3x3
// neighbours (pblocks) are recorded; particles are sorted to cell
// granularity.  "Rebuild-Mapping": particle blocks are shifted by -dx/2 so a
// particle block with its 3x3x3 neighbours covers a (10 dx)^3 free zone.
//
// MI355X design: the block table is a dense array over the padded domain
// (288 GB of HBM make a dense (n/4+2)^3 table trivial), so no hash is needed
// and block activation is a mark + compaction, deterministic and in block
// order.  Sorting is a stable LSD radix sort with 8-bit digits, ranks taken
// inside each wave64 from eight ballots (no atomics), so the permutation is
// exactly a stable sort by particle code.  A batched context puts the scene's
// rank above the Morton bits, so one sort orders every scene, scene by
// scene, and every later list (blocks, chunks, physical blocks) comes out
// rank-major; the per-rank ends of those lists let a substep run a prefix of
// the ranks.
#include "mpm_internal.h"

namespace mpm {

namespace {

constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = WG * RS_ITEMS;  // 4096 keys per radix tile
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = WG * SCAN_ITEMS;  // 2048 entries per scan tile

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane_id() >= d) v += t;
    }
    return v;
}

// Exclusive scan over the 256 threads of a workgroup; *total gets the sum.
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[WG / 64];
    const int w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
        off += (i < w) ? wsum[i] : 0;
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ------------------------------------------------------------ particle code
// c = floor(x/dx + 1/2) = floor(x n - 1/2) + 1 per axis.  For power-of-two
// n, x*n is exact in FP32 and x*n - 1/2 is exact wherever it matters, so the
// code is bit-identical to one computed in FP64 from the same FP32 x.  The
// scene's rank goes above the Morton bits.
__global__ __launch_bounds__(WG) void k_keys(const float* __restrict__ S, int64_t cap, int N, Scenes T,
                                             uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                             int* __restrict__ ctl) {
    const int j = blockIdx.x * WG + threadIdx.x;
    if (j >= N) return;
    const Scene& sc = T.scene[fsid_scene(S[sidx(FSID, j, cap)])];
    const float fn = sc.P.fn;
    const int n = sc.P.n;
    uint32_t code = (uint32_t)sc.rank << T.shift;
    unsigned err = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = S[sidx(FX + a, j, cap)];
        const float b = floorf(x * fn - 0.5f);
        int c;
        if (!(b == b)) {
            err |= MPM_ERR_NONFINITE;
            c = 0;
        } else {
            if (!(b >= 0.0f && b <= (float)(n - 2))) err |= MPM_ERR_DOMAIN;
            c = (int)fminf(fmaxf(b + 1.0f, 0.0f), (float)(n - 1));
        }
        code |= spread3((uint32_t)c) << a;
    }
    keys[j] = code;
    vals[j] = (uint32_t)j;
    if (err) atomicOr(&ctl[CTL_ERROR], (int)err);
}

// --------------------------------------------------------------- radix sort
__global__ __launch_bounds__(WG) void k_rs_hist(const uint32_t* __restrict__ keys, int N, int shift, int tiles,
                                                int* __restrict__ hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = base + r * WG + threadIdx.x;
        if (i < N) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of the tile are taken in order, 256 at a time; inside
// a wave the rank among lanes with the same digit comes from eight ballots,
// across the four waves from per-wave digit counts in LDS.
__global__ __launch_bounds__(WG) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int N,
                                                   int shift, int tiles, const int* __restrict__ offs) {
    __shared__ int base[256];
    __shared__ int wcnt[WG / 64][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    base[tid] = offs[tid * tiles + blockIdx.x];
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) wcnt[i][tid] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = blockIdx.x * RS_TILE + r * WG + tid;
        const bool valid = i < N;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int off = base[d] + rank;
#pragma unroll
            for (int k = 0; k < WG / 64; ++k) off += (k < w) ? wcnt[k][d] : 0;
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int k = 0; k < WG / 64; ++k) {
            add += wcnt[k][tid];
            wcnt[k][tid] = 0;
        }
        base[tid] += add;
        __syncthreads();
    }
}

// --------------------------------------------------------- generic scan
// Three launches: per-tile totals, a one-workgroup scan of the totals, and a
// per-tile exclusive scan that hands each element its output offset.
template <class Op>
__global__ __launch_bounds__(WG) void k_scan_count(Op op, int n, int* __restrict__ tile_sums) {
    const int first = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (first + i < n) s += op.count(first + i);
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(WG) void k_scan_top(int* __restrict__ a, int n, int* __restrict__ total) {
    int carry = 0;
    for (int base = 0; base < n; base += WG) {
        const int i = base + threadIdx.x;
        const int v = i < n ? a[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, &tot);
        if (i < n) a[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

template <class Op>
__global__ __launch_bounds__(WG) void k_scan_emit(Op op, int n, const int* __restrict__ tile_offs) {
    const int first = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int c[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        c[i] = (first + i < n) ? op.count(first + i) : 0;
        s += c[i];
    }
    int tot;
    int off = tile_offs[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (c[i] > 0) op.emit(first + i, off, c[i]);
        off += c[i];
    }
}

template <class Op>
void device_scan(hipStream_t st, const Op& op, int n, int* tile_sums, int* total) {
    const int tiles = cdiv(n > 0 ? n : 1, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_count<Op>, dim3(tiles), dim3(WG), 0, st, op, n, tile_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(WG), 0, st, tile_sums, tiles, total);
    hipLaunchKernelGGL(k_scan_emit<Op>, dim3(tiles), dim3(WG), 0, st, op, n, tile_sums);
}

struct OpHistScan {  // exclusive scan of the radix histogram in place
    int* h;
    __device__ int count(int i) const { return h[i]; }
    __device__ void emit(int i, int off, int) const { h[i] = off; }
};

// Geometric blocks: positions where the block code (code >> 6) changes.
struct OpGBlocks {
    const uint32_t* keys;
    int N;
    int* gstart;
    uint32_t* gcode;
    __device__ int count(int j) const { return (j == 0 || (keys[j] >> 6) != (keys[j - 1] >> 6)) ? 1 : 0; }
    __device__ void emit(int j, int off, int) const {
        gstart[off] = j;
        gcode[off] = keys[j] >> 6;
    }
};

// Merge groups: runs of geometric blocks of one 2x2x1 slab of blocks (equal
// code >> 2; the rank bits make groups never cross scenes).
struct OpGroups {
    const uint32_t* gcode;
    int* group_start;
    const int* ctl;
    int pack;  // 0: every block is a group of its own (one block per chunk)
    __device__ int count(int g) const {
        if (g >= ctl[CTL_NGB]) return 0;
        return (g == 0 || !pack || (gcode[g] >> 2) != (gcode[g - 1] >> 2)) ? 1 : 0;
    }
    __device__ void emit(int g, int off, int) const { group_start[off] = g; }
};

// Work chunks, per merge group: consecutive blocks are packed into one chunk
// while the total stays within `chunk` particles; a block larger than that
// is cut into runs of `chunk`.  (Sparse regions then still fill the
// workgroups; a chunk's tile box stays within a 2x2x1 slab of blocks.)
struct OpChunks {
    const int* gstart;
    const uint32_t* gcode;
    const int* group_start;
    const int* ctl;
    int N, chunk;
    Chunk* out;
    Scenes T;
    __device__ int len(int g) const {
        const int ng = ctl[CTL_NGB];
        const int end = (g + 1 < ng) ? gstart[g + 1] : N;
        return end - gstart[g];
    }
    __device__ int group_end(int s) const { return s + 1 < ctl[CTL_NGROUP] ? group_start[s + 1] : ctl[CTL_NGB]; }
    // walk the group's blocks, calling put(start, count, first block) for each chunk
    template <class Put>
    __device__ int walk(int s, Put put) const {
        int k = 0, run0 = -1, runn = 0, runb = 0;
        for (int g = group_start[s]; g < group_end(s); ++g) {
            const int l = len(g);
            if (l > chunk) {
                if (runn) put(k++, run0, runn, runb);
                runn = 0;
                for (int i = 0; i < l; i += chunk) put(k++, gstart[g] + i, min(chunk, l - i), g);
            } else {
                if (runn && runn + l > chunk) {
                    put(k++, run0, runn, runb);
                    runn = 0;
                }
                if (!runn) {
                    run0 = gstart[g];
                    runb = g;
                }
                runn += l;
            }
        }
        if (runn) put(k++, run0, runn, runb);
        return k;
    }
    __device__ int count(int s) const {
        if (s >= ctl[CTL_NGROUP]) return 0;
        return walk(s, [](int, int, int, int) {});
    }
    __device__ void emit(int s, int off, int) const {
        const int bshift = T.shift - 6;
        walk(s, [&](int k, int start, int n, int g) {
            Chunk c;
            c.start = start;
            c.count = n;
            c.tile = 1;
            c.scene = T.rank_scene[gcode[g] >> bshift];
            out[off + k] = c;
        });
    }
};

struct OpActive {
    const int* state;
    int* active;
    __device__ int count(int b) const { return state[b] != 0 ? 1 : 0; }
    __device__ void emit(int b, int off, int) const { active[off] = b; }
};

// ------------------------------------------------------------ data movement
// Slot of rank r when a chunk's `count` particles are dealt over its 16-lane
// passes (pass k = slots 16k .. 16k+15; the last pass holds the remainder):
// rank r goes to place q = r / P of pass r mod P in the order 0, 2, 4, ...,
// 1, 3, 5, ... (P passes; places of the short last pass run out first), so
// consecutive ranks land in different passes, mostly two passes (32 lanes)
// apart.
__device__ __forceinline__ int dealt_slot(int count, int r) {
    const int P = (count + 15) >> 4, last = count - 16 * (P - 1), E = (P + 1) >> 1;
    int q, i, evens = E;
    if (r < last * P) {
        q = r / P;
        i = r - q * P;
    } else {
        const int r2 = r - last * P, Pm = P - 1;
        q = last + r2 / Pm;
        i = r2 - (q - last) * Pm;
        if (P & 1) evens = E - 1;  // the last pass is the last even one: drop it
    }
    const int pass = i < evens ? 2 * i : 2 * (i - evens) + 1;
    return pass * 16 + q;
}

// Gather the whole particle state into sorted order, one chunk per
// workgroup.  A chunk holds one to four blocks (segments of its sorted run).
// Unless `spread` is 0 (plain sorted order), the chunk's particles are
// ranked by the LDS bank pair of their cell in the P2G tile -- (x + 12 y +
// 8 z) mod 16 for cell (x, y, z), the tile's layout with a row pitch of 12
// (mod 16) and a plane pitch of 8 (mod 16) -- then by cell, and dealt over
// the 16-lane passes of the P2G scatter: a pass then meets each bank pair
// about as often as the chunk's cells allow, and particles of one cell sit in
// different passes.  Each particle's field FSID gets its block (its free
// zone).  Also records the insertion ids in plain sorted order for the
// binning view.
constexpr int PERMUTE_MAX = 512;  // the largest chunk
__global__ __launch_bounds__(WG) void k_permute_chunks(const float* __restrict__ Sin, float* __restrict__ Sout,
                                                       const int* __restrict__ idin, int* __restrict__ idout,
                                                       int* __restrict__ sorted_ids, const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ keys,
                                                       const Chunk* __restrict__ chunks, const int* __restrict__ ctl,
                                                       int64_t cap, int spread, int shift) {
    constexpr int NRK = 4096;  // ranking keys: 4-bit bank pair, 8-bit segment and cell
    __shared__ int rk[PERMUTE_MAX];
    __shared__ int below[NRK];  // per ranking key: how many of the chunk's particles rank lower
    const int nch = ctl[CTL_NCHUNK];
    const uint32_t mmask = (1u << shift) - 1u;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = chunks[c];
        const bool deal = spread && ch.count <= PERMUTE_MAX;  // workgroup-uniform
        if (deal) {
            // a counting sort of the ranking keys: histogram, then its exclusive prefix sums
            for (int t = threadIdx.x; t < NRK; t += WG) below[t] = 0;
            __syncthreads();
            for (int t = threadIdx.x; t < ch.count; t += WG) {
                const uint32_t key = keys[ch.start + t] & mmask;
                const uint32_t bcode = key >> 6, cell = key & 63u;
                const int x = 4 * (int)compact3(bcode) + (int)compact3(cell);
                const int y = 4 * (int)compact3(bcode >> 1) + (int)compact3(cell >> 1);
                const int z = 4 * (int)compact3(bcode >> 2) + (int)compact3(cell >> 2);
                rk[t] = (((x + 12 * y + 8 * z) & 15) << 8) | (int)(key & 255u);  // bank, segment, cell
                atomicAdd(&below[rk[t]], 1);
            }
            __syncthreads();
            constexpr int PER = NRK / WG;
            int h[PER], sum = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                h[k] = below[threadIdx.x * PER + k];
                sum += h[k];
            }
            int total;
            int run = block_excl_scan(sum, &total);
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                below[threadIdx.x * PER + k] = run;
                run += h[k];
            }
            __syncthreads();
        }
        for (int t = threadIdx.x; t < ch.count; t += WG) {
            const int j = ch.start + t;  // sorted position
            const uint32_t key = keys[j];
            int slot = t;
            if (deal) {
                // rank = the particles with a lower ranking key + those before it with the same one.
                // Within a chunk (blocks of one 2x2x1 slab) the segment and cell bits identify the
                // particle code, so equal ranking keys are a run of equal codes, consecutive in
                // sorted order.
                const int mine = rk[t];
                int first = t;
                while (first > 0 && rk[first - 1] == mine) --first;
                slot = dealt_slot(ch.count, below[mine] + (t - first));
            }
            const int k = (int)src[j];  // its position before the sort
            const int dst = ch.start + slot;
#pragma unroll
            for (int f = 0; f < FSID; ++f) Sout[sidx(f, dst, cap)] = Sin[sidx(f, k, cap)];
            const uint32_t bcode = (key & mmask) >> 6;
            const int scene = fsid_scene(Sin[sidx(FSID, k, cap)]);
            Sout[sidx(FSID, dst, cap)] = __int_as_float(scene | (int)(compact3(bcode) << 8) |
                                                    (int)(compact3(bcode >> 1) << 16) |
                                                    (int)(compact3(bcode >> 2) << 24));
            const int id = idin[k];
            idout[dst] = id;
            sorted_ids[j] = id;
        }
        if (deal) __syncthreads();
    }
}

__global__ __launch_bounds__(WG) void k_copy_codes(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                   int n, uint32_t mask) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < n) dst[i] = src[i] & mask;
}

__global__ __launch_bounds__(WG) void k_fill(int* __restrict__ p, int v, int n) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < n) p[i] = v;
}

// Mark the 3x3x3 neighbourhood of every geometric block as physical, in
// the block grid of the block's scene.
__global__ __launch_bounds__(WG) void k_dilate(const uint32_t* __restrict__ gcode, const int* __restrict__ ctl,
                                               Scenes T, int* __restrict__ state) {
    const int total = ctl[CTL_NGB] * 27;
    const int bshift = T.shift - 6;
    for (int t = blockIdx.x * WG + threadIdx.x; t < total; t += gridDim.x * WG) {
        const int g = t / 27, o = t % 27;
        const uint32_t code = gcode[g] & ((1u << bshift) - 1u);
        const Scene& sc = T.scene[T.rank_scene[gcode[g] >> bshift]];
        const int NB = sc.P.NB;
        const int B0 = (int)compact3(code), B1 = (int)compact3(code >> 1), B2 = (int)compact3(code >> 2);
        const int bx = B0 + (o % 3);  // (B - 1) + o + 1 in padded coordinates
        const int by = B1 + (o / 3) % 3;
        const int bz = B2 + o / 9;
        state[sc.brick_base + (bz * NB + by) * NB + bx] = 1;
    }
}

// After compaction a physical block's state names its position in the active
// list (3 + i), under which the rebuild lists the chunks whose tiles can reach
// it.
__global__ __launch_bounds__(WG) void k_mark_active(const int* __restrict__ active, const int* __restrict__ ctl,
                                                    int* __restrict__ state) {
    const int n = ctl[CTL_NACTIVE];
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) state[active[i]] = 3 + i;
}

// Per-rank ends of the sorted particles, geometric blocks, chunks and
// physical blocks (binary searches over the rank-major lists).
__global__ __launch_bounds__(WG) void k_rank_ends(const uint32_t* __restrict__ keys, int N,
                                                  const uint32_t* __restrict__ gcode, const Chunk* __restrict__ chunks,
                                                  const int* __restrict__ active, const int* __restrict__ ctl,
                                                  Scenes T) {
    for (int r = threadIdx.x; r < T.S; r += WG) {
        auto upper = [&](int n, auto rank_at) {  // first index whose rank exceeds r
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rank_at(mid) <= r)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            return lo;
        };
        T.rank_end[RE_PART * T.S + r] = upper(N, [&](int i) { return (int)(keys[i] >> T.shift); });
        T.rank_end[RE_GBLOCK * T.S + r] =
            upper(ctl[CTL_NGB], [&](int i) { return (int)(gcode[i] >> (T.shift - 6)); });
        T.rank_end[RE_CHUNK * T.S + r] = upper(ctl[CTL_NCHUNK], [&](int i) { return T.scene[chunks[i].scene].rank; });
        T.rank_end[RE_ACTIVE * T.S + r] =
            upper(ctl[CTL_NACTIVE], [&](int i) { return active[i] >= T.rank_brick[r + 1] ? r + 1 : r; });
    }
}

// The rebuild also starts the overflow lists and fallback counts afresh.
// Tile registrations, one wave per chunk: the chunk's particle blocks (the
// blocks of its sorted range, at most the four of one 2x2x1 slab) reach
// padded blocks B .. B+2 per axis with in-zone stencils; the chunk is listed
// with each physical block of that region.  A full list clears the chunk's
// `tile` flag.
__global__ __launch_bounds__(WG) void k_register(Chunk* __restrict__ chunks, const uint32_t* __restrict__ keys,
                                                 const int* __restrict__ ctl, const int* __restrict__ state,
                                                 int* __restrict__ reg_n, int* __restrict__ reg, Scenes T) {
    const int nch = ctl[CTL_NCHUNK];
    const int lane = threadIdx.x & 63;
    const uint32_t mmask = (1u << T.shift) - 1u;
    for (int c = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); c < nch; c += gridDim.x * (WG / 64)) {
        const Chunk ch = chunks[c];
        const Scene& sc = T.scene[ch.scene];
        const int NB = sc.P.NB;
        const uint32_t b0 = (keys[ch.start] & mmask) >> 6, b1 = (keys[ch.start + ch.count - 1] & mmask) >> 6;
        int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
        for (uint32_t b = b0; b <= b1; ++b) {  // Morton codes of one slab: at most four
            const int q[3] = {(int)compact3(b), (int)compact3(b >> 1), (int)compact3(b >> 2)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = min(lo[a], q[a]);
                hi[a] = max(hi[a], q[a] + 2);
            }
        }
        const int n0 = hi[0] - lo[0] + 1, n1 = hi[1] - lo[1] + 1, n2 = hi[2] - lo[2] + 1;
        bool fail = false;
        for (int k = lane; k < n0 * n1 * n2; k += 64) {
            const int bx = lo[0] + k % n0, by = lo[1] + (k / n0) % n1, bz = lo[2] + k / (n0 * n1);
            const int s = state[sc.brick_base + (bz * NB + by) * NB + bx];
            if (s >= 3) {
                const int slot = atomicAdd(&reg_n[s - 3], 1);
                if (slot < REG_MAX)
                    reg[(int64_t)(s - 3) * REG_MAX + slot] = c;
                else
                    fail = true;
            }
        }
        if (__ballot(fail) != 0ull && lane == 0) chunks[c].tile = 0;
    }
}

// Each physical block's registration list in ascending chunk order (one wave
// per block; a lane's rank is the count of smaller entries), so the grid
// update sums the tiles in a fixed order.
__global__ __launch_bounds__(WG) void k_sort_registrations(const int* __restrict__ ctl, const int* __restrict__ reg_n,
                                                           int* __restrict__ reg) {
    __shared__ int buf[WG / 64][REG_MAX];
    const int nact = ctl[CTL_NACTIVE];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = blockIdx.x * (WG / 64) + wv; i < nact; i += gridDim.x * (WG / 64)) {
        const int m = min(__builtin_amdgcn_readfirstlane(reg_n[i]), REG_MAX);
        int* list = reg + (int64_t)i * REG_MAX;
        for (int k = lane; k < m; k += 64) buf[wv][k] = list[k];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        int v[REG_MAX / 64], r[REG_MAX / 64];
#pragma unroll
        for (int u = 0; u < REG_MAX / 64; ++u) {
            const int k = lane + 64 * u;
            v[u] = k < m ? buf[wv][k] : 0;
            r[u] = 0;
        }
        for (int j = 0; j < m; ++j) {  // entries are distinct chunk indices
            const int e = buf[wv][j];
#pragma unroll
            for (int u = 0; u < REG_MAX / 64; ++u) r[u] += e < v[u] ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < REG_MAX / 64; ++u)
            if (lane + 64 * u < m) list[r[u]] = v[u];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
}

__global__ void k_finish_rebuild(int* ctl) {
    ctl[CTL_REBUILD] = 0;
    ctl[CTL_OVF] = ctl[CTL_OVF + 1] = 0;
    ctl[CTL_FB] = ctl[CTL_FB + 1] = 0;
}

}  // namespace

// The overflow-block and tile-fallback counts of both substep parities
// cleared between substeps, as a rebuild leaves them (a graph frame without
// a rebuild starts with this).
__global__ void k_clear_overflow(int* ctl) {
    ctl[CTL_OVF] = ctl[CTL_OVF + 1] = 0;
    ctl[CTL_FB] = ctl[CTL_FB + 1] = 0;
}

void enqueue_clear_overflow(hipStream_t st, int* ctl) {
    hipLaunchKernelGGL(k_clear_overflow, dim3(1), dim3(1), 0, st, ctl);
}

void enqueue_copy_codes(hipStream_t st, uint32_t* dst, const uint32_t* src, int count, uint32_t mask) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_copy_codes, dim3(cdiv(count, WG)), dim3(WG), 0, st, dst, src, count, mask);
}

void enqueue_rebuild(hipStream_t st, const Scenes& T, float* S_cur, float* S_alt, int* id_cur, int* id_alt,
                     int64_t cap, int N, int chunk, int spread, int pack, BinBuffers& B, int* ctl, int nbricks,
                     int key_bits,
                     int* reg_n, int* reg) {
    const int nb = cdiv(N > 0 ? N : 1, WG);
    // 1. particle codes
    hipLaunchKernelGGL(k_keys, dim3(nb), dim3(WG), 0, st, S_cur, cap, N, T, B.keys[0], B.vals[0], ctl);
    // 2. stable radix sort of (code, position)
    const int passes = (key_bits + 7) / 8;
    const int tiles = cdiv(N > 0 ? N : 1, RS_TILE);
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(WG), 0, st, B.keys[cur], N, 8 * p, tiles, B.hist);
        device_scan(st, OpHistScan{B.hist}, 256 * tiles, B.scan_tiles, ctl + CTL_SCAN);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(WG), 0, st, B.keys[cur], B.vals[cur], B.keys[cur ^ 1],
                           B.vals[cur ^ 1], N, 8 * p, tiles, B.hist);
        cur ^= 1;
    }
    B.sorted = cur;  // slot holding the sorted codes and their source positions
    // 3. geometric blocks and work chunks
    device_scan(st, OpGBlocks{B.keys[cur], N, B.gstart, B.gcode}, N, B.scan_tiles, ctl + CTL_NGB);
    device_scan(st, OpGroups{B.gcode, B.group_start, ctl, pack}, N, B.scan_tiles, ctl + CTL_NGROUP);
    device_scan(st, OpChunks{B.gstart, B.gcode, B.group_start, ctl, N, chunk, B.chunks, T}, N, B.scan_tiles,
                ctl + CTL_NCHUNK);
    // 4. gather the whole particle state into (chunk-spread) sorted order
    hipLaunchKernelGGL(k_permute_chunks, dim3(2048), dim3(WG), 0, st, S_cur, S_alt, id_cur, id_alt, B.sorted_ids,
                       B.vals[cur], B.keys[cur], B.chunks, ctl, cap, spread, T.shift);
    // 5. physical blocks: 3x3x3 dilation, compacted in padded linear order
    hipLaunchKernelGGL(k_fill, dim3(cdiv(nbricks, WG)), dim3(WG), 0, st, B.brick_state, 0, nbricks);
    hipLaunchKernelGGL(k_dilate, dim3(512), dim3(WG), 0, st, B.gcode, ctl, T, B.brick_state);
    device_scan(st, OpActive{B.brick_state, B.active}, nbricks, B.scan_tiles, ctl + CTL_NACTIVE);
    hipLaunchKernelGGL(k_mark_active, dim3(512), dim3(WG), 0, st, B.active, ctl, B.brick_state);
    // 6. tile registrations of the chunks with the physical blocks
    hipLaunchKernelGGL(k_fill, dim3(cdiv(nbricks, WG)), dim3(WG), 0, st, reg_n, 0, nbricks);
    hipLaunchKernelGGL(k_register, dim3(1024), dim3(WG), 0, st, B.chunks, B.keys[cur], ctl, B.brick_state, reg_n, reg,
                       T);
    hipLaunchKernelGGL(k_sort_registrations, dim3(1024), dim3(WG), 0, st, ctl, reg_n, reg);
    hipLaunchKernelGGL(k_finish_rebuild, dim3(1), dim3(1), 0, st, ctl);
    hipLaunchKernelGGL(k_rank_ends, dim3(1), dim3(WG), 0, st, B.keys[cur], N, B.gcode, B.chunks, B.active, ctl, T);
}

}  // namespace mpm
