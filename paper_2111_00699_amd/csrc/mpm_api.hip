// Host runtime behind the C ABI of include/mpm.h.
//
// Capacity: particle buffers grow 4x once more than half full, and only in
// mpm_add_particles (paper, "Principles": a vector that reserves ahead
// avoids reallocation during the simulation; scan/sort scratch is allocated
// up front).  The dense block grids of all scenes are allocated once at
// creation, in one brick space laid out in rank order.
//
// Rebuild scheduling without draining the stream: G2P sets a device flag when
// a particle leaves its free zone and, the first time, writes it to a pinned
// host ring slot of that substep; an event marks the end of every group of
// substeps (four with the default lag: an event on the stream delays the next
// kernel by about 6 us, which per substep cost 3% of the snow frame).  Before
// enqueueing substep k the host reads the slots of the groups that have
// finished, waiting only for the group of substep k - lag (its last substep is
// at most k - lag + 3), so the device keeps at least lag - 4 substeps queued
// (one with the default lag of 5).  A particle that leaves its free zone
// before the rebuild lands is still transferred exactly (through global
// atomics), so the lag costs speed, never correctness.
//
// Batched scenes: every scene is a rank in one particle-code order, so each
// phase of a substep is one launch over all scenes; a frame gives scene s
// ceil(frame_dt / dt_s) substeps, and because ranks follow increasing dt the
// scenes still running at a given substep of the frame are a prefix of the
// ranks (`act`).  With MPM_FLAG_FRAME_GRAPHS a frame -- rebuild, then all
// substeps -- is recorded once per particle-buffer parity as a HIP graph and
// replayed.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "mpm_internal.h"
#include "mpm_surrogate.h"

using namespace mpm;

namespace {

constexpr int RING = 128;
constexpr int PROF_SLOTS = 4096;

std::string g_create_error;

struct SceneHost {
    mpm_scene desc{};
    mpm_material mat{};
    bool has_mat = false;
    int64_t N = 0;             // particles of the scene
    int64_t N_at_rebuild = 0;  // ... at the last rebuild
    int64_t substeps = 0;
    int64_t last_step = -2;    // index of its last substep (stamp of the blocks it updated)
};

struct FrameGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t N = -1;
    float frame_dt = 0.0f;
    int chunk = 0;
};

}  // namespace

struct mpm_ctx {
    mpm_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    int nsc = 1;                      // scenes
    std::vector<SceneHost> sh;        // by scene index
    std::vector<int> rank_scene;      // scene index of each rank
    std::vector<Scene> table;         // host copy of the device scene table
    Scene* scene_dev = nullptr;
    int* rank_scene_dev = nullptr;
    int* rank_brick_dev = nullptr;    // [S + 1]
    int* rank_end_dev = nullptr;      // [4 S]
    int shift = 0, key_bits = 0;
    int nbricks = 0;
    Launch L{};

    int64_t N = 0, cap = 0;
    int cur = 0;  // which particle buffer is current
    float* S[2] = {nullptr, nullptr};
    int* ids[2] = {nullptr, nullptr};
    BinBuffers B{};
    GridBuffers G{};
    int* ctl = nullptr;

    int* ring = nullptr;      // pinned host flags
    int* ring_dev = nullptr;  // device view of the same memory
    hipEvent_t ev[RING] = {};

    int64_t step = 0, checked = 0, last_rebuild = -1, rebuilds = 0;
    int64_t parity_ctr = 0;  // parity of the next substep (overflow-list slot)
    int64_t n_at_rebuild = 0;
    bool need_rebuild = true;
    int pending = 0;
    // The G2P of the last substep of ranks [0, g2p_due_act) has not run yet:
    // the next substep's P2G runs it first (fused), or bring_up_to_date()
    // does before the state is read, extended, sampled or rebuilt.
    int g2p_due_act = 0;
    // frame graphs by particle-buffer parity and by whether the frame starts with a rebuild
    FrameGraph graphs[2][2];
    hipEvent_t graph_done = nullptr;  // recorded after the last graph frame
    bool graph_inflight = false;
    // snow return map without SVD (see mpm_use_surrogate)
    const float* sur_theta = nullptr;
    const float* sur_norm = nullptr;
    float sur_tol = 1e-3f, sur_dt_ref = 1.0f;
    int sur_any = 0;
    // ASFLIP (mpm_set_transfer) and the automatic frame time step (mpm_set_auto_dt)
    bool any_flip = false;
    float auto_cfl = 0.0f, auto_dt_max = 0.0f;
    float* speed_dev = nullptr;  // [0..1]: the largest particle speed and the sum of speeds (auto dt,
                                 // exit horizon); [2..3]: the same, reduced at the end of each graph frame
    bool graph_speed = false;    // ring[RING + 1 ..] holds the speeds at the end of the last frame

    // profiling
    uint32_t prof_mask = 0;
    struct Pair {
        hipEvent_t a, b;
        int phase;
        bool live;
    };
    std::vector<Pair> prof;
    int prof_next = 0;
    int64_t prof_launch[4] = {0, 0, 0, 0};
    uint32_t prof_every = 1;                 // bracket every prof_every-th launch of a phase
    int64_t prof_seen[4] = {0, 0, 0, 0};     // launches of each phase since mpm_profile
    double prof_ms[4] = {0, 0, 0, 0};

    std::string err;
};

namespace {

int fail(mpm_ctx* c, int code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return code;
}

#define HIP_OK(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), e_ == hipErrorOutOfMemory ? MPM_ENOMEM : MPM_EDEVICE,            \
                        std::string(#call) + ": " + hipGetErrorString(e_));                      \
    } while (0)

Mat derive_material(const mpm_material& m, const Step& P) {
    Mat M{};
    M.kind = m.kind;
    M.mu = m.E / (2.0f * (1.0f + m.nu));
    M.la = m.E * m.nu / ((1.0f + m.nu) * (1.0f - 2.0f * m.nu));
    const double dx = 1.0 / P.n;
    const double V0 = dx * dx * dx / m.ppc;
    M.mp = (float)(m.rho * V0);
    M.scale = (float)(4.0 * P.dt * V0 / (dx * dx));
    M.lo = 1.0f - m.theta_c;
    M.hi = 1.0f + m.theta_s;
    M.xi = m.xi;
    M.bulk = m.bulk;
    const float deg = 3.14159265358979f / 180.0f;
    M.h0 = m.h0 * deg;
    M.h1 = m.h1 * deg;
    M.h2 = m.h2;
    M.h3 = m.h3 * deg;
    M.kdp = (3.0f * M.la + 2.0f * M.mu) / (2.0f * M.mu);
    return M;
}

bool same_material(const mpm_material& a, const mpm_material& b) {
    return a.kind == b.kind && a.E == b.E && a.nu == b.nu && a.rho == b.rho && a.ppc == b.ppc &&
           a.theta_c == b.theta_c && a.theta_s == b.theta_s && a.xi == b.xi && a.bulk == b.bulk && a.h0 == b.h0 &&
           a.h1 == b.h1 && a.h2 == b.h2 && a.h3 == b.h3;
}

Step make_step(const mpm_scene& d) {
    Step P{};
    P.n = d.n;
    P.NB = d.n / 4 + 2;
    P.fn = (float)d.n;
    P.dx = 1.0f / (float)d.n;
    P.dt = d.dt;
    P.g0 = d.gravity[0];
    P.g1 = d.gravity[1];
    P.g2 = d.gravity[2];
    P.bc = d.bc;
    P.bc_cells = d.bc_cells;
    return P;
}

const char* check_scene(const mpm_scene& d) {
    if (d.n < 16 || d.n > 512 || (d.n & (d.n - 1))) return "n must be a power of two in [16, 512]";
    if (d.bc < 0 || d.bc > 2) return "bad bc";
    if (d.bc_cells < 0 || d.bc_cells > d.n / 2) return "bad bc_cells";
    if (!(d.dt > 0.0f)) return "dt must be positive";
    return nullptr;
}

int log2i(int v) {
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

Scenes tables(const mpm_ctx* c) {
    Scenes T{c->scene_dev, c->rank_scene_dev, c->rank_brick_dev, c->rank_end_dev, c->nsc, c->shift};
    T.sur_theta = c->sur_theta;
    T.sur_norm = c->sur_norm;
    T.sur_tol = c->sur_tol;
    T.sur_gap = 0.1f;
    T.sur_dt_ref = c->sur_dt_ref;
    T.sur_any = c->sur_any;
    return T;
}

int scan_tiles_needed(int64_t cap, int nbricks) {
    int64_t rs_tiles = (cap + 4095) / 4096;
    int64_t m = cap;
    if (nbricks > m) m = nbricks;
    if (256 * rs_tiles > m) m = 256 * rs_tiles;
    return (int)((m + 2047) / 2048) + 1;
}

void free_particle_buffers(mpm_ctx* c) {
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(c->S[i]);
        (void)hipFree(c->ids[i]);
        (void)hipFree(c->B.keys[i]);
        (void)hipFree(c->B.vals[i]);
        c->S[i] = nullptr;
        c->ids[i] = nullptr;
        c->B.keys[i] = c->B.vals[i] = nullptr;
    }
    (void)hipFree(c->B.hist);
    (void)hipFree(c->B.scan_tiles);
    (void)hipFree(c->B.gstart);
    (void)hipFree(c->B.gcode);
    (void)hipFree(c->B.chunks);
    (void)hipFree(c->B.group_start);
    (void)hipFree(c->B.sorted_ids);
    (void)hipFree(c->G.stage);
    (void)hipFree(c->G.box);
    c->B.group_start = c->B.sorted_ids = nullptr;
    c->G.stage = nullptr;
    c->G.box = nullptr;
    c->B.hist = c->B.scan_tiles = c->B.gstart = nullptr;
    c->B.gcode = nullptr;
    c->B.chunks = nullptr;
}

// Allocate particle-sized buffers for `newcap`, keeping the current state.
int grow(mpm_ctx* c, int64_t newcap) {
    newcap = (newcap + 255) / 256 * 256;  // whole groups of the grouped layout, aligned arrays
    float* S[2] = {nullptr, nullptr};
    int* ids[2] = {nullptr, nullptr};
    uint32_t *keys[2] = {nullptr, nullptr}, *vals[2] = {nullptr, nullptr};
    int *hist = nullptr, *tiles = nullptr, *gstart = nullptr;
    uint32_t* gcode = nullptr;
    Chunk* chunks = nullptr;
    int *group_start = nullptr, *sorted_ids = nullptr;
    float4* stage = nullptr;
    int4* box = nullptr;
    const int64_t rs_tiles = (newcap + 4095) / 4096;
    // P2G staging: 16 nodes per particle of capacity (a block-sized chunk stages about one node per
    // particle) plus two full tiles per P2G workgroup, so small systems never run short.
    int64_t stage_nodes = 16 * newcap + 2 * 512 * (int64_t)c->L.p2g_grid;
    if (stage_nodes > (int64_t)INT32_MAX - 4096) stage_nodes = (int64_t)INT32_MAX - 4096;
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) {
        ok = ok && hipMalloc(&S[i], sizeof(float) * NF * newcap) == hipSuccess;
        ok = ok && hipMalloc(&ids[i], sizeof(int) * newcap) == hipSuccess;
        ok = ok && hipMalloc(&keys[i], sizeof(uint32_t) * newcap) == hipSuccess;
        ok = ok && hipMalloc(&vals[i], sizeof(uint32_t) * newcap) == hipSuccess;
    }
    ok = ok && hipMalloc(&hist, sizeof(int) * 256 * rs_tiles) == hipSuccess;
    ok = ok && hipMalloc(&tiles, sizeof(int) * scan_tiles_needed(newcap, c->nbricks)) == hipSuccess;
    ok = ok && hipMalloc(&gstart, sizeof(int) * (newcap + 1)) == hipSuccess;
    ok = ok && hipMalloc(&gcode, sizeof(uint32_t) * (newcap + 1)) == hipSuccess;
    ok = ok && hipMalloc(&chunks, sizeof(Chunk) * (newcap + 1)) == hipSuccess;
    ok = ok && hipMalloc(&group_start, sizeof(int) * (newcap + 2)) == hipSuccess;
    ok = ok && hipMalloc(&sorted_ids, sizeof(int) * newcap) == hipSuccess;
    ok = ok && hipMalloc(&stage, sizeof(float4) * (stage_nodes + 1)) == hipSuccess;
    ok = ok && hipMalloc(&box, sizeof(int4) * (newcap + 1)) == hipSuccess;
    if (!ok) {
        for (int i = 0; i < 2; ++i) {
            (void)hipFree(S[i]);
            (void)hipFree(ids[i]);
            (void)hipFree(keys[i]);
            (void)hipFree(vals[i]);
        }
        (void)hipFree(hist);
        (void)hipFree(tiles);
        (void)hipFree(gstart);
        (void)hipFree(gcode);
        (void)hipFree(chunks);
        (void)hipFree(group_start);
        (void)hipFree(sorted_ids);
        (void)hipFree(stage);
        (void)hipFree(box);
        (void)hipGetLastError();
        return fail(c, MPM_ENOMEM, "particle buffer allocation failed for capacity " + std::to_string(newcap));
    }
    if (c->N > 0) {
#if MPM_AOSOA  // the groups of the first N particles do not depend on the capacity
        HIP_OK(c, hipMemcpyAsync(S[0], c->S[c->cur], sizeof(float) * NF * ((c->N + AOSOA_B - 1) / AOSOA_B * AOSOA_B),
                                 hipMemcpyDeviceToDevice, c->stream));
#else
        HIP_OK(c, hipMemcpy2DAsync(S[0], sizeof(float) * newcap, c->S[c->cur], sizeof(float) * c->cap,
                                   sizeof(float) * c->N, NF, hipMemcpyDeviceToDevice, c->stream));
#endif
        HIP_OK(c, hipMemcpyAsync(ids[0], c->ids[c->cur], sizeof(int) * c->N, hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_OK(c, hipMemsetAsync(box, 0, sizeof(int4) * (newcap + 1), c->stream));
    HIP_OK(c, hipMemsetAsync(stage + stage_nodes, 0, sizeof(float4), c->stream));  // the zero node
    HIP_OK(c, hipStreamSynchronize(c->stream));
    free_particle_buffers(c);
    for (int i = 0; i < 2; ++i) {
        c->S[i] = S[i];
        c->ids[i] = ids[i];
        c->B.keys[i] = keys[i];
        c->B.vals[i] = vals[i];
    }
    c->B.hist = hist;
    c->B.scan_tiles = tiles;
    c->B.gstart = gstart;
    c->B.gcode = gcode;
    c->B.chunks = chunks;
    c->B.group_start = group_start;
    c->B.sorted_ids = sorted_ids;
    c->G.stage = stage;
    c->G.stage_nodes = (int)stage_nodes;
    c->G.box = box;
    c->cur = 0;
    c->cap = newcap;
    c->need_rebuild = true;
    return MPM_OK;
}

// --------------------------------------------------------------- profiling
int prof_accumulate(mpm_ctx* c, mpm_ctx::Pair& p) {
    if (!p.live) return MPM_OK;
    HIP_OK(c, hipEventSynchronize(p.b));
    float ms = 0.0f;
    HIP_OK(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->prof_ms[p.phase] += ms;
    c->prof_launch[p.phase] += 1;
    p.live = false;
    return MPM_OK;
}

int prof_begin(mpm_ctx* c, int phase, int* slot) {
    *slot = -1;
    if (!(c->prof_mask & (1u << phase))) return MPM_OK;
    if (c->prof_seen[phase]++ % c->prof_every != 0) return MPM_OK;
    if (c->prof.empty()) {
        c->prof.resize(PROF_SLOTS);
        for (auto& p : c->prof) {
            HIP_OK(c, hipEventCreate(&p.a));
            HIP_OK(c, hipEventCreate(&p.b));
            p.live = false;
        }
    }
    auto& p = c->prof[c->prof_next];
    int r = prof_accumulate(c, p);
    if (r) return r;
    p.phase = phase;
    HIP_OK(c, hipEventRecord(p.a, c->stream));
    *slot = c->prof_next;
    c->prof_next = (c->prof_next + 1) % PROF_SLOTS;
    return MPM_OK;
}

int prof_end(mpm_ctx* c, int slot) {
    if (slot < 0) return MPM_OK;
    auto& p = c->prof[slot];
    HIP_OK(c, hipEventRecord(p.b, c->stream));
    p.live = true;
    return MPM_OK;
}

// Substeps close their group of ev_every(c) with an event (a marker costs the
// stream a few microseconds between kernels, so not every substep records one).
int ev_every(const mpm_ctx* c) { return c->cfg.lag >= 5 ? 4 : c->cfg.lag >= 3 ? 2 : 1; }
bool closes_group(const mpm_ctx* c, int64_t t) { return ((t + 1) % ev_every(c)) == 0; }

// Read the rebuild flag of substep t (finished).
void read_flag(mpm_ctx* c, int64_t t) {
    if (__atomic_load_n(&c->ring[(int)(t % RING)], __ATOMIC_ACQUIRE) && t >= c->last_rebuild &&
        !(c->cfg.flags & MPM_FLAG_MANUAL_REBUILD))
        c->need_rebuild = true;
}

// Read the rebuild flags of finished substeps, waiting for the group that
// holds substep `must_upto` (the group's closing event is never more than
// ev_every - 1 substeps later; `must_upto` >= the last substep drains the
// stream instead).
int poll_flags(mpm_ctx* c, int64_t must_upto) {
    if (c->checked < c->step && must_upto >= c->step - 1) {
        HIP_OK(c, hipStreamSynchronize(c->stream));
        for (; c->checked < c->step; ++c->checked) read_flag(c, c->checked);
        return MPM_OK;
    }
    const int64_t k = ev_every(c);
    while (c->checked < c->step) {
        const int64_t t = (c->checked / k) * k + k - 1;  // the substep closing checked's group
        if (t >= c->step) break;                            // not enqueued yet
        const int slot = (int)(t % RING);
        if (c->checked <= must_upto) {
            hipError_t e;
            while ((e = hipEventQuery(c->ev[slot])) == hipErrorNotReady) {
            }
            if (e != hipSuccess) return fail(c, MPM_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
        } else {
            const hipError_t e = hipEventQuery(c->ev[slot]);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return fail(c, MPM_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
        }
        for (; c->checked <= t; ++c->checked) read_flag(c, c->checked);
    }
    return MPM_OK;
}


void drop_graphs(mpm_ctx* c) {
    for (auto& gp : c->graphs)
        for (auto& g : gp) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
            g = FrameGraph{};
        }
}

// Wait for the last graph frame and take over its rebuild request (the
// pinned word after the ring slots, which graph frames' kernels set when a
// particle leaves its free zone).
int settle_graph_frame(mpm_ctx* c) {
    if (!c->graph_inflight) return MPM_OK;
    HIP_OK(c, hipEventSynchronize(c->graph_done));
    c->graph_inflight = false;
    if (__atomic_load_n(c->ring + RING, __ATOMIC_ACQUIRE)) {
        c->need_rebuild = true;
        __atomic_store_n(c->ring + RING, 0, __ATOMIC_RELEASE);
    }
    return MPM_OK;
}

// Substeps each rank takes in a frame of length frame_dt (non-increasing in
// rank, since ranks follow increasing dt).
std::vector<int> frame_substeps(const mpm_ctx* c, float frame_dt) {
    std::vector<int> ns(c->nsc);
    for (int r = 0; r < c->nsc; ++r) {
        const double q = (double)frame_dt / (double)c->sh[c->rank_scene[r]].desc.dt;
        int n = (int)q;
        if (q - n > 1e-4) ++n;
        ns[r] = n < 1 ? 1 : n;
    }
    return ns;
}

int active_ranks(const std::vector<int>& ns, int k) {
    int a = 0;
    while (a < (int)ns.size() && ns[a] > k) ++a;
    return a;
}

// In-zone particles that may lose their chunk's tile in one substep before
// the next substep asks for a rebuild (1/256 of the particles).  With
// MPM_FLAG_MANUAL_REBUILD the request is ignored like the free-zone one.
int fb_limit(const mpm_ctx* c) { return (int)(c->N >> 8); }

// Rebuild from particle buffer `cur` into the other one.
void enqueue_rebuild_into_alt(mpm_ctx* c, int cur) {
    enqueue_rebuild(c->stream, tables(c), c->S[cur], c->S[cur ^ 1], c->ids[cur], c->ids[cur ^ 1], c->cap,
                    (int)c->N, c->cfg.chunk, (c->cfg.flags & MPM_FLAG_P2G_SORTED_LANES) ? 0 : 1,
                    (c->cfg.flags & MPM_FLAG_CHUNK_PER_BLOCK) ? 0 : 1, c->B, c->ctl, c->nbricks, c->key_bits,
                    c->G.reg_n, c->G.reg);
}
void enqueue_rebuild_into_alt(mpm_ctx* c) { enqueue_rebuild_into_alt(c, c->cur); }

void note_rebuild(mpm_ctx* c) {
    c->cur ^= 1;
    c->need_rebuild = false;
    c->last_rebuild = c->step;
    c->n_at_rebuild = c->N;
    for (auto& s : c->sh) s.N_at_rebuild = s.N;
    ++c->rebuilds;
}

void note_substep(mpm_ctx* c, int act) {
    for (int r = 0; r < act; ++r) {
        SceneHost& s = c->sh[c->rank_scene[r]];
        s.substeps += 1;
        s.last_step = c->step;
    }
    c->pending = 1;
    ++c->step;
    ++c->parity_ctr;
}

int check_error_word(mpm_ctx* c) {
    int h[CTL_WORDS];
    HIP_OK(c, hipMemcpyAsync(h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (h[CTL_ERROR]) {
        char buf[96];
        snprintf(buf, sizeof buf, "device error word 0x%x", (unsigned)h[CTL_ERROR]);
        return fail(c, MPM_ESTATE, buf);
    }
    return MPM_OK;
}

// Whether a substep may leave its G2P to the next substep's P2G (the fused
// kernel needs the LDS tile path, the exact return map and the node-box
// gather).  The paper keeps G2P2G below 100K particles (instruction-cache
// misses beyond that on its GPU); on gfx950 with the fixed-point tile it
// saves 8-10% of a frame at 6.6K-99K particles and 3% at 1.28M, so it is
// the default at every size.
// G2P may run inside the next substep's P2G (graph frames fuse within the
// frame and end with the G2P done).
bool fusion_allowed(const mpm_ctx* c) {
    const bool wanted = (c->cfg.flags & MPM_FLAG_FUSED_G2P) || !(c->cfg.flags & MPM_FLAG_SEPARATE_G2P);
    return wanted && !c->sur_any && !c->any_flip &&
           !(c->cfg.flags & (MPM_FLAG_P2G_GLOBAL_ATOMICS | MPM_FLAG_REBUILD_EVERY_STEP |
                             MPM_FLAG_G2P_GLOBAL_GATHER));
}

// Grid-update passes run as launches of their own (the kernel-merging
// ablations): bit 0 the wall condition, bit 1 the accumulator clearing.
int grid_separate(const mpm_ctx* c) {
    return ((c->cfg.flags & MPM_FLAG_SEPARATE_WALLS) ? 1 : 0) | ((c->cfg.flags & MPM_FLAG_SEPARATE_CLEAR) ? 2 : 0);
}

// P2G's launch for the current particle count.  query_launch sizes it at
// four times the resident workgroups, which evens out the chunks' uneven
// costs when there are several chunks per workgroup; with fewer chunks than
// half that many workgroups, twice the resident count does better (the
// workgroups without a chunk cost dispatch time): the fused P2G of 55,296
// sand particles takes 20.4 us with twice and 22.1 us with four times the
// resident count, and 30.7 us when the grid is cut to the chunk count.
Launch p2g_launch(const mpm_ctx* c) {
    Launch L = c->L;
    if (c->N / std::max(c->cfg.chunk, 64) <= L.p2g_grid / 2) L.p2g_grid = std::max(8, L.p2g_grid / 16 * 8);
    return L;
}

// Run the G2P that the last substep left to its successor (see g2p_due_act).
int bring_up_to_date(mpm_ctx* c) {
    if (!c->g2p_due_act) return MPM_OK;
    int slot;
    if (int r = prof_begin(c, 3, &slot)) return r;
    enqueue_g2p(c->stream, c->L, tables(c), c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->G, nullptr,
                (c->cfg.flags & MPM_FLAG_G2P_GLOBAL_GATHER) ? 0 : 1, 0, fb_limit(c), c->cfg.chunk, c->g2p_due_act, 0);
    if (int r = prof_end(c, slot)) return r;
    HIP_OK(c, hipGetLastError());
    c->g2p_due_act = 0;
    return MPM_OK;
}

// One substep of the first `act` ranks, enqueued directly (host-lagged
// rebuild decision, optional phase events).  When fusion is allowed the
// substep ends after its grid update and its G2P runs at the start of the
// next substep's P2G.
int substep_one(mpm_ctx* c, int act) {
    int r = settle_graph_frame(c);
    if (r) return r;
    c->graph_speed = false;  // the state moves on from the last graph frame's end
    if ((r = poll_flags(c, c->step - c->cfg.lag))) return r;
    int slot;
    const bool rebuild = c->need_rebuild || (c->cfg.flags & MPM_FLAG_REBUILD_EVERY_STEP);
    const bool fusable = fusion_allowed(c);
    if (c->g2p_due_act && (rebuild || !fusable || act > c->g2p_due_act)) {
        if ((r = bring_up_to_date(c))) return r;
    }
    const bool fused = fusable && c->g2p_due_act >= act;
    if (rebuild) {
        if ((r = prof_begin(c, 0, &slot))) return r;
        enqueue_rebuild_into_alt(c);
        if ((r = prof_end(c, slot))) return r;
        note_rebuild(c);
    }
    const int rs = (int)(c->step % RING);
    c->ring[rs] = 0;
    const int parity = (int)(c->parity_ctr & 1);
    const Scenes T = tables(c);
    if ((r = prof_begin(c, 1, &slot))) return r;
    enqueue_p2g(c->stream, p2g_launch(c), T, c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->G, c->B.brick_state,
                fused ? 1 : c->pending, parity, (c->cfg.flags & MPM_FLAG_P2G_GLOBAL_ATOMICS) ? 1 : 0, c->nbricks,
                c->cfg.chunk, act, fused ? 1 : 0, c->ring_dev + rs, fb_limit(c));
    if ((r = prof_end(c, slot))) return r;
    if ((r = prof_begin(c, 2, &slot))) return r;
    enqueue_grid(c->stream, c->L, T, c->B, c->ctl, c->G, parity, c->nbricks, act, grid_separate(c));
    if ((r = prof_end(c, slot))) return r;
    if (fusable) {
        c->g2p_due_act = std::max(c->g2p_due_act, act);
    } else {
        if ((r = prof_begin(c, 3, &slot))) return r;
        enqueue_g2p(c->stream, c->L, T, c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->G, c->ring_dev + rs,
                    (c->cfg.flags & MPM_FLAG_G2P_GLOBAL_GATHER) ? 0 : 1, parity, fb_limit(c), c->cfg.chunk, act, 1);
        if ((r = prof_end(c, slot))) return r;
    }
    HIP_OK(c, hipGetLastError());
    if (closes_group(c, c->step)) HIP_OK(c, hipEventRecord(c->ev[rs], c->stream));
    note_substep(c, act);
    return MPM_OK;
}

// A frame as a replayed graph.  Each particle-buffer parity has two
// recordings: with a rebuild at the frame start (into the other buffer) and
// without.  The host picks one from the rebuild request the previous graph
// frame left (it waits for that frame first), so rebuilds keep the free
// zone's cadence; a frame without one starts by clearing the overflow
// counts, as a rebuild does.  Inside the frame each substep's G2P runs within
// the next substep's P2G when fusion is allowed, and the frame ends with the
// G2P still due.  A recording holds for one particle count, frame length
// and chunk size.
// Record the frame graph of particle buffer `cur`, with or without the
// rebuild at its start.
int record_frame_graph(mpm_ctx* c, int cur, bool rebuild, float frame_dt, const std::vector<int>& ns) {
    FrameGraph& g = c->graphs[cur][rebuild ? 1 : 0];
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = FrameGraph{};
    const bool fuse = fusion_allowed(c);
    int* flag = c->ring_dev + RING;
    HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    if (rebuild)
        enqueue_rebuild_into_alt(c, cur);
    else
        enqueue_clear_overflow(c->stream, c->ctl);
    const int buf = rebuild ? cur ^ 1 : cur;
    const Scenes T = tables(c);
    const int lds_box = (c->cfg.flags & MPM_FLAG_G2P_GLOBAL_GATHER) ? 0 : 1;
    for (int k = 0; k < ns[0]; ++k) {
        const int act = active_ranks(ns, k);
        const int parity = k & 1;  // both overflow slots start cleared
        const bool fused = fuse && k > 0;
        enqueue_p2g(c->stream, p2g_launch(c), T, c->S[buf], c->cap, c->B.chunks, c->ctl, c->G, c->B.brick_state, 1,
                    parity, (c->cfg.flags & MPM_FLAG_P2G_GLOBAL_ATOMICS) ? 1 : 0, c->nbricks, c->cfg.chunk, act,
                    fused ? 1 : 0, flag, fb_limit(c));
        enqueue_grid(c->stream, c->L, T, c->B, c->ctl, c->G, parity, c->nbricks, act, grid_separate(c));
        if (!fuse)
            enqueue_g2p(c->stream, c->L, T, c->S[buf], c->cap, c->B.chunks, c->ctl, c->G, flag, lds_box, parity,
                        fb_limit(c), c->cfg.chunk, act, 1);
    }
    if (fuse)  // every scene's last substep of the frame
        enqueue_g2p(c->stream, c->L, T, c->S[buf], c->cap, c->B.chunks, c->ctl, c->G, flag, lds_box,
                    (ns[0] - 1) & 1, fb_limit(c), c->cfg.chunk, active_ranks(ns, 0), 1);
    // the speeds the next frame's exit horizon starts from
    enqueue_speeds_to_host(c->stream, c->S[buf], c->cap, (int)c->N, c->speed_dev + 2, c->ring_dev + RING + 1);
    hipGraph_t graph = nullptr;
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, MPM_EDEVICE, std::string("frame graph capture: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    g.graph = graph;
    HIP_OK(c, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    g.N = c->N;
    g.frame_dt = frame_dt;
    g.chunk = c->cfg.chunk;
    return MPM_OK;
}

// Substeps after which a particle moving at speed v could first leave its
// free zone: it must move more than 3 cells, so with the gravity g not before
// 3 dx = v t + g t^2 / 2; the smallest such t over the scenes, in each
// scene's steps.
double exit_horizon(const mpm_ctx* c, double v) {
    double out = 1e30;
    for (const SceneHost& s : c->sh) {
        if (s.N == 0) continue;
        const double dx = 1.0 / s.desc.n;
        const double g = std::sqrt((double)s.desc.gravity[0] * s.desc.gravity[0] +
                                   (double)s.desc.gravity[1] * s.desc.gravity[1] +
                                   (double)s.desc.gravity[2] * s.desc.gravity[2]);
        const double t = g > 0.0 ? (std::sqrt(v * v + 6.0 * g * dx) - v) / g : (v > 0.0 ? 3.0 * dx / v : 1e30);
        out = std::min(out, t / (double)s.desc.dt);
    }
    return out;
}

// The mean particle speed now: from the last graph frame's end when that is
// current (published to pinned memory inside the frame), else one reduction
// read back.
int current_mean_speed(mpm_ctx* c, double& v) {
    float w[2] = {0.0f, 0.0f};
    if (c->graph_speed) {
        for (int k = 0; k < 2; ++k) {
            const int bits = __atomic_load_n(c->ring + RING + 1 + k, __ATOMIC_ACQUIRE);
            memcpy(&w[k], &bits, sizeof(float));
        }
    } else {
        if (int r = bring_up_to_date(c)) return r;
        HIP_OK(c, hipMemsetAsync(c->speed_dev, 0, 2 * sizeof(float), c->stream));
        enqueue_speeds(c->stream, c->S[c->cur], c->cap, (int)c->N, c->speed_dev);
        HIP_OK(c, hipMemcpyAsync(w, c->speed_dev, 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(c, hipStreamSynchronize(c->stream));
    }
    v = c->N > 0 ? (double)w[1] / (double)c->N : 0.0;
    return MPM_OK;
}

// A graph frame can rebuild only at its start, so a particle that leaves its
// zone mid-frame keeps the global path until the next frame.  Besides the
// request the previous frame left, the frame therefore also rebuilds when the
// exit horizon (above) ends within it.
int graph_frame(mpm_ctx* c, float frame_dt, const std::vector<int>& ns, double horizon) {
    if (int r = settle_graph_frame(c)) return r;
    const int64_t since = c->step - c->last_rebuild;
    const bool due = c->last_rebuild >= 0 && (double)(since + ns[0]) > horizon;
    const bool rebuild = c->need_rebuild || due || (c->cfg.flags & MPM_FLAG_REBUILD_EVERY_STEP);
    const FrameGraph& g = c->graphs[c->cur][rebuild ? 1 : 0];
    if (!(g.exec && g.N == c->N && g.frame_dt == frame_dt && g.chunk == c->cfg.chunk)) {
        // all four at once, so that a run does not stop to record mid-way
        for (int cur = 0; cur < 2; ++cur)
            for (int rb = 0; rb < 2; ++rb)
                if (int r = record_frame_graph(c, cur, rb != 0, frame_dt, ns)) return r;
    }
    HIP_OK(c, hipGraphLaunch(g.exec, c->stream));
    HIP_OK(c, hipEventRecord(c->graph_done, c->stream));
    c->graph_inflight = true;
    c->graph_speed = true;
    if (rebuild) note_rebuild(c);
    c->parity_ctr = 0;
    for (int k = 0; k < ns[0]; ++k) note_substep(c, active_ranks(ns, k));
    c->checked = c->step;  // graph frames leave no ring flags to read
    return MPM_OK;
}

// The automatic time step of a single-scene context for the frame about to
// run: dt = min(dt_max, cfl dx / (max |v_p| + |g| T + c)) with c the speed of
// the material's pressure wave, then the smallest whole number of substeps
// that covers the frame (dt = T / n_s).  The largest particle speed is read
// back from the device (the frame starts from a synchronized stream).
int update_auto_dt(mpm_ctx* c, float frame_dt) {
    if (int r = bring_up_to_date(c)) return r;
    HIP_OK(c, hipMemsetAsync(c->speed_dev, 0, 2 * sizeof(float), c->stream));
    enqueue_speeds(c->stream, c->S[c->cur], c->cap, (int)c->N, c->speed_dev);
    float vmax = 0.0f;
    HIP_OK(c, hipMemcpyAsync(&vmax, c->speed_dev, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    SceneHost& sh = c->sh[0];
    const mpm_material& m = sh.mat;
    const double mu = m.E / (2.0 * (1.0 + m.nu)), la = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
    const double wave = m.kind == MPM_WATER ? std::sqrt((double)m.bulk / m.rho) : std::sqrt((la + 2.0 * mu) / m.rho);
    const double g = std::sqrt((double)sh.desc.gravity[0] * sh.desc.gravity[0] +
                               (double)sh.desc.gravity[1] * sh.desc.gravity[1] +
                               (double)sh.desc.gravity[2] * sh.desc.gravity[2]);
    const double dt = std::min((double)c->auto_dt_max,
                               (double)c->auto_cfl / sh.desc.n / ((double)vmax + g * frame_dt + wave));
    const int n = (int)std::ceil((double)frame_dt / dt - 1e-9);
    const float dt_new = (float)((double)frame_dt / (n < 1 ? 1 : n));
    if (dt_new != sh.desc.dt) {
        sh.desc.dt = dt_new;
        c->table[0].P.dt = dt_new;
        if (sh.has_mat) c->table[0].M = derive_material(sh.mat, c->table[0].P);
        HIP_OK(c, hipMemcpyAsync(c->scene_dev, &c->table[0], sizeof(Scene), hipMemcpyHostToDevice, c->stream));
    }
    return MPM_OK;
}

int run_frame(mpm_ctx* c, float frame_dt) {
    if (c->N == 0) return MPM_OK;
    if (c->auto_cfl > 0.0f)
        if (int r = update_auto_dt(c, frame_dt)) return r;
    const std::vector<int> ns = frame_substeps(c, frame_dt);
    if ((c->cfg.flags & MPM_FLAG_FRAME_GRAPHS) && c->pending && !(c->cfg.flags & MPM_FLAG_REBUILD_EVERY_STEP)) {
        int r = settle_graph_frame(c);
        if (r) return r;
        // A graph frame rebuilds only at its start: while particles could leave their zones
        // within a frame even right after a rebuild, frames run directly, rebuilding where
        // needed, and return to graphs once the motion allows a whole frame.
        // the horizon of the bulk (the mean speed): a few fast particles that leave their
        // zones cost little on the global path and ask for the next frame's rebuild
        double vmean;
        if ((r = current_mean_speed(c, vmean))) return r;
        const double horizon = exit_horizon(c, vmean);
        c->graph_speed = false;
        if (horizon >= (double)ns[0]) {
            if ((r = poll_flags(c, c->step))) return r;  // the ring is idle across a graph frame
            if ((r = bring_up_to_date(c))) return r;
            return graph_frame(c, frame_dt, ns, horizon);
        }
    }
    for (int k = 0; k < ns[0]; ++k) {
        int r = substep_one(c, active_ranks(ns, k));
        if (r) return r;
    }
    return MPM_OK;
}

// Per-rank list ends of the last rebuild (host copy).
int read_rank_ends(mpm_ctx* c, std::vector<int>& e) {
    e.assign(4 * c->nsc, 0);
    HIP_OK(c, hipMemcpyAsync(e.data(), c->rank_end_dev, sizeof(int) * 4 * c->nsc, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return MPM_OK;
}

void rank_range(const std::vector<int>& e, int S, int kind, int r, int& b, int& en) {
    b = r > 0 ? e[kind * S + r - 1] : 0;
    en = e[kind * S + r];
}

int scene_arg(mpm_ctx* c, int32_t scene) {
    if (scene < 0 || scene >= c->nsc) return fail(c, MPM_EINVAL, "scene index out of range");
    return MPM_OK;
}

}  // namespace

namespace {

// Apply the deferred deformation update of the last G2P to the stored state
// (with each snow scene's map), after which no update is pending.
int land_pending(mpm_ctx* c) {
    if (c->sur_any)
        enqueue_materialize_map(c->stream, c->L, tables(c), c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->cfg.chunk);
    else
        enqueue_materialize(c->stream, tables(c), c->S[c->cur], c->cap, (int)c->N);
    HIP_OK(c, hipGetLastError());
    c->pending = 0;
    return MPM_OK;
}

}  // namespace

extern "C" {

int mpm_create(const mpm_config* cfg, mpm_ctx** out) {
    if (!cfg || !out) return fail(nullptr, MPM_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->num_scenes < 1 || cfg->num_scenes > MPM_MAX_SCENES)
        return fail(nullptr, MPM_EINVAL, "num_scenes must be in [1, 256]");
    const int S = cfg->num_scenes;
    std::vector<mpm_scene> desc(S);
    for (int s = 0; s < S; ++s) {
        if (cfg->scenes) {
            desc[s] = cfg->scenes[s];
        } else {
            desc[s].n = cfg->n;
            desc[s].bc = cfg->bc;
            desc[s].bc_cells = cfg->bc_cells;
            for (int a = 0; a < 3; ++a) desc[s].gravity[a] = cfg->gravity[a];
            desc[s].dt = cfg->dt;
        }
        if (const char* why = check_scene(desc[s])) return fail(nullptr, MPM_EINVAL, why);
    }
    if (cfg->capacity < 0) return fail(nullptr, MPM_EINVAL, "negative capacity");
    if (cfg->lag < 0 || cfg->lag > 64) return fail(nullptr, MPM_EINVAL, "lag must be in [0, 64]");
    if (cfg->chunk != 0 && (cfg->chunk < 64 || cfg->chunk > 512 || cfg->chunk % 64))
        return fail(nullptr, MPM_EINVAL, "chunk must be a multiple of 64 in [64, 512]");
    if ((cfg->flags & MPM_FLAG_FRAME_GRAPHS) && cfg->stream == 0)
        return fail(nullptr, MPM_EINVAL, "frame graphs need a stream other than the null stream");
    int nmax = 0;
    for (auto& d : desc) nmax = std::max(nmax, d.n);
    const int shift = 3 * log2i(nmax), key_bits = shift + log2i(S);
    if (key_bits > 32) return fail(nullptr, MPM_EINVAL, "too many scenes for the largest grid: 3 log2(n) + log2(S) > 32");
    int64_t bricks = 0;
    for (auto& d : desc) bricks += (int64_t)(d.n / 4 + 2) * (d.n / 4 + 2) * (d.n / 4 + 2);
    if (bricks * BLOCK_NODES > INT32_MAX) return fail(nullptr, MPM_EINVAL, "the scenes' grids exceed 2^31 nodes");

    mpm_ctx* c = new mpm_ctx();
    c->cfg = *cfg;
    c->cfg.scenes = nullptr;  // copied below
    if (c->cfg.lag == 0) c->cfg.lag = 5;
    if (c->cfg.chunk == 0) c->cfg.chunk = 256;
    c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    (void)hipGetDevice(&c->device);
    c->nsc = S;
    c->shift = shift;
    c->key_bits = key_bits;
    c->sh.resize(S);
    for (int s = 0; s < S; ++s) c->sh[s].desc = desc[s];
    // ranks: increasing dt, ties by scene index
    c->rank_scene.resize(S);
    for (int s = 0; s < S; ++s) c->rank_scene[s] = s;
    std::stable_sort(c->rank_scene.begin(), c->rank_scene.end(),
                     [&](int a, int b) { return desc[a].dt < desc[b].dt; });
    c->table.resize(S);
    std::vector<int> rank_brick(S + 1, 0);
    for (int r = 0; r < S; ++r) {
        const int s = c->rank_scene[r];
        Scene& t = c->table[s];
        t.P = make_step(desc[s]);
        t.M = Mat{};
        t.rank = r;
        t.brick_base = rank_brick[r];
        rank_brick[r + 1] = rank_brick[r] + t.P.NB * t.P.NB * t.P.NB;
    }
    c->nbricks = rank_brick[S];
    query_launch(c->L, c->cfg.chunk);

    auto bail = [&](int code) {
        std::string msg = c->err;
        mpm_destroy(c);
        return fail(nullptr, code, msg);
    };
    const size_t nb = (size_t)c->nbricks;
    bool ok = hipMalloc(&c->G.acc, sizeof(float) * 4 * 64 * nb) == hipSuccess &&
              hipMalloc(&c->G.acc_dirty, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.vel, sizeof(float4) * 64 * nb) == hipSuccess &&
              hipMalloc(&c->G.stamp, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.ovf[0], sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.ovf[1], sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->B.brick_state, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->B.active, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.reg_n, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.reg, sizeof(int) * REG_MAX * nb) == hipSuccess &&
              hipMalloc(&c->ctl, sizeof(int) * CTL_ALLOC_WORDS) == hipSuccess &&
              hipMalloc(&c->speed_dev, 4 * sizeof(float)) == hipSuccess &&
              hipMalloc(&c->scene_dev, sizeof(Scene) * S) == hipSuccess &&
              hipMalloc(&c->rank_scene_dev, sizeof(int) * S) == hipSuccess &&
              hipMalloc(&c->rank_brick_dev, sizeof(int) * (S + 1)) == hipSuccess &&
              hipMalloc(&c->rank_end_dev, sizeof(int) * 4 * S) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        c->err = "grid allocation failed";
        return bail(MPM_ENOMEM);
    }
    if (hipMemsetAsync(c->G.acc, 0, sizeof(float) * 4 * 64 * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.acc_dirty, 0, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.vel, 0, sizeof(float4) * 64 * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.stamp, 0xff, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->B.brick_state, 0, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.reg_n, 0, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ctl, 0, sizeof(int) * CTL_ALLOC_WORDS, c->stream) != hipSuccess ||
        hipMemsetAsync(c->speed_dev, 0, 4 * sizeof(float), c->stream) != hipSuccess ||
        hipMemsetAsync(c->rank_end_dev, 0, sizeof(int) * 4 * S, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->scene_dev, c->table.data(), sizeof(Scene) * S, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->rank_scene_dev, c->rank_scene.data(), sizeof(int) * S, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->rank_brick_dev, rank_brick.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = "initialisation failed";
        return bail(MPM_EDEVICE);
    }
    if (hipHostMalloc(&c->ring, sizeof(int) * (RING + 3), hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&c->ring_dev), c->ring, 0) != hipSuccess) {
        (void)hipGetLastError();
        c->err = "pinned ring allocation failed";
        return bail(MPM_ENOMEM);
    }
    memset(c->ring, 0, sizeof(int) * (RING + 3));
    for (int i = 0; i < RING; ++i)
        if (hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming) != hipSuccess) {
            c->err = "event creation failed";
            return bail(MPM_EDEVICE);
        }
    if (hipEventCreateWithFlags(&c->graph_done, hipEventDisableTiming) != hipSuccess) {
        c->err = "event creation failed";
        return bail(MPM_EDEVICE);
    }
    int64_t cap0 = cfg->capacity > 0 ? cfg->capacity : 4096;
    cap0 = (cap0 + 255) / 256 * 256;
    int r = grow(c, cap0);
    if (r) return bail(r);
    *out = c;
    return MPM_OK;
}

int mpm_destroy(mpm_ctx* c) {
    if (!c) return MPM_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    free_particle_buffers(c);
    (void)hipFree(c->G.acc);
    (void)hipFree(c->G.acc_dirty);
    (void)hipFree(c->G.vel);
    (void)hipFree(c->G.dvel);
    (void)hipFree(c->speed_dev);
    (void)hipFree(c->G.stamp);
    (void)hipFree(c->G.ovf[0]);
    (void)hipFree(c->G.ovf[1]);
    (void)hipFree(c->B.brick_state);
    (void)hipFree(c->B.active);
    (void)hipFree(c->G.reg_n);
    (void)hipFree(c->G.reg);
    (void)hipFree(c->ctl);
    (void)hipFree(c->scene_dev);
    (void)hipFree(c->rank_scene_dev);
    (void)hipFree(c->rank_brick_dev);
    (void)hipFree(c->rank_end_dev);
    if (c->ring) (void)hipHostFree(c->ring);
    for (int i = 0; i < RING; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->graph_done) (void)hipEventDestroy(c->graph_done);
    for (auto& p : c->prof) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    delete c;
    return MPM_OK;
}

int mpm_add_particles(mpm_ctx* c, int32_t scene, const mpm_material* mat, int64_t count, const float* x,
                      const float* v, const float* C, const float* F, const float* s) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (count < 0 || (count > 0 && !x)) return fail(c, MPM_EINVAL, "bad count or null positions");
    if (c->N + count > (int64_t)1 << 30) return fail(c, MPM_EINVAL, "too many particles");
    c->graph_speed = false;  // new particles bring their own speeds
    SceneHost& sh = c->sh[scene];
    if (mat) {
        if (mat->kind < 0 || mat->kind > 3) return fail(c, MPM_EINVAL, "bad material kind");
        if (mat->kind == MPM_SAND && !(mat->E > 0)) return fail(c, MPM_EINVAL, "sand needs E > 0");
        if (!(mat->ppc > 0) || !(mat->rho > 0)) return fail(c, MPM_EINVAL, "ppc and rho must be positive");
        if (mat->kind != MPM_WATER && !(mat->nu > -1.0f && mat->nu < 0.5f)) return fail(c, MPM_EINVAL, "bad nu");
        if (sh.has_mat && !same_material(sh.mat, *mat))
            return fail(c, MPM_EINVAL, "a scene holds one material; pass the same constants or NULL");
        if (!sh.has_mat) {
            sh.mat = *mat;
            sh.has_mat = true;
            c->table[scene].M = derive_material(*mat, c->table[scene].P);
            HIP_OK(c, hipMemcpyAsync(c->scene_dev + scene, &c->table[scene], sizeof(Scene), hipMemcpyHostToDevice,
                                     c->stream));
        }
    } else if (!sh.has_mat) {
        return fail(c, MPM_EINVAL, "the first call for a scene must pass a material");
    }
    if (count == 0) return MPM_OK;
    // the pending G2P walks the current chunk list, which growing the buffers replaces
    if (int r = bring_up_to_date(c)) return r;
    if ((c->cfg.flags & MPM_FLAG_ALLOC_EXACT) ? c->N + count > c->cap : c->N + count > c->cap / 2) {
        int64_t newcap = c->cap;
        if (c->cfg.flags & MPM_FLAG_ALLOC_EXACT)  // the allocation ablation: just what is needed
            newcap = c->N + count;
        else
            while (c->N + count > newcap / 2) newcap *= 4;
        int r = grow(c, newcap);
        if (r) return r;
    }
    if (c->pending) {  // land the deferred update so old and new particles share one state convention
        if (int r = land_pending(c)) return r;
    }
    enqueue_insert(c->stream, c->S[c->cur], c->ids[c->cur], c->cap, (int)c->N, (int)count, scene, (int)sh.N, x, v, C,
                   F, s, c->ctl);
    HIP_OK(c, hipGetLastError());
    c->N += count;
    sh.N += count;
    c->need_rebuild = true;
    return MPM_OK;
}

int mpm_substep(mpm_ctx* c, int32_t nsteps) {
    if (!c) return MPM_EINVAL;
    if (nsteps < 0) return fail(c, MPM_EINVAL, "negative step count");
    if (c->N == 0) return MPM_OK;
    for (int k = 0; k < nsteps; ++k) {
        int r = substep_one(c, c->nsc);
        if (r) return r;
    }
    return MPM_OK;
}

int mpm_frame(mpm_ctx* c, float frame_dt) {
    if (!c) return MPM_EINVAL;
    if (!(frame_dt > 0.0f)) return fail(c, MPM_EINVAL, "frame_dt must be positive");
    return run_frame(c, frame_dt);
}

int mpm_rebuild(mpm_ctx* c) {
    if (!c) return MPM_EINVAL;
    c->need_rebuild = true;
    return MPM_OK;
}

int mpm_synchronize(mpm_ctx* c) {
    if (!c) return MPM_EINVAL;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return poll_flags(c, c->step);
}

int mpm_read_particles(mpm_ctx* c, int32_t scene, int64_t count, float* x, float* v, float* C, float* F, float* s) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (count != c->sh[scene].N) return fail(c, MPM_EINVAL, "count must equal the scene's particle count");
    if (int r = bring_up_to_date(c)) return r;
    // a snow map without SVD (learned or closed form) is landed by its own kernel first, so the
    // state read is the one the next P2G would use
    if (c->pending && c->sur_any && (F || s))
        if (int r = land_pending(c)) return r;
    enqueue_read(c->stream, tables(c), c->S[c->cur], c->ids[c->cur], c->cap, (int)c->N, scene, (int)count, c->pending,
                 x, v, C, F, s);
    HIP_OK(c, hipGetLastError());
    return check_error_word(c);
}

int mpm_read_grid(mpm_ctx* c, int32_t scene, float* m, float* v) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    enqueue_read_grid(c->stream, c->table[scene], c->G, (int)c->sh[scene].last_step, m, v);
    HIP_OK(c, hipGetLastError());
    return check_error_word(c);
}

int mpm_read_binning(mpm_ctx* c, int32_t scene, int64_t count, uint32_t* keys, int32_t* perm) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (c->last_rebuild < 0) return fail(c, MPM_EINVAL, "no rebuild has run yet");
    if (count != c->sh[scene].N_at_rebuild)
        return fail(c, MPM_EINVAL, "count must equal the scene's particle count at the last rebuild");
    std::vector<int> e;
    if (int r = read_rank_ends(c, e)) return r;
    int b, en;
    rank_range(e, c->nsc, RE_PART, c->table[scene].rank, b, en);
    if (en - b != count) return fail(c, MPM_EDEVICE, "rank range does not match the particle count");
    if (keys)
        enqueue_copy_codes(c->stream, keys, c->B.keys[c->B.sorted] + b, (int)count, (1u << c->shift) - 1u);
    if (perm)
        HIP_OK(c, hipMemcpyAsync(perm, c->B.sorted_ids + b, sizeof(int32_t) * count, hipMemcpyDeviceToDevice,
                                 c->stream));
    HIP_OK(c, hipGetLastError());
    return check_error_word(c);
}

int mpm_read_blocks(mpm_ctx* c, int32_t scene, uint32_t* gcode, int32_t* gstart, int32_t* gcount, int32_t* active) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    std::vector<int> e;
    if (int r = read_rank_ends(c, e)) return r;
    const int rk = c->table[scene].rank;
    int pb, pe, gb, ge, ab, ae;
    rank_range(e, c->nsc, RE_PART, rk, pb, pe);
    rank_range(e, c->nsc, RE_GBLOCK, rk, gb, ge);
    rank_range(e, c->nsc, RE_ACTIVE, rk, ab, ae);
    const int ng = ge - gb, na = ae - ab;
    const uint32_t bmask = (1u << (c->shift - 6)) - 1u;
    if (ng > 0 && gcode) {
        HIP_OK(c, hipMemcpy(gcode, c->B.gcode + gb, sizeof(uint32_t) * ng, hipMemcpyDeviceToHost));
        for (int i = 0; i < ng; ++i) gcode[i] &= bmask;
    }
    if (ng > 0 && (gstart || gcount)) {
        std::vector<int> st(ng + 1);
        HIP_OK(c, hipMemcpy(st.data(), c->B.gstart + gb, sizeof(int) * ng, hipMemcpyDeviceToHost));
        st[ng] = pe;
        for (int i = 0; i < ng; ++i) {
            if (gstart) gstart[i] = st[i] - pb;
            if (gcount) gcount[i] = st[i + 1] - st[i];
        }
    }
    if (na > 0 && active) {
        HIP_OK(c, hipMemcpy(active, c->B.active + ab, sizeof(int) * na, hipMemcpyDeviceToHost));
        for (int i = 0; i < na; ++i) active[i] -= c->table[scene].brick_base;
    }
    return check_error_word(c);
}

int mpm_get_stats(mpm_ctx* c, mpm_stats* o) {
    if (!c || !o) return MPM_EINVAL;
    int h[CTL_ALLOC_WORDS];
    HIP_OK(c, hipMemcpyAsync(h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    int r = poll_flags(c, c->step);
    if (r) return r;
    memset(o, 0, sizeof *o);
    o->num_particles = c->N;
    o->capacity = c->cap;
    o->substeps = c->step;
    o->rebuilds = c->rebuilds;
    o->gblocks = h[CTL_NGB];
    o->active_blocks = h[CTL_NACTIVE];
    o->chunks = h[CTL_NCHUNK];
    o->overflow_blocks = c->step > 0 ? h[CTL_OVF + ((c->parity_ctr - 1) & 1)] : 0;
    o->error = (uint32_t)h[CTL_ERROR];
    o->pending_update = (uint32_t)c->pending;
    unsigned long long c64[CTL64_WORDS] = {};
    for (int st = 0; st < CTL64_STRIPES; ++st) {
        unsigned long long w[CTL64_WORDS];
        memcpy(w, h + CTL64_BASE + 2 * CTL64_STRIDE * st, sizeof w);
        for (int k = 0; k < CTL64_WORDS; ++k) c64[k] += w[k];
    }
    o->p2g_fallback_chunks = (int64_t)c64[CTL64_FALLBACK_CHUNKS];
    o->p2g_global_particles = (int64_t)c64[CTL64_GLOBAL_PARTICLES];
    o->surrogate_particles = (int64_t)c64[CTL64_SUR_PARTICLES];
    o->surrogate_fallbacks = (int64_t)c64[CTL64_SUR_FALLBACKS];
    return o->error ? fail(c, MPM_ESTATE, "device error word set") : MPM_OK;
}

int mpm_get_scene_stats(mpm_ctx* c, int32_t scene, mpm_scene_stats* o) {
    if (!c || !o) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    std::vector<int> e;
    if (int r = read_rank_ends(c, e)) return r;
    const int rk = c->table[scene].rank;
    int gb, ge, ab, ae;
    rank_range(e, c->nsc, RE_GBLOCK, rk, gb, ge);
    rank_range(e, c->nsc, RE_ACTIVE, rk, ab, ae);
    memset(o, 0, sizeof *o);
    o->num_particles = c->sh[scene].N;
    o->substeps = c->sh[scene].substeps;
    o->gblocks = ge - gb;
    o->active_blocks = ae - ab;
    o->n = c->sh[scene].desc.n;
    o->dt = c->sh[scene].desc.dt;
    return MPM_OK;
}

int mpm_clear_error(mpm_ctx* c) {
    if (!c) return MPM_EINVAL;
    HIP_OK(c, hipMemsetAsync(c->ctl + CTL_ERROR, 0, sizeof(int), c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return MPM_OK;
}

int mpm_autotune(mpm_ctx* c, float frame_dt, int32_t frames, int32_t* chunk_out) {
    if (!c) return MPM_EINVAL;
    if (!(frame_dt > 0.0f) || frames < 1) return fail(c, MPM_EINVAL, "frame_dt must be positive and frames >= 1");
    const int orig_chunk = c->cfg.chunk;
    c->graph_speed = false;
    if (c->N == 0) {
        if (chunk_out) *chunk_out = orig_chunk;
        return MPM_OK;
    }
    if (int r = bring_up_to_date(c)) return r;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (int r = poll_flags(c, c->step)) return r;
    // snapshot of the device state and of the host counters
    float* snap = nullptr;
    int* snap_ids = nullptr;
    int snap_ctl[CTL_ALLOC_WORDS];
    if (hipMalloc(&snap, sizeof(float) * NF * c->cap) != hipSuccess ||
        hipMalloc(&snap_ids, sizeof(int) * c->cap) != hipSuccess) {
        (void)hipFree(snap);
        (void)hipGetLastError();
        return fail(c, MPM_ENOMEM, "autotune snapshot allocation failed");
    }
    const int cur0 = c->cur;
    auto restore_host = [](mpm_ctx* dst, const mpm_ctx& s) {
        dst->step = s.step;
        dst->checked = s.checked;
        dst->last_rebuild = s.last_rebuild;
        dst->rebuilds = s.rebuilds;
        dst->parity_ctr = s.parity_ctr;
        dst->n_at_rebuild = s.n_at_rebuild;
        dst->pending = s.pending;
        dst->g2p_due_act = 0;  // the snapshot holds the state brought up to date
        dst->sh = s.sh;
        dst->graph_speed = false;
    };
    mpm_ctx saved;  // host counters only
    saved.step = c->step;
    saved.checked = c->checked;
    saved.last_rebuild = c->last_rebuild;
    saved.rebuilds = c->rebuilds;
    saved.parity_ctr = c->parity_ctr;
    saved.n_at_rebuild = c->n_at_rebuild;
    saved.pending = c->pending;
    saved.sh = c->sh;
    const uint32_t prof_mask = c->prof_mask;
    c->prof_mask = 0;
    int rc = MPM_OK;
    auto copy_state = [&](bool to_snap) -> int {
        if (to_snap) {
            HIP_OK(c, hipMemcpyAsync(snap, c->S[cur0], sizeof(float) * NF * c->cap, hipMemcpyDeviceToDevice,
                                     c->stream));
            HIP_OK(c, hipMemcpyAsync(snap_ids, c->ids[cur0], sizeof(int) * c->cap, hipMemcpyDeviceToDevice,
                                     c->stream));
            HIP_OK(c, hipMemcpyAsync(snap_ctl, c->ctl, sizeof snap_ctl, hipMemcpyDeviceToHost, c->stream));
        } else {
            HIP_OK(c, hipMemcpyAsync(c->S[cur0], snap, sizeof(float) * NF * c->cap, hipMemcpyDeviceToDevice,
                                     c->stream));
            HIP_OK(c, hipMemcpyAsync(c->ids[cur0], snap_ids, sizeof(int) * c->cap, hipMemcpyDeviceToDevice,
                                     c->stream));
            HIP_OK(c, hipMemcpyAsync(c->ctl, snap_ctl, sizeof snap_ctl, hipMemcpyHostToDevice, c->stream));
        }
        HIP_OK(c, hipStreamSynchronize(c->stream));
        return MPM_OK;
    };
    rc = copy_state(true);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(c, MPM_EDEVICE, "event creation failed");
    int best = orig_chunk;
    float best_ms = -1.0f;
    const int cand[3] = {128, 256, 512};
    for (int i = 0; i < 3 && !rc; ++i) {
        c->cur = cur0;
        restore_host(c, saved);
        if ((rc = copy_state(false))) break;
        c->cfg.chunk = cand[i];
        query_launch(c->L, c->cfg.chunk);
        drop_graphs(c);
        c->need_rebuild = true;
        if ((rc = run_frame(c, frame_dt))) break;  // warm-up (and graph recording)
        if (hipEventRecord(e0, c->stream) != hipSuccess) {
            rc = fail(c, MPM_EDEVICE, "event record failed");
            break;
        }
        for (int f = 0; f < frames && !rc; ++f) rc = run_frame(c, frame_dt);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(c, MPM_EDEVICE, "event timing failed");
            break;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = cand[i];
        }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)poll_flags(c, c->step);
    // put everything back; keep the winner
    c->cur = cur0;
    restore_host(c, saved);
    if (!rc) rc = copy_state(false);
    c->cfg.chunk = rc ? orig_chunk : best;
    query_launch(c->L, c->cfg.chunk);
    drop_graphs(c);
    c->need_rebuild = true;
    c->prof_mask = prof_mask;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
    (void)hipFree(snap_ids);
    if (!rc && chunk_out) *chunk_out = c->cfg.chunk;
    return rc;
}

int mpm_profile(mpm_ctx* c, uint32_t mask) {
    if (!c) return MPM_EINVAL;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->prof) p.live = false;
    c->prof_mask = 0;
    c->prof_every = (mask >> 16) ? (mask >> 16) : 1u;
    for (int i = 0; i < 4; ++i) {
        if (mask & (1u << i)) c->prof_mask |= 1u << i;
        c->prof_launch[i] = 0;
        c->prof_ms[i] = 0.0;
        c->prof_seen[i] = 0;
    }
    return MPM_OK;
}

int mpm_profile_read(mpm_ctx* c, mpm_profile_data* o) {
    if (!c || !o) return MPM_EINVAL;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->prof) {
        int r = prof_accumulate(c, p);
        if (r) return r;
    }
    for (int i = 0; i < 4; ++i) {
        o->launches[i] = c->prof_launch[i];
        o->ms[i] = c->prof_ms[i];
    }
    return MPM_OK;
}

const char* mpm_last_error(const mpm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------- surrogate
struct mpm_surrogate {
    hipStream_t stream = nullptr;
    float* theta = nullptr;  // [SUR_PARAMS] FP32 master parameters
    float* norm = nullptr;   // [SUR_NORM]
    float* grad = nullptr;   // [SUR_PARAMS]
    float* m = nullptr;      // Adam moments
    float* v = nullptr;
    float* loss = nullptr;   // [loss_cap] per-step minibatch losses
    int loss_cap = 0;
    int* idx = nullptr;      // minibatch rows
    int idx_cap = 0;
    int step = 0;            // Adam steps taken
    unsigned long long* counter = nullptr;
};

namespace {

int sfail(mpm_surrogate*, int code, const std::string& msg) {
    g_create_error = msg;
    return code;
}

#define SHIP_OK(call)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return sfail(nullptr, e_ == hipErrorOutOfMemory ? MPM_ENOMEM : MPM_EDEVICE,                 \
                         std::string(#call) + ": " + hipGetErrorString(e_));                            \
    } while (0)

__global__ void k_identity_norm(float* norm) {
    const int i = threadIdx.x;
    if (i < SUR_NORM) norm[i] = ((i >= SUR_IN && i < 2 * SUR_IN) || i >= 2 * SUR_IN + SUR_OUT) ? 1.0f : 0.0f;
}

}  // namespace

extern "C" {

int mpm_surrogate_create(uint64_t stream, mpm_surrogate** out) {
    if (!out) return sfail(nullptr, MPM_EINVAL, "null argument");
    *out = nullptr;
    mpm_surrogate* s = new mpm_surrogate();
    s->stream = reinterpret_cast<hipStream_t>(stream);
    bool ok = hipMalloc(&s->theta, sizeof(float) * SUR_PARAMS) == hipSuccess &&
              hipMalloc(&s->norm, sizeof(float) * SUR_NORM) == hipSuccess &&
              hipMalloc(&s->grad, sizeof(float) * SUR_PARAMS) == hipSuccess &&
              hipMalloc(&s->m, sizeof(float) * SUR_PARAMS) == hipSuccess &&
              hipMalloc(&s->v, sizeof(float) * SUR_PARAMS) == hipSuccess &&
              hipMalloc(&s->counter, sizeof(unsigned long long)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        mpm_surrogate_destroy(s);
        return sfail(nullptr, MPM_ENOMEM, "surrogate allocation failed");
    }
    sur_zero(s->stream, s->theta, SUR_PARAMS);
    sur_zero(s->stream, s->grad, SUR_PARAMS);
    sur_zero(s->stream, s->m, SUR_PARAMS);
    sur_zero(s->stream, s->v, SUR_PARAMS);
    hipLaunchKernelGGL(k_identity_norm, dim3(1), dim3(64), 0, s->stream, s->norm);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess) {
        mpm_surrogate_destroy(s);
        return sfail(nullptr, MPM_EDEVICE, "surrogate initialisation failed");
    }
    *out = s;
    return MPM_OK;
}

int mpm_surrogate_destroy(mpm_surrogate* s) {
    if (!s) return MPM_OK;
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->theta);
    (void)hipFree(s->norm);
    (void)hipFree(s->grad);
    (void)hipFree(s->m);
    (void)hipFree(s->v);
    (void)hipFree(s->loss);
    (void)hipFree(s->idx);
    (void)hipFree(s->counter);
    delete s;
    return MPM_OK;
}

int mpm_surrogate_set(mpm_surrogate* s, const float* theta, const float* norm) {
    if (!s) return MPM_EINVAL;
    if (theta) SHIP_OK(hipMemcpyAsync(s->theta, theta, sizeof(float) * SUR_PARAMS, hipMemcpyDeviceToDevice, s->stream));
    if (norm) SHIP_OK(hipMemcpyAsync(s->norm, norm, sizeof(float) * SUR_NORM, hipMemcpyDeviceToDevice, s->stream));
    return MPM_OK;
}

int mpm_surrogate_get(mpm_surrogate* s, float* theta, float* norm) {
    if (!s) return MPM_EINVAL;
    if (theta) SHIP_OK(hipMemcpyAsync(theta, s->theta, sizeof(float) * SUR_PARAMS, hipMemcpyDeviceToDevice, s->stream));
    if (norm) SHIP_OK(hipMemcpyAsync(norm, s->norm, sizeof(float) * SUR_NORM, hipMemcpyDeviceToDevice, s->stream));
    return MPM_OK;
}

int mpm_surrogate_forward(mpm_surrogate* s, int32_t precision, int64_t count, const float* X, float* Y) {
    if (!s || count < 0 || (count > 0 && (!X || !Y)) || (precision != 0 && precision != 1))
        return sfail(s, MPM_EINVAL, "bad surrogate forward arguments");
    sur_forward(s->stream, precision, s->theta, s->norm, X, count, Y);
    SHIP_OK(hipGetLastError());
    return MPM_OK;
}

int mpm_surrogate_loss_grad(mpm_surrogate* s, int32_t precision, int64_t count, const float* X, const float* T,
                            float* grad, float* loss) {
    if (!s || count < 1 || !X || !T || !grad || !loss || (precision != 0 && precision != 1))
        return sfail(s, MPM_EINVAL, "bad surrogate gradient arguments");
    sur_grad(s->stream, precision, s->theta, s->norm, X, T, count, nullptr, grad, loss, true);
    SHIP_OK(hipGetLastError());
    return MPM_OK;
}

int mpm_surrogate_fit_norm(mpm_surrogate* s, int64_t count, const float* X, const float* T) {
    if (!s || count < 1 || !X || !T) return sfail(s, MPM_EINVAL, "bad normalisation arguments");
    sur_norm(s->stream, X, T, count, s->norm);
    SHIP_OK(hipGetLastError());
    return MPM_OK;
}

}  // extern "C"

namespace {

// `steps` Adam steps with the minibatch rows in idx[batch] and the per-step
// losses in loss[steps] (device scratch of the caller's choosing), then the
// losses to loss_host and a stream synchronization.
int train_steps(mpm_surrogate* s, int64_t count, const float* X, const float* T, int32_t steps, int32_t batch,
                float lr, uint64_t seed, float* loss_host, int* idx, float* loss) {
    for (int k = 0; k < steps; ++k) {
        sur_indices(s->stream, seed, s->step, batch, count, idx);
        sur_grad(s->stream, 1, s->theta, s->norm, X, T, batch, idx, s->grad, loss + k, true);
        sur_adam(s->stream, s->theta, s->grad, s->m, s->v, s->step + 1, lr);
        ++s->step;
    }
    SHIP_OK(hipGetLastError());
    if (loss_host && steps > 0)
        SHIP_OK(hipMemcpyAsync(loss_host, loss, sizeof(float) * steps, hipMemcpyDeviceToHost, s->stream));
    SHIP_OK(hipStreamSynchronize(s->stream));
    return MPM_OK;
}

int check_train_args(mpm_surrogate* s, int64_t count, const float* X, const float* T, int32_t steps, int32_t batch,
                     float lr) {
    if (!s || count < 1 || !X || !T || steps < 0 || batch < 16 || !(lr > 0.0f))
        return sfail(s, MPM_EINVAL, "bad training arguments");
    if (count > INT32_MAX) return sfail(s, MPM_EINVAL, "too many training rows");
    return MPM_OK;
}

// Scratch of mpm_surrogate_train_noalloc: the minibatch row indices
// [MPM_SUR_NOALLOC_MAX_BATCH], then the per-step losses
// [MPM_SUR_NOALLOC_MAX_STEPS] (FP32 bits).  Each device holds its own copy
// for the life of the process.  In host code the name stands for no device
// address: kernels get the address hipGetSymbolAddress returns for the
// current device (scratch_on_device).
__device__ __align__(256) int scratch[MPM_SUR_NOALLOC_MAX_BATCH + MPM_SUR_NOALLOC_MAX_STEPS];

constexpr int SCRATCH_MAX_DEVICES = 64;
int* g_scratch_dev[SCRATCH_MAX_DEVICES];  // per device, filled on the entry point's first call there
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up once per
// device), or nullptr with the HIP error in *err.
int* scratch_on_device(hipError_t* err) {
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_dev[dev] = static_cast<int*>(ptr);
    }
    return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

int mpm_surrogate_train(mpm_surrogate* s, int64_t count, const float* X, const float* T, int32_t steps, int32_t batch,
                        float lr, uint64_t seed, float* loss_host) {
    if (int r = check_train_args(s, count, X, T, steps, batch, lr)) return r;
    if (batch > s->idx_cap) {
        (void)hipFree(s->idx);
        s->idx = nullptr;
        SHIP_OK(hipMalloc(&s->idx, sizeof(int) * batch));
        s->idx_cap = batch;
    }
    if (steps > s->loss_cap) {
        (void)hipFree(s->loss);
        s->loss = nullptr;
        SHIP_OK(hipMalloc(&s->loss, sizeof(float) * steps));
        s->loss_cap = steps;
    }
    return train_steps(s, count, X, T, steps, batch, lr, seed, loss_host, s->idx, s->loss);
}

int mpm_surrogate_train_noalloc(mpm_surrogate* s, int64_t count, const float* X, const float* T, int32_t steps,
                                int32_t batch, float lr, uint64_t seed, float* loss_host) {
    if (int r = check_train_args(s, count, X, T, steps, batch, lr)) return r;
    if (batch > MPM_SUR_NOALLOC_MAX_BATCH || steps > MPM_SUR_NOALLOC_MAX_STEPS)
        return sfail(s, MPM_EINVAL, "mpm_surrogate_train_noalloc: batch above MPM_SUR_NOALLOC_MAX_BATCH or steps "
                                    "above MPM_SUR_NOALLOC_MAX_STEPS");
    hipError_t e = hipSuccess;
    int* ptr = scratch_on_device(&e);
    if (!ptr)
        return sfail(s, MPM_EDEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(e));
    // every index is written by the step that reads it and every loss slot is
    // cleared by its step, so nothing left from an earlier call is read
    return train_steps(s, count, X, T, steps, batch, lr, seed, loss_host, ptr,
                       reinterpret_cast<float*>(ptr + MPM_SUR_NOALLOC_MAX_BATCH));
}

int mpm_use_surrogate(mpm_ctx* c, int32_t scene, const mpm_surrogate* s, int32_t mode, float tol, float dt_ref) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (mode < 0 || mode > 2) return fail(c, MPM_EINVAL, "mode must be exact (0), surrogate (1) or closed form (2)");
    if (mode == 1 && !s) return fail(c, MPM_EINVAL, "the surrogate mode needs a surrogate");
    if (mode == 1 && (!(tol > 0.0f) || !(dt_ref > 0.0f))) return fail(c, MPM_EINVAL, "tol and dt_ref must be positive");
    if (mode != 0 && (!c->sh[scene].has_mat || c->sh[scene].mat.kind != MPM_SNOW))
        return fail(c, MPM_EINVAL, "only snow scenes take the surrogate (add the scene's particles first)");
    if (s) {
        c->sur_theta = s->theta;
        c->sur_norm = s->norm;
        c->sur_tol = tol;
        c->sur_dt_ref = dt_ref;
    }
    c->table[scene].ret = mode;
    c->table[scene].E = c->sh[scene].has_mat ? c->sh[scene].mat.E : 0.0f;
    HIP_OK(c, hipMemcpyAsync(c->scene_dev + scene, &c->table[scene], sizeof(Scene), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->sur_any = 0;  // 2 if some scene runs the network, 1 if only the closed form
    for (int k = 0; k < c->nsc; ++k)
        c->sur_any = std::max(c->sur_any, c->table[k].ret == 1 ? 2 : c->table[k].ret == 2 ? 1 : 0);
    if (!c->sur_any) c->sur_theta = c->sur_norm = nullptr;
    if (c->sur_any && !c->sur_theta && mode == 1) return fail(c, MPM_EINVAL, "no surrogate attached");
    drop_graphs(c);  // recorded kernels carry the old choice
    return MPM_OK;
}

int mpm_set_transfer(mpm_ctx* c, int32_t scene, float flip, float beta_min, float beta_max) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (!(flip >= 0.0f && flip <= 1.0f) || !(beta_min >= 0.0f && beta_min <= beta_max && beta_max <= 1.0f))
        return fail(c, MPM_EINVAL, "need 0 <= flip <= 1 and 0 <= beta_min <= beta_max <= 1");
    if (int r = bring_up_to_date(c)) return r;  // an outstanding fused G2P ran with the old transfer
    if (flip > 0.0f && !c->G.dvel) {
        const int64_t nodes = (int64_t)c->nbricks * 64;
        HIP_OK(c, hipMalloc(&c->G.dvel, sizeof(float4) * nodes));
        HIP_OK(c, hipMemsetAsync(c->G.dvel, 0, sizeof(float4) * nodes, c->stream));
    }
    Step& P = c->table[scene].P;
    P.flip = flip;
    P.bmin = beta_min;
    P.bmax = beta_max;
    HIP_OK(c, hipMemcpyAsync(c->scene_dev + scene, &c->table[scene], sizeof(Scene), hipMemcpyHostToDevice, c->stream));
    c->any_flip = false;
    for (int k = 0; k < c->nsc; ++k) c->any_flip = c->any_flip || c->table[k].P.flip > 0.0f;
    drop_graphs(c);
    return MPM_OK;
}

int mpm_set_auto_dt(mpm_ctx* c, float cfl, float dt_max) {
    if (!c) return MPM_EINVAL;
    if (c->nsc != 1) return fail(c, MPM_EINVAL, "the automatic time step needs a single-scene context");
    if (!(cfl >= 0.0f && cfl <= 1.0f) || (cfl > 0.0f && !(dt_max > 0.0f)))
        return fail(c, MPM_EINVAL, "need 0 <= cfl <= 1 and dt_max > 0");
    c->auto_cfl = cfl;
    c->auto_dt_max = dt_max;
    drop_graphs(c);
    return MPM_OK;
}

int mpm_surrogate_sample(mpm_ctx* c, int32_t scene, float dt_ref, int64_t max_count, float* X, float* T,
                         int64_t* written) {
    if (!c) return MPM_EINVAL;
    if (int r = scene_arg(c, scene)) return r;
    if (!X || !T || max_count < 0 || !(dt_ref > 0.0f)) return fail(c, MPM_EINVAL, "bad sampling arguments");
    if (!c->sh[scene].has_mat || c->sh[scene].mat.kind != MPM_SNOW) return fail(c, MPM_EINVAL, "the scene is not snow");
    if (int r = bring_up_to_date(c)) return r;
    unsigned long long* counter = nullptr;
    HIP_OK(c, hipMalloc(&counter, sizeof(unsigned long long)));
    sur_zero(c->stream, reinterpret_cast<float*>(counter), 2);
    sur_sample(c->stream, c->S[c->cur], c->cap, (int)c->N, tables(c), scene, c->pending, c->sh[scene].mat.E, dt_ref,
               max_count, X, T, counter);
    unsigned long long n = 0;
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipMemcpyAsync(&n, counter, sizeof n, hipMemcpyDeviceToHost, c->stream);
    const hipError_t e3 = hipStreamSynchronize(c->stream);
    (void)hipFree(counter);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(c, MPM_EDEVICE, "sampling failed");
    if (written) *written = (int64_t)(n < (unsigned long long)max_count ? n : (unsigned long long)max_count);
    return check_error_word(c);
}

}  // extern "C"
