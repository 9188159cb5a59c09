// Host runtime behind the C ABI of include/mpm.h.
//
// Capacity: particle buffers grow 4x once more than half full, and only in
// mpm_add_particles (paper, "Principles": a vector that reserves ahead
// avoids reallocation during the simulation; scan/sort scratch is allocated
// up front).  The dense block grid is allocated once at creation.
//
// Rebuild scheduling without draining the stream: G2P sets a device flag when
// a particle leaves its free zone and, the first time, writes it to a pinned
// host ring slot of that substep; an event marks the substep's end.  Before
// enqueueing substep k the host reads the slots of substeps that have
// finished, waiting only for substep k - lag, so the device keeps `lag`
// substeps queued.  A particle that leaves its free zone before the rebuild
// lands is still transferred exactly (through global atomics), so the lag
// costs speed, never correctness.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "mpm_internal.h"

using namespace mpm;

namespace {

constexpr int RING = 128;
constexpr int PROF_SLOTS = 4096;

std::string g_create_error;

}  // namespace

struct mpm_ctx {
    mpm_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    Step P{};
    Mat M{};
    mpm_material mat{};
    bool has_mat = false;
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
    int64_t n_at_rebuild = 0;
    bool need_rebuild = true;
    int pending = 0;

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
    return M;
}

bool same_material(const mpm_material& a, const mpm_material& b) {
    return a.kind == b.kind && a.E == b.E && a.nu == b.nu && a.rho == b.rho && a.ppc == b.ppc &&
           a.theta_c == b.theta_c && a.theta_s == b.theta_s && a.xi == b.xi && a.bulk == b.bulk;
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
    (void)hipFree(c->B.gchunk);
    (void)hipFree(c->B.sorted_ids);
    (void)hipFree(c->G.stage);
    (void)hipFree(c->G.box);
    c->B.gchunk = c->B.sorted_ids = nullptr;
    c->G.stage = nullptr;
    c->G.box = nullptr;
    c->B.hist = c->B.scan_tiles = c->B.gstart = nullptr;
    c->B.gcode = nullptr;
    c->B.chunks = nullptr;
}

// Allocate particle-sized buffers for `newcap`, keeping the current state.
int grow(mpm_ctx* c, int64_t newcap) {
    float* S[2] = {nullptr, nullptr};
    int* ids[2] = {nullptr, nullptr};
    uint32_t *keys[2] = {nullptr, nullptr}, *vals[2] = {nullptr, nullptr};
    int *hist = nullptr, *tiles = nullptr, *gstart = nullptr;
    uint32_t* gcode = nullptr;
    Chunk* chunks = nullptr;
    int *gchunk = nullptr, *sorted_ids = nullptr;
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
    ok = ok && hipMalloc(&gchunk, sizeof(int) * (newcap + 2)) == hipSuccess;
    ok = ok && hipMalloc(&sorted_ids, sizeof(int) * newcap) == hipSuccess;
    ok = ok && hipMalloc(&stage, sizeof(float4) * stage_nodes) == hipSuccess;
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
        (void)hipFree(gchunk);
        (void)hipFree(sorted_ids);
        (void)hipFree(stage);
        (void)hipFree(box);
        (void)hipGetLastError();
        return fail(c, MPM_ENOMEM, "particle buffer allocation failed for capacity " + std::to_string(newcap));
    }
    if (c->N > 0) {
        HIP_OK(c, hipMemcpy2DAsync(S[0], sizeof(float) * newcap, c->S[c->cur], sizeof(float) * c->cap,
                                   sizeof(float) * c->N, NF, hipMemcpyDeviceToDevice, c->stream));
        HIP_OK(c, hipMemcpyAsync(ids[0], c->ids[c->cur], sizeof(int) * c->N, hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_OK(c, hipMemsetAsync(box, 0, sizeof(int4) * (newcap + 1), c->stream));
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
    c->B.gchunk = gchunk;
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

// Read the rebuild flags of finished substeps, waiting for those at or
// before `must_upto`.
int poll_flags(mpm_ctx* c, int64_t must_upto) {
    while (c->checked < c->step) {
        const int slot = (int)(c->checked % RING);
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
        if (__atomic_load_n(&c->ring[slot], __ATOMIC_ACQUIRE) && c->checked >= c->last_rebuild &&
            !(c->cfg.flags & MPM_FLAG_MANUAL_REBUILD))
            c->need_rebuild = true;
        ++c->checked;
    }
    return MPM_OK;
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

}  // namespace

extern "C" {

int mpm_create(const mpm_config* cfg, mpm_ctx** out) {
    if (!cfg || !out) return fail(nullptr, MPM_EINVAL, "null argument");
    *out = nullptr;
    const int n = cfg->n;
    if (n < 16 || n > 512 || (n & (n - 1))) return fail(nullptr, MPM_EINVAL, "n must be a power of two in [16, 512]");
    if (cfg->bc < 0 || cfg->bc > 2) return fail(nullptr, MPM_EINVAL, "bad bc");
    if (cfg->bc_cells < 0 || cfg->bc_cells > n / 2) return fail(nullptr, MPM_EINVAL, "bad bc_cells");
    if (cfg->num_scenes != 1) return fail(nullptr, MPM_EINVAL, "num_scenes must be 1");
    if (!(cfg->dt > 0.0f)) return fail(nullptr, MPM_EINVAL, "dt must be positive");
    if (cfg->capacity < 0) return fail(nullptr, MPM_EINVAL, "negative capacity");
    if (cfg->lag < 0 || cfg->lag > 64) return fail(nullptr, MPM_EINVAL, "lag must be in [0, 64]");
    if (cfg->chunk != 0 && (cfg->chunk < 64 || cfg->chunk > 512 || cfg->chunk % 64))
        return fail(nullptr, MPM_EINVAL, "chunk must be a multiple of 64 in [64, 512]");
    mpm_ctx* c = new mpm_ctx();
    c->cfg = *cfg;
    if (c->cfg.lag == 0) c->cfg.lag = 3;
    if (c->cfg.chunk == 0) c->cfg.chunk = 256;
    c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    (void)hipGetDevice(&c->device);
    c->P.n = n;
    c->P.NB = n / 4 + 2;
    c->P.fn = (float)n;
    c->P.dx = 1.0f / (float)n;
    c->P.dt = cfg->dt;
    c->P.g0 = cfg->gravity[0];
    c->P.g1 = cfg->gravity[1];
    c->P.g2 = cfg->gravity[2];
    c->P.bc = cfg->bc;
    c->P.bc_cells = cfg->bc_cells;
    c->nbricks = c->P.NB * c->P.NB * c->P.NB;
    query_launch(c->L, c->cfg.chunk);

    auto bail = [&](int code) {
        std::string msg = c->err;
        mpm_destroy(c);
        return fail(nullptr, code, msg);
    };
    const size_t nb = (size_t)c->nbricks;
    bool ok = hipMalloc(&c->G.acc, sizeof(float) * 4 * 64 * nb) == hipSuccess &&
              hipMalloc(&c->G.vel, sizeof(float4) * 64 * nb) == hipSuccess &&
              hipMalloc(&c->G.stamp, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.ovf[0], sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->G.ovf[1], sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->B.brick_state, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->B.active, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->B.gindex, sizeof(int) * nb) == hipSuccess &&
              hipMalloc(&c->ctl, sizeof(int) * CTL_ALLOC_WORDS) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        c->err = "grid allocation failed";
        return bail(MPM_ENOMEM);
    }
    if (hipMemsetAsync(c->G.acc, 0, sizeof(float) * 4 * 64 * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.vel, 0, sizeof(float4) * 64 * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G.stamp, 0xff, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->B.brick_state, 0, sizeof(int) * nb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ctl, 0, sizeof(int) * CTL_ALLOC_WORDS, c->stream) != hipSuccess) {
        c->err = "initialisation failed";
        return bail(MPM_EDEVICE);
    }
    if (hipHostMalloc(&c->ring, sizeof(int) * RING, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&c->ring_dev), c->ring, 0) != hipSuccess) {
        (void)hipGetLastError();
        c->err = "pinned ring allocation failed";
        return bail(MPM_ENOMEM);
    }
    memset(c->ring, 0, sizeof(int) * RING);
    for (int i = 0; i < RING; ++i)
        if (hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming) != hipSuccess) {
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
    free_particle_buffers(c);
    (void)hipFree(c->G.acc);
    (void)hipFree(c->G.vel);
    (void)hipFree(c->G.stamp);
    (void)hipFree(c->G.ovf[0]);
    (void)hipFree(c->G.ovf[1]);
    (void)hipFree(c->B.brick_state);
    (void)hipFree(c->B.active);
    (void)hipFree(c->B.gindex);
    (void)hipFree(c->ctl);
    if (c->ring) (void)hipHostFree(c->ring);
    for (int i = 0; i < RING; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
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
    if (scene != 0) return fail(c, MPM_EINVAL, "scene must be 0");
    if (count < 0 || (count > 0 && !x)) return fail(c, MPM_EINVAL, "bad count or null positions");
    if (c->N + count > (int64_t)1 << 30) return fail(c, MPM_EINVAL, "too many particles");
    if (mat) {
        if (mat->kind < 0 || mat->kind > 2) return fail(c, MPM_EINVAL, "bad material kind");
        if (!(mat->ppc > 0) || !(mat->rho > 0)) return fail(c, MPM_EINVAL, "ppc and rho must be positive");
        if (mat->kind != MPM_WATER && !(mat->nu > -1.0f && mat->nu < 0.5f)) return fail(c, MPM_EINVAL, "bad nu");
        if (c->has_mat && !same_material(c->mat, *mat))
            return fail(c, MPM_EINVAL, "a context holds one material; pass the same constants or NULL");
        if (!c->has_mat) {
            c->mat = *mat;
            c->has_mat = true;
            c->M = derive_material(*mat, c->P);
        }
    } else if (!c->has_mat) {
        return fail(c, MPM_EINVAL, "the first call must pass a material");
    }
    if (count == 0) return MPM_OK;
    if (c->N + count > c->cap / 2) {
        int64_t newcap = c->cap;
        while (c->N + count > newcap / 2) newcap *= 4;
        int r = grow(c, newcap);
        if (r) return r;
    }
    if (c->pending) {  // land the deferred update so old and new particles share one state convention
        enqueue_materialize(c->stream, c->P, c->M, c->S[c->cur], c->cap, (int)c->N);
        c->pending = 0;
    }
    enqueue_insert(c->stream, c->S[c->cur], c->ids[c->cur], c->cap, (int)c->N, (int)count, x, v, C, F, s, c->ctl);
    HIP_OK(c, hipGetLastError());
    c->N += count;
    c->need_rebuild = true;
    return MPM_OK;
}

// In-zone particles that may lose their chunk's tile in one substep before
// the next substep asks for a rebuild (1/256 of the particles).  With
// MPM_FLAG_MANUAL_REBUILD the request is ignored like the free-zone one.
int fb_limit(const mpm_ctx* c) { return (int)(c->N >> 8); }

int mpm_substep(mpm_ctx* c, int32_t nsteps) {
    if (!c) return MPM_EINVAL;
    if (nsteps < 0) return fail(c, MPM_EINVAL, "negative step count");
    if (c->N == 0) return MPM_OK;
    const int N = (int)c->N;
    for (int k = 0; k < nsteps; ++k) {
        int r = poll_flags(c, c->step - c->cfg.lag);
        if (r) return r;
        if (c->need_rebuild || (c->cfg.flags & MPM_FLAG_REBUILD_EVERY_STEP)) {
            int slot;
            if ((r = prof_begin(c, 0, &slot))) return r;
            enqueue_rebuild(c->stream, c->P, c->S[c->cur], c->S[c->cur ^ 1], c->ids[c->cur], c->ids[c->cur ^ 1],
                            c->cap, N, c->cfg.chunk, (c->cfg.flags & MPM_FLAG_P2G_SORTED_LANES) ? 0 : 1, c->B,
                            c->ctl, c->nbricks);
            if ((r = prof_end(c, slot))) return r;
            c->cur ^= 1;
            c->need_rebuild = false;
            c->last_rebuild = c->step;
            c->n_at_rebuild = c->N;
            ++c->rebuilds;
        }
        const int rs = (int)(c->step % RING);
        c->ring[rs] = 0;
        const int parity = (int)(c->step & 1);
        int slot;
        if ((r = prof_begin(c, 1, &slot))) return r;
        enqueue_p2g(c->stream, c->L, c->P, c->M, c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->G, c->B.brick_state,
                    c->pending, parity, (c->cfg.flags & MPM_FLAG_P2G_GLOBAL_ATOMICS) ? 1 : 0, c->nbricks,
                    c->cfg.chunk);
        if ((r = prof_end(c, slot))) return r;
        if ((r = prof_begin(c, 2, &slot))) return r;
        enqueue_grid(c->stream, c->L, c->P, c->B, c->ctl, c->G, parity, (int)c->step);
        if ((r = prof_end(c, slot))) return r;
        if ((r = prof_begin(c, 3, &slot))) return r;
        enqueue_g2p(c->stream, c->L, c->P, c->S[c->cur], c->cap, c->B.chunks, c->ctl, c->G, c->ring_dev + rs,
                    (c->cfg.flags & MPM_FLAG_G2P_GLOBAL_GATHER) ? 0 : 1, parity, fb_limit(c), c->cfg.chunk);
        if ((r = prof_end(c, slot))) return r;
        HIP_OK(c, hipGetLastError());
        HIP_OK(c, hipEventRecord(c->ev[rs], c->stream));
        c->pending = 1;
        ++c->step;
    }
    return MPM_OK;
}

int mpm_frame(mpm_ctx* c, float frame_dt) {
    if (!c) return MPM_EINVAL;
    if (!(frame_dt > 0.0f)) return fail(c, MPM_EINVAL, "frame_dt must be positive");
    const double ns = (double)frame_dt / (double)c->cfg.dt;
    int n = (int)ns;
    if (ns - n > 1e-4) ++n;
    if (n < 1) n = 1;
    return mpm_substep(c, n);
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
    if (scene != 0 || count != c->N) return fail(c, MPM_EINVAL, "count must equal the particle count of scene 0");
    enqueue_read(c->stream, c->P, c->M, c->S[c->cur], c->ids[c->cur], c->cap, (int)c->N, c->pending, x, v, C, F, s);
    HIP_OK(c, hipGetLastError());
    return check_error_word(c);
}

int mpm_read_grid(mpm_ctx* c, int32_t scene, float* m, float* v) {
    if (!c) return MPM_EINVAL;
    if (scene != 0) return fail(c, MPM_EINVAL, "scene must be 0");
    enqueue_read_grid(c->stream, c->P, c->G, (int)(c->step - 1), m, v);
    HIP_OK(c, hipGetLastError());
    return check_error_word(c);
}

int mpm_read_binning(mpm_ctx* c, int32_t scene, int64_t count, uint32_t* keys, int32_t* perm) {
    if (!c) return MPM_EINVAL;
    if (scene != 0) return fail(c, MPM_EINVAL, "scene must be 0");
    if (c->last_rebuild < 0) return fail(c, MPM_EINVAL, "no rebuild has run yet");
    if (count != c->n_at_rebuild) return fail(c, MPM_EINVAL, "count must equal the particle count at the last rebuild");
    if (keys)
        HIP_OK(c, hipMemcpyAsync(keys, c->B.keys[c->B.sorted], sizeof(uint32_t) * count, hipMemcpyDeviceToDevice,
                                 c->stream));
    if (perm)
        HIP_OK(c, hipMemcpyAsync(perm, c->B.sorted_ids, sizeof(int32_t) * count, hipMemcpyDeviceToDevice, c->stream));
    return check_error_word(c);
}

int mpm_read_blocks(mpm_ctx* c, int32_t scene, uint32_t* gcode, int32_t* gstart, int32_t* gcount, int32_t* active) {
    if (!c) return MPM_EINVAL;
    if (scene != 0) return fail(c, MPM_EINVAL, "scene must be 0");
    int h[CTL_WORDS];
    HIP_OK(c, hipMemcpyAsync(h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    const int ng = h[CTL_NGB], na = h[CTL_NACTIVE];
    if (gcode) HIP_OK(c, hipMemcpy(gcode, c->B.gcode, sizeof(uint32_t) * ng, hipMemcpyDeviceToHost));
    if (gstart || gcount) {
        std::vector<int> st(ng + 1);
        HIP_OK(c, hipMemcpy(st.data(), c->B.gstart, sizeof(int) * ng, hipMemcpyDeviceToHost));
        st[ng] = (int)c->n_at_rebuild;
        for (int i = 0; i < ng; ++i) {
            if (gstart) gstart[i] = st[i];
            if (gcount) gcount[i] = st[i + 1] - st[i];
        }
    }
    if (active) HIP_OK(c, hipMemcpy(active, c->B.active, sizeof(int) * na, hipMemcpyDeviceToHost));
    return h[CTL_ERROR] ? fail(c, MPM_ESTATE, "device error word set") : MPM_OK;
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
    o->overflow_blocks = c->step > 0 ? h[CTL_OVF + ((c->step - 1) & 1)] : 0;
    o->error = (uint32_t)h[CTL_ERROR];
    o->pending_update = (uint32_t)c->pending;
    unsigned long long c64[CTL64_WORDS];
    memcpy(c64, h + CTL_WORDS, sizeof c64);
    o->p2g_fallback_chunks = (int64_t)c64[CTL64_FALLBACK_CHUNKS];
    o->p2g_global_particles = (int64_t)c64[CTL64_GLOBAL_PARTICLES];
    return o->error ? fail(c, MPM_ESTATE, "device error word set") : MPM_OK;
}

int mpm_clear_error(mpm_ctx* c) {
    if (!c) return MPM_EINVAL;
    HIP_OK(c, hipMemsetAsync(c->ctl + CTL_ERROR, 0, sizeof(int), c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return MPM_OK;
}

int mpm_profile(mpm_ctx* c, uint32_t mask) {
    if (!c) return MPM_EINVAL;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->prof) p.live = false;
    c->prof_mask = 0;
    for (int i = 0; i < 4; ++i) {
        if (mask & (1u << i)) c->prof_mask |= 1u << i;
        c->prof_launch[i] = 0;
        c->prof_ms[i] = 0.0;
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
