/*
 * mpm.h -- C ABI of the MI355X (gfx950) explicit MLS-MPM substep library.
 *
 * The library advances particles with the five-phase explicit MPM step the
 * paper lays out in "Material Point Method on a Single GPU": rebuild-mapping,
 * sort-particle, particle-to-grid transfer (P2G, with the material update and
 * stress fused in), grid update (with boundary conditions and buffer clearing
 * fused in), and grid-to-particle transfer (G2P).  Rebuild-mapping and sorting
 * run only when a particle leaves its free zone ("Minimize nonessential
 * computations", subsection "Rebuild-Mapping").  The transfer scheme is
 * MLS-MPM with APIC and quadratic B-splines (the Results section builds on
 * MLS-MPM).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an mpm_status (0 = MPM_OK, negative = error)
 *     and never throws.  mpm_last_error() returns a message for the last
 *     failure on that context.
 *   - Pointers named *_dev are DEVICE pointers (hipMalloc'd or a torch CUDA
 *     tensor's data_ptr()) on the context's device.  The caller owns them;
 *     the library never frees them and never keeps them after the call's
 *     work has run on the stream.  Other pointers are host pointers.
 *   - All device work is enqueued on config.stream in stream order; a caller
 *     that reads outputs on another stream must synchronize first.  The
 *     read/stats calls synchronize the stream themselves.
 *   - Particle arrays are structure-of-arrays FP32: x and v are [3][count]
 *     (all x components, then y, then z); C and F are [9][count] with entry
 *     (a,b) at component a*3+b; s is [count] (J_P for snow, J for water,
 *     ignored for jelly).
 *   - A context is single-threaded: do not call into one context from two
 *     threads at once.  Different contexts are independent.
 *   - A context holds 1..256 independent scenes (config.num_scenes).  Each
 *     scene has its own grid, time step, material and particles; a batched
 *     context advances all of them with one launch per phase per substep
 *     (the particle code carries the scene in its top bits, so one sort and
 *     one work list cover every scene).
 *   - Faults the device detects (non-finite state, a particle stencil
 *     leaving the grid, capacity exceeded) set a sticky error word; the next
 *     mpm_read_* or mpm_get_stats call returns MPM_ESTATE, and the word stays
 *     set until mpm_clear_error().
 *   - Statistics are read with mpm_get_stats (the counters a "stats" call
 *     returns).  A trained network is loaded in two calls: mpm_surrogate_set
 *     puts parameters and normalisation into a surrogate object, and
 *     mpm_use_surrogate lets a scene take it, so one network can serve
 *     several contexts.
 */
#ifndef MPM_H
#define MPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ctx mpm_ctx; /* opaque; created and owned by the library */

typedef enum {
    MPM_OK = 0,
    MPM_EINVAL = -1,  /* bad argument; nothing was enqueued */
    MPM_ENOMEM = -2,  /* a device or pinned allocation failed; context unchanged */
    MPM_EDEVICE = -3, /* a HIP call failed; the context should be destroyed */
    MPM_ESTATE = -4   /* the sticky device error word is set */
} mpm_status;

typedef enum { MPM_JELLY = 0, MPM_SNOW = 1, MPM_WATER = 2, MPM_SAND = 3 } mpm_kind;
typedef enum { MPM_BC_STICKY = 0, MPM_BC_SLIP = 1, MPM_BC_SEPARATE = 2 } mpm_bc;

/* bits of the sticky device error word */
#define MPM_ERR_NONFINITE 0x1u /* a particle position/velocity became NaN or Inf */
#define MPM_ERR_DOMAIN 0x2u    /* a particle's 3x3x3 stencil left nodes [0, n] */
#define MPM_ERR_CAPACITY 0x4u  /* an internal list overflowed */

/* config.flags */
#define MPM_FLAG_REBUILD_EVERY_STEP 0x1u /* disable the free zone: rebuild and sort before every substep */
#define MPM_FLAG_P2G_GLOBAL_ATOMICS 0x2u /* P2G scatters straight to global atomics (no LDS tile) */
#define MPM_FLAG_MANUAL_REBUILD 0x4u     /* ignore the free-zone flag: rebuild only after mpm_add_particles
                                            or mpm_rebuild (particles outside their free zone still
                                            transfer exactly, through global atomics) */
#define MPM_FLAG_G2P_GLOBAL_GATHER 0x10u /* G2P gathers every node from the dense grid instead of an LDS
                                            copy of the chunk's node box */
#define MPM_FLAG_P2G_SORTED_LANES 0x8u   /* store each chunk in plain sorted order instead of the
                                            order that deals it over the LDS passes by bank */
#define MPM_FLAG_FRAME_GRAPHS 0x20u      /* mpm_frame replays a whole frame (every scene's substeps, G2P
                                            inside the next P2G) as a HIP graph: four recordings, by
                                            particle-buffer parity and with or without a rebuild at the
                                            frame's start, picked from the rebuild request the previous
                                            frame left and from the exit horizon: the substeps before a
                                            particle could move 3 cells at the mean particle speed and
                                            the gravity (reduced at the end of each graph frame).  Within
                                            a graph frame the free-zone flag is not acted on (a particle that leaves its
                                            zone transfers through global atomics until the next frame);
                                            when the horizon is shorter than the frame, the frame runs
                                            directly instead.  Needs config.stream != 0.  The graphs are
                                            recorded again after mpm_add_particles, a new frame_dt or a
                                            new chunk size.                                            */
#define MPM_FLAG_FUSED_G2P 0x40u        /* run each substep's G2P inside the next substep's P2G (the
                                            default; see mpm_substep)                                  */
#define MPM_FLAG_SEPARATE_G2P 0x80u     /* never: every substep launches its own G2P               */
/* Ablations of the paper's "Merge Kernels" and "Reduce memory reallocation"
 * (slower on purpose; results are unchanged):                              */
#define MPM_FLAG_SEPARATE_WALLS 0x100u  /* the wall condition as a launch of its own after the grid update */
#define MPM_FLAG_SEPARATE_CLEAR 0x200u  /* clearing the global accumulators as a launch of its own         */
#define MPM_FLAG_ALLOC_EXACT 0x400u     /* mpm_add_particles grows the particle buffers to exactly what is
                                           needed instead of 4x when half full (every emission reallocates) */
#define MPM_FLAG_CHUNK_PER_BLOCK 0x800u /* each work chunk holds the particles of one block only, instead of
                                           consecutive blocks packed up to the chunk size (the paper's
                                           "virtual blocks" of Gao et al.: more, emptier workgroups) */

#define MPM_MAX_SCENES 256

/* Grid and time step of one scene of a batched context. */
typedef struct {
    int32_t n;        /* cells per axis, power of two in [16, 512] */
    int32_t bc;       /* mpm_bc */
    int32_t bc_cells; /* wall thickness in cells */
    float gravity[3];
    float dt;         /* substep length of this scene (> 0) */
} mpm_scene;

typedef struct {
    int32_t n;          /* cells per axis on the unit cube; power of two, 16 <= n <= 512; dx = 1/n */
    int32_t bc;         /* mpm_bc applied on nodes with a coordinate < bc_cells or > n - bc_cells */
    int32_t bc_cells;   /* wall thickness in cells (>= 0) */
    int32_t num_scenes; /* 1..MPM_MAX_SCENES; with S scenes and largest n = 2^L, 3L + ceil(log2 S) <= 32 */
    float gravity[3];   /* m/s^2 */
    float dt;           /* substep length in seconds (> 0) */
    int64_t capacity;   /* initial particle reservation; grows 4x when more than half full */
    uint64_t stream;    /* hipStream_t as an integer (e.g. torch.cuda.Stream.cuda_stream); 0 = null stream */
    uint32_t flags;     /* MPM_FLAG_* */
    int32_t lag;        /* substeps the host may run ahead of the device before it must read the
                           rebuild flag (1..64; 0 selects the default 5).  Substeps are marked
                           in groups (every 4th substep with lag >= 5, every 2nd with lag >= 3),
                           so a flag is read once its group has ended */
    int32_t chunk;      /* particles per P2G/G2P work chunk: 64..512, multiple of 64 (0 = 256) */
    int32_t reserved;
    const mpm_scene* scenes; /* num_scenes descriptors (copied), or NULL: every scene takes n, bc,
                                bc_cells, gravity and dt from this struct */
} mpm_config;

/* Material constants.  Lame parameters mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu));
 * particle volume V0 = dx^3/ppc and mass rho V0.
 *   jelly: fixed-corotated elasticity (E, nu)
 *   snow : fixed-corotated with hardening exp(xi (1 - J_P)) and singular values
 *          clamped to [1 - theta_c, 1 + theta_s]
 *   water: tau = bulk (J - 1) J I
 *   sand : a stand-in for the sand model the paper cites (not given in it):
 *          Hencky elasticity tau = U diag(2 mu eps + lambda tr eps) U^T with
 *          eps = log |sig| (floored at log 1e-6), and the Drucker-Prager
 *          return map of Klar et al. 2016 in logarithmic strain: expansion
 *          (tr eps > 0) releases all elastic strain; otherwise, with d the
 *          deviator of eps and dg = |d| + (3 lambda + 2 mu)/(2 mu) tr eps alpha,
 *          dg > 0 scales d down by dg (the volume is kept).  alpha =
 *          sqrt(2/3) 2 sin phi / (3 - sin phi) for the friction angle
 *          phi = h0 + (h1 q - h3) exp(-h2 q) degrees, q the hardening state,
 *          which grows by the log strain each return map removes.  The
 *          particle's s holds 1 + q (so the default s = 1 is q = 0).        */
typedef struct {
    int32_t kind; /* mpm_kind */
    float E, nu, rho, ppc, theta_c, theta_s, xi, bulk;
    float h0, h1, h2, h3; /* sand hardening constants (degrees, degrees, 1, degrees); ignored otherwise */
} mpm_material;

typedef struct {
    int64_t num_particles;
    int64_t capacity;
    int64_t substeps;        /* substeps enqueued so far */
    int64_t rebuilds;        /* rebuild-mapping + sort passes enqueued so far */
    int64_t gblocks;         /* particle (geometric) blocks at the last rebuild */
    int64_t active_blocks;   /* physical blocks (3x3x3 dilation of the gblocks) at the last rebuild */
    int64_t chunks;          /* work chunks at the last rebuild */
    int64_t overflow_blocks; /* blocks touched outside the physical set in the last substep */
    uint32_t error;          /* sticky MPM_ERR_* bits */
    uint32_t pending_update; /* 1 if the deformation update of the last G2P is deferred to the next P2G */
    /* running totals since mpm_create (all substeps):                                   */
    int64_t p2g_fallback_chunks;  /* chunks whose stencil box exceeded the LDS tile; their particles
                                     scattered with global atomics                          */
    int64_t p2g_global_particles; /* particle transfers done with global atomics (particles outside
                                     their free zone, plus those of fallback chunks)        */
    int64_t surrogate_particles;  /* snow return maps done without SVD (mpm_use_surrogate)  */
    int64_t surrogate_fallbacks;  /* ... that fell back to the exact map                    */
} mpm_stats;

/* Phases that mpm_profile can bracket with HIP events. */
#define MPM_PHASE_REBUILD 0x1u
#define MPM_PHASE_P2G 0x2u
#define MPM_PHASE_GRID 0x4u
#define MPM_PHASE_G2P 0x8u
/* Bracket only every n-th launch of each phase (n in 1..65535), so that the
 * events (each a few microseconds of stream time) barely disturb what is
 * being measured. */
#define MPM_PROFILE_EVERY(n) ((uint32_t)(n) << 16)

typedef struct {
    int64_t launches[4]; /* rebuild, p2g, grid, g2p */
    double ms[4];        /* summed event-measured device time per phase */
} mpm_profile_data;

/* Create a context on the current HIP device.  cfg (and cfg->scenes) is
 * copied.  Fails with MPM_EINVAL on a bad field, MPM_ENOMEM if the dense
 * block grids (per scene (n/4+2)^3 blocks x 64 nodes x 32 B) or the particle
 * buffers do not fit. */
int mpm_create(const mpm_config* cfg, mpm_ctx** out);

/* Synchronize the stream and free everything the context owns.  NULL is OK. */
int mpm_destroy(mpm_ctx* ctx);

/* Append `count` particles to `scene` (0 <= scene < num_scenes).  x_dev is
 * required; v_dev, C_dev, F_dev, s_dev may be NULL (defaults 0, 0, I, 1).
 * The first call for a scene fixes that scene's material; later calls must
 * pass the same constants or NULL.  Particles of a scene are numbered in
 * insertion order (0, 1, ...), the order mpm_read_particles returns.  Grows
 * capacity 4x when the total exceeds half of it (no other call allocates,
 * except graph recording in mpm_frame).  Forces a rebuild before the next
 * substep.  Particle generation ("Fountain": a per-frame source) is done by
 * calling this between substeps.                                            */
int mpm_add_particles(mpm_ctx* ctx, int32_t scene, const mpm_material* mat, int64_t count,
                      const float* x_dev, const float* v_dev, const float* C_dev, const float* F_dev,
                      const float* s_dev);

/* Enqueue `nsteps` substeps of every scene.  Each is: [rebuild-mapping + sort
 * when a particle left its free zone] -> P2G -> grid update -> G2P, one launch
 * per phase for all scenes.  A substep's G2P runs inside the next substep's
 * P2G launch (paper, "Merge Kernels": G2P2G) unless MPM_FLAG_SEPARATE_G2P,
 * MPM_FLAG_P2G_GLOBAL_ATOMICS,
 * MPM_FLAG_REBUILD_EVERY_STEP, MPM_FLAG_G2P_GLOBAL_GATHER, ASFLIP or a
 * learned / closed-form return map is in use.
 * Calls that read, extend, sample or rebuild the state run the outstanding
 * G2P first, so what they see does not change.  The host waits for the
 * device only to keep at most `lag` substeps in flight, so that it can read
 * the device's rebuild flag; it never drains the stream.                    */
int mpm_substep(mpm_ctx* ctx, int32_t nsteps);

/* Advance one frame (frame_dt > 0): scene s runs ceil(frame_dt/dt_s)
 * substeps.  The frame takes as many launches per phase as the longest
 * scene needs; scenes that are done sit out the remaining launches.  With
 * MPM_FLAG_FRAME_GRAPHS the frame is a replayed HIP graph.                  */
int mpm_frame(mpm_ctx* ctx, float frame_dt);

/* Force rebuild-mapping and sorting before the next substep.              */
int mpm_rebuild(mpm_ctx* ctx);

/* Block until every enqueued operation of the context has finished.       */
int mpm_synchronize(mpm_ctx* ctx);

/* Copy the particles of `scene` into caller device arrays, in insertion
 * order.  count must equal the scene's particle count.  Any output may be
 * NULL.  F/s are the state after the last G2P's deformation update (the
 * update is applied on the fly when it is still deferred; in a context where
 * a snow scene takes the learned or closed-form map, it is first landed in
 * the stored state with each scene's own map, as the next P2G would apply
 * it).  Synchronizes.                                                      */
int mpm_read_particles(mpm_ctx* ctx, int32_t scene, int64_t count, float* x_dev, float* v_dev, float* C_dev,
                       float* F_dev, float* s_dev);

/* Dense view of the scene's grid after its last substep (test/debug use):
 * m_dev [(n+1)^3] node masses and v_dev [3][(n+1)^3] updated node velocities,
 * node (i,j,k) at ((i*(n+1))+j)*(n+1)+k, i along x.  Nodes the last substep
 * did not touch read as zero.  Either pointer may be NULL.  Synchronizes.  */
int mpm_read_grid(mpm_ctx* ctx, int32_t scene, float* m_dev, float* v_dev);

/* The binning of the scene at the last rebuild: keys_dev[count] the sorted
 * particle codes (the scene's Morton code, without scene bits) and
 * perm_dev[count] the scene-local insertion index of the particle at each
 * sorted position (a stable sort: ties keep their storage order before the
 * rebuild).  Storage layout after a rebuild: scenes in order of increasing dt
 * (ties by scene index), inside a scene geometric blocks in code order;
 * chunks of at most config.chunk particles: consecutive blocks of one
 * 2x2x1 slab of blocks (equal block code >> 2) share a chunk while they fit
 * (each block a chunk of its own with MPM_FLAG_CHUNK_PER_BLOCK), a larger
 * block is cut into runs of config.chunk; inside a chunk of
 * `count` particles the particles are ranked by the bank pair
 * (x + 12 y + 8 z) mod 16 of their cell (x, y, z), then by block and cell
 * code, ties in sorted order, and rank r is stored at slot 16 p + q of the
 * chunk, where the ranks are dealt place by place (q = 0, 1, ...) over the
 * chunk's P = ceil(count / 16) passes in the pass order 0, 2, 4, ..., 1, 3,
 * 5, ..., the last pass (count - 16 (P - 1) places) dropping out once full
 * (plain sorted order with MPM_FLAG_P2G_SORTED_LANES).
 * count must equal the scene's particle count at the last rebuild.
 * Synchronizes.                                                             */
int mpm_read_binning(mpm_ctx* ctx, int32_t scene, int64_t count, uint32_t* keys_dev, int32_t* perm_dev);

/* Blocks of the scene at the last rebuild (host arrays, sized by
 * mpm_get_scene_stats): gcode[gblocks] block codes (particle code >> 6)
 * ascending, gstart/gcount their ranges in the scene's sorted order,
 * active[active_blocks] the physical blocks as padded linear codes
 * ((bz*NB)+by)*NB+bx with b = block coordinate + 1 and NB = n/4 + 2,
 * ascending.  Any pointer may be NULL.  Synchronizes.                       */
int mpm_read_blocks(mpm_ctx* ctx, int32_t scene, uint32_t* gcode, int32_t* gstart, int32_t* gcount,
                    int32_t* active);

/* Synchronize and report counters (totals over all scenes).  Returns
 * MPM_ESTATE if the error word is set (the struct is still filled).         */
int mpm_get_stats(mpm_ctx* ctx, mpm_stats* out);

typedef struct {
    int64_t num_particles;
    int64_t substeps;      /* substeps this scene has taken */
    int64_t gblocks;       /* at the last rebuild */
    int64_t active_blocks; /* at the last rebuild */
    int32_t n;
    float dt;
} mpm_scene_stats;

/* Per-scene counters.  Synchronizes.                                        */
int mpm_get_scene_stats(mpm_ctx* ctx, int32_t scene, mpm_scene_stats* out);

/* Pick the chunk size (particles per P2G/G2P workgroup: 128, 256 or 512)
 * that advances the current state fastest: each candidate runs `frames`
 * frames of frame_dt from a device copy of the current state, timed with
 * HIP events; the state and counters are then restored and the winner kept
 * (written to *chunk_out if not NULL).  The copy takes one more particle
 * buffer of device memory for the duration of the call.  Synchronizes.     */
int mpm_autotune(mpm_ctx* ctx, float frame_dt, int32_t frames, int32_t* chunk_out);

/* Clear the sticky device error word.                                      */
int mpm_clear_error(mpm_ctx* ctx);

/* Bracket the phases in `phase_mask` (MPM_PHASE_*, optionally with
 * MPM_PROFILE_EVERY(n)) of every later substep, or of every n-th launch of
 * each phase, with HIP events on the context's stream; 0 turns it off.
 * Synchronizes and resets the accumulated data.                             */
int mpm_profile(mpm_ctx* ctx, uint32_t phase_mask);

/* Synchronize and return the accumulated per-phase launch counts and
 * event-measured device times since the last mpm_profile call.           */
int mpm_profile_read(mpm_ctx* ctx, mpm_profile_data* out);

/* Message for the last failed call on ctx (or of mpm_create when ctx is
 * NULL).  Owned by the library; valid until the next call on that context. */
const char* mpm_last_error(const mpm_ctx* ctx);

/* ASFLIP transfer for `scene` (the integrator the paper's fountain uses,
 * "Fountain" in its Results section, after Fei et al. 2021; the formulas are
 * not in the paper, this is the library's reading of them).  With v the
 * particle's velocity before the substep, v^ = sum w v_i' the interpolated
 * new grid velocity, v- = sum w v~_i the interpolated grid velocity the
 * particles transferred (v~_i = p_i / m_i, before gravity and walls):
 *   v' = v^ + flip (v - v-)                     (flip = 1: FLIP, 0: APIC)
 *   x' = x + dt (v^ + beta flip (v - v-))       (beta = 0: positions by PIC)
 * with beta = beta_max unless the particle's volume is being compressed
 * (J' < 1, J' = J det(I + dt C') for water and det(I + dt C') otherwise),
 * where beta = beta_min.  C' stays the APIC gradient of the new grid
 * velocity.  flip = 0 restores APIC.  Needs 0 <= flip <= 1 and 0 <= beta_min
 * <= beta_max <= 1 (else MPM_EINVAL).  The first call with flip > 0
 * allocates one float4 per node of the context's block grids; scenes with
 * flip > 0 run G2P as its own launch (no G2P2G fusion).                    */
int mpm_set_transfer(mpm_ctx* ctx, int32_t scene, float flip, float beta_min, float beta_max);

/* Automatic time step (single-scene contexts; the paper's fountain and snow
 * runs deduce their steps automatically, after Fang et al. 2018; this is the
 * library's reading): at the start of every mpm_frame the step becomes
 *   dt = min(dt_max, cfl dx / (max_p |v_p| + |g| frame_dt + c))
 * with c the material's pressure-wave speed (sqrt(bulk/rho) for water,
 * sqrt((lambda + 2 mu)/rho) otherwise), then frame_dt / ceil(frame_dt / dt),
 * so the frame's substeps tile it.  The largest speed is read back from the
 * device (one synchronization per frame).  cfl = 0 turns it off (the step
 * stays where it is); otherwise 0 < cfl <= 1 and dt_max > 0.  mpm_substep
 * keeps the current step.  MPM_EINVAL for a batched context.               */
int mpm_set_auto_dt(mpm_ctx* ctx, float cfl, float dt_max);

/* ------------------------------------------------ learned snow surrogate
 * An MLP 12 -> 64 -> 64 -> 12 (tanh hidden layers, linear output) standing
 * in for the snow return map and stress in principal space.  Inputs, for
 * trial singular values s (descending) and plastic volume J_P:
 *   [s1..s3, ln s1..s3, J_P, ln J_P, exp(xi (1 - J_P)), dt/dt_ref, s1 s2 s3, 1]
 * targets: [s'1..s'3, ln(s'/s)1..3, tau1..3 / E, J_P'/J_P, exp(xi (1 - J_P')), s'1 s'2 s'3]
 * with s' the projected singular values and tau the principal Kirchhoff
 * stress.  The network works on z-scored inputs and targets (means and
 * standard deviations held with the parameters).  Rows are [count][12] FP32.
 * Parameters: flat FP32 [W1 (64x12), b1, W2 (64x64), b2, W3 (12x64), b3],
 * weights row-major (output, input).  All pointers are device pointers. */
typedef struct mpm_surrogate mpm_surrogate;

#define MPM_SUR_IN 12
#define MPM_SUR_OUT 12
#define MPM_SUR_PARAMS 5772
#define MPM_SUR_NORM 48 /* input means, input sds, output means, output sds (12 each) */
#define MPM_SUR_FP32 0  /* FP32 operands (gradient checking) */
#define MPM_SUR_BF16 1  /* BF16 operands, FP32 accumulation (MFMA) */

/* Create on the current device, work enqueued on `stream` (0 = null
 * stream).  Parameters start at zero and the normalisation at identity. */
int mpm_surrogate_create(uint64_t stream, mpm_surrogate** out);
int mpm_surrogate_destroy(mpm_surrogate* s);
/* Copy parameters / normalisation in or out; either pointer may be NULL. */
int mpm_surrogate_set(mpm_surrogate* s, const float* theta_dev, const float* norm_dev);
int mpm_surrogate_get(mpm_surrogate* s, float* theta_dev, float* norm_dev);
/* Y = network(X) in physical (de-normalised) units.  MPM_SUR_BF16 runs the
 * inference path P2G runs: weights rounded to BF16 once as they are staged,
 * BF16 MFMA with FP32 accumulation, P2G's input normalisation.              */
int mpm_surrogate_forward(mpm_surrogate* s, int32_t precision, int64_t count, const float* X_dev, float* Y_dev);
/* Mean over the rows of 1/2 |y~ - t~|^2 in z-scored units into loss_dev[0]
 * and its gradient into grad_dev[MPM_SUR_PARAMS].                          */
int mpm_surrogate_loss_grad(mpm_surrogate* s, int32_t precision, int64_t count, const float* X_dev,
                            const float* T_dev, float* grad_dev, float* loss_dev);
/* Set the normalisation to the column means and standard deviations
 * (floored at 1e-6) of X and T.                                             */
int mpm_surrogate_fit_norm(mpm_surrogate* s, int64_t count, const float* X_dev, const float* T_dev);
/* `steps` Adam steps (lr, betas 0.9 / 0.999, eps 1e-8; the step counter
 * continues across calls) on minibatches of `batch` rows drawn uniformly
 * with replacement by a counter-based generator (splitmix64 of seed, step
 * and row), BF16 MFMA forward/backward.  loss_host (may be NULL) receives the
 * minibatch loss of every step.  Synchronizes.                            */
int mpm_surrogate_train(mpm_surrogate* s, int64_t count, const float* X_dev, const float* T_dev, int32_t steps,
                        int32_t batch, float lr, uint64_t seed, float* loss_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc):
 * mpm_surrogate_train with its scratch -- the minibatch row indices and the
 * per-step losses, which mpm_surrogate_train allocates on demand -- in a
 * fixed device array that the library holds for the life of the process
 * (one per device, MPM_SUR_NOALLOC_MAX_BATCH + MPM_SUR_NOALLOC_MAX_STEPS
 * 32-bit words, 272 KiB).  Arguments, results and the synchronization at the
 * end are those of mpm_surrogate_train; the same seed gives the same
 * minibatches.  batch > MPM_SUR_NOALLOC_MAX_BATCH or steps >
 * MPM_SUR_NOALLOC_MAX_STEPS fails with MPM_EINVAL before anything is
 * enqueued.  Calls nothing that allocates (no hipMalloc, hipFree or
 * allocating library routine); the surrogate's parameters and Adam state
 * come from mpm_surrogate_create.  Every call on a device shares that
 * device's array: calls that overlap on one device (from any thread, stream
 * or surrogate) race, so the caller must order them.  The device current at
 * the call must be the surrogate's.                                        */
#define MPM_SUR_NOALLOC_MAX_BATCH 65536
#define MPM_SUR_NOALLOC_MAX_STEPS 4096
int mpm_surrogate_train_noalloc(mpm_surrogate* s, int64_t count, const float* X_dev, const float* T_dev,
                                int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss_host);
/* Training pairs from the current state of a snow scene: for every particle
 * (in storage order), the trial state of its next return map (the deferred
 * deformation update applied) through the exact return map, as inputs and
 * targets above.  Writes min(particles, max_count) rows; *written gets the
 * count.                                                                    */
/* Choose how P2G maps a snow scene's trial state (mode):
 *   0  exact: singular values by Jacobi rotations, clamp, stress (default);
 *   1  the surrogate s predicts the projected singular values (as ln(s'/s))
 *      and J_P'/J_P; the stress is evaluated from that state and must agree
 *      with the network's principal stress outputs within tol (x E); F_E'
 *      and tau are rebuilt from the eigenvalues of F^ F^T by Sylvester's
 *      formula (no eigenvectors);
 *   2  the same eigenvector-free path with the exact clamp instead of the
 *      network (the method without the network).
 * Modes 1 and 2 fall back to mode 0 per particle when two eigenvalues of
 * F^ F^T are closer than 0.1 of their spread or the particle is inverted;
 * mode 1 also when a predicted singular value leaves [1 - theta_c,
 * 1 + theta_s] by more than tol or the total volume J_P det F_E changes by
 * more than tol (log).  dt_ref: the time step the surrogate was trained at.
 * The surrogate must outlive its use by ctx; one surrogate per context (the
 * last one passed).  Counts go to mpm_stats.surrogate_*.                   */
int mpm_use_surrogate(mpm_ctx* ctx, int32_t scene, const mpm_surrogate* s, int32_t mode, float tol, float dt_ref);

int mpm_surrogate_sample(mpm_ctx* ctx, int32_t scene, float dt_ref, int64_t max_count, float* X_dev, float* T_dev,
                         int64_t* written);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H */
