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
 *   - Faults the device detects (non-finite state, a particle stencil
 *     leaving the grid, capacity exceeded) set a sticky error word; the next
 *     mpm_read_* or mpm_get_stats call returns MPM_ESTATE, and the word stays
 *     set until mpm_clear_error().
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

typedef enum { MPM_JELLY = 0, MPM_SNOW = 1, MPM_WATER = 2 } mpm_kind;
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
                                            strided order that spreads a wave over cells */

typedef struct {
    int32_t n;          /* cells per axis on the unit cube; power of two, 16 <= n <= 512; dx = 1/n */
    int32_t bc;         /* mpm_bc applied on nodes with a coordinate < bc_cells or > n - bc_cells */
    int32_t bc_cells;   /* wall thickness in cells (>= 0) */
    int32_t num_scenes; /* must be 1 */
    float gravity[3];   /* m/s^2 */
    float dt;           /* substep length in seconds (> 0) */
    int64_t capacity;   /* initial particle reservation; grows 4x when more than half full */
    uint64_t stream;    /* hipStream_t as an integer (e.g. torch.cuda.Stream.cuda_stream); 0 = null stream */
    uint32_t flags;     /* MPM_FLAG_* */
    int32_t lag;        /* substeps the host may run ahead of the device before it must read the
                           rebuild flag (1..64; 0 selects the default 3) */
    int32_t chunk;      /* particles per P2G/G2P work chunk: 64..512, multiple of 64 (0 = 256) */
    int32_t reserved;
} mpm_config;

/* Material constants.  Lame parameters mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu));
 * particle volume V0 = dx^3/ppc and mass rho V0.
 *   jelly: fixed-corotated elasticity (E, nu)
 *   snow : fixed-corotated with hardening exp(xi (1 - J_P)) and singular values
 *          clamped to [1 - theta_c, 1 + theta_s]
 *   water: tau = bulk (J - 1) J I                                           */
typedef struct {
    int32_t kind; /* mpm_kind */
    float E, nu, rho, ppc, theta_c, theta_s, xi, bulk;
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
} mpm_stats;

/* Phases that mpm_profile can bracket with HIP events. */
#define MPM_PHASE_REBUILD 0x1u
#define MPM_PHASE_P2G 0x2u
#define MPM_PHASE_GRID 0x4u
#define MPM_PHASE_G2P 0x8u

typedef struct {
    int64_t launches[4]; /* rebuild, p2g, grid, g2p */
    double ms[4];        /* summed event-measured device time per phase */
} mpm_profile_data;

/* Create a context on the current HIP device.  cfg is copied.  Fails with
 * MPM_EINVAL on a bad field, MPM_ENOMEM if the dense block grid
 * ((n/4+2)^3 blocks x 64 nodes x 32 B) or the particle buffers do not fit. */
int mpm_create(const mpm_config* cfg, mpm_ctx** out);

/* Synchronize the stream and free everything the context owns.  NULL is OK. */
int mpm_destroy(mpm_ctx* ctx);

/* Append `count` particles to `scene` (must be 0).  x_dev is required;
 * v_dev, C_dev, F_dev, s_dev may be NULL (defaults 0, 0, I, 1).  The first
 * call fixes the context's material; later calls must pass the same
 * constants or NULL.  Particles are numbered in insertion order (0, 1, ...),
 * the order mpm_read_particles returns.  Grows capacity 4x when the total
 * exceeds half of it (no other call allocates).  Forces a rebuild before
 * the next substep.  Particle generation ("Fountain": a per-frame source) is
 * done by calling this between substeps.                                    */
int mpm_add_particles(mpm_ctx* ctx, int32_t scene, const mpm_material* mat, int64_t count,
                      const float* x_dev, const float* v_dev, const float* C_dev, const float* F_dev,
                      const float* s_dev);

/* Enqueue `nsteps` substeps.  Each is: [rebuild-mapping + sort when a particle
 * left its free zone] -> P2G -> grid update -> G2P.  The host waits for the
 * device only to keep at most `lag` substeps in flight, so that it can read
 * the device's rebuild flag; it never drains the stream.                    */
int mpm_substep(mpm_ctx* ctx, int32_t nsteps);

/* Advance one frame: ceil(frame_dt/dt) substeps (frame_dt > 0).          */
int mpm_frame(mpm_ctx* ctx, float frame_dt);

/* Force rebuild-mapping and sorting before the next substep.              */
int mpm_rebuild(mpm_ctx* ctx);

/* Block until every enqueued operation of the context has finished.       */
int mpm_synchronize(mpm_ctx* ctx);

/* Copy the particles of `scene` into caller device arrays, in insertion
 * order.  count must equal the number of particles.  Any output may be
 * NULL.  F/s are the state after the last G2P's deformation update (the
 * update is applied on the fly when it is still deferred).  Synchronizes.  */
int mpm_read_particles(mpm_ctx* ctx, int32_t scene, int64_t count, float* x_dev, float* v_dev, float* C_dev,
                       float* F_dev, float* s_dev);

/* Dense view of the grid of the last substep (test/debug use): m_dev
 * [(n+1)^3] node masses and v_dev [3][(n+1)^3] updated node velocities,
 * node (i,j,k) at ((i*(n+1))+j)*(n+1)+k, i along x.  Nodes the last substep
 * did not touch read as zero.  Either pointer may be NULL.  Synchronizes.  */
int mpm_read_grid(mpm_ctx* ctx, int32_t scene, float* m_dev, float* v_dev);

/* The binning of the last rebuild: keys_dev[count] the sorted particle
 * codes and perm_dev[count] the insertion index of the particle at each
 * sorted position (a stable sort: ties keep their storage order before the
 * rebuild).  Storage layout after a rebuild: geometric blocks in code order,
 * each cut into chunks of config.chunk particles; inside a chunk of c
 * particles, slot t holds sorted position (t*K) mod c with K the smallest of
 * 9, 11, 13, 17 coprime to c (identity with MPM_FLAG_P2G_SORTED_LANES).
 * count must equal the number of particles at the last rebuild.
 * Synchronizes.                                                             */
int mpm_read_binning(mpm_ctx* ctx, int32_t scene, int64_t count, uint32_t* keys_dev, int32_t* perm_dev);

/* Blocks of the last rebuild (host arrays, sized by mpm_get_stats):
 * gcode[gblocks] block codes (particle code >> 6) ascending, gstart/gcount
 * their sorted-particle ranges, active[active_blocks] the physical blocks
 * as padded linear codes ((bz*NB)+by)*NB+bx with b = block coordinate + 1
 * and NB = n/4 + 2, ascending.  Any pointer may be NULL.  Synchronizes.     */
int mpm_read_blocks(mpm_ctx* ctx, int32_t scene, uint32_t* gcode, int32_t* gstart, int32_t* gcount,
                    int32_t* active);

/* Synchronize and report counters.  Returns MPM_ESTATE if the error word is set
 * (the struct is still filled).                                             */
int mpm_get_stats(mpm_ctx* ctx, mpm_stats* out);

/* Clear the sticky device error word.                                      */
int mpm_clear_error(mpm_ctx* ctx);

/* Bracket the phases in `phase_mask` (MPM_PHASE_*) of every later substep
 * with HIP events on the context's stream; 0 turns it off.  Resets the
 * accumulated data.                                                          */
int mpm_profile(mpm_ctx* ctx, uint32_t phase_mask);

/* Synchronize and return the accumulated per-phase launch counts and
 * event-measured device times since the last mpm_profile call.           */
int mpm_profile_read(mpm_ctx* ctx, mpm_profile_data* out);

/* Message for the last failed call on ctx (or of mpm_create when ctx is
 * NULL).  Owned by the library; valid until the next call on that context. */
const char* mpm_last_error(const mpm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H */
