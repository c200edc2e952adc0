/*
 * tpkmc.h -- C ABI of the MI355X (gfx950) collision step of the
 * test-particle kinetic Monte Carlo method of Sagert et al., "Hydrodynamic
 * Shock Wave Studies within a Kinetic Monte Carlo Approach" (arXiv:1210.8084).
 *
 * One call of tpkmc_step advances N test particles by one time step dt, as
 * laid out in Sec. 3 of the paper (flow chart, Fig. 2):
 *   1. sort the particles into c-bins of a uniform grid;
 *   2. for every particle, search its own c-bin and the neighbouring ones
 *      (8 in 2D, 26 in 3D; Sec. 3, Fig. 1) for partners that satisfy the
 *      three criteria: negative crossing number chi within dt (Sec. 2.4,
 *      crossing-number equation), real overlap times of the effective radii,
 *      i.e. closest-approach distance d_min <= D with D^2 = sigma/pi
 *      (Sec. 2.4, effective-radius relation and overlap-time quadratic), and
 *      smallest d_min among the candidates (ties to the lower id);
 *   3. keep only unambiguous partners: i and j are paired when each is the
 *      other's closest candidate (end of Sec. 3);
 *   4. scatter each pair elastically and isotropically in its centre-of-mass
 *      frame, with outgoing velocities random and opposite (Sec. 3);
 *   5. move colliders to their point of closest approach with the old
 *      velocity and on with the new one, stream the rest freely (Sec. 3,
 *      t_poca and position-update equations); apply the walls;
 *   6. accumulate o-bin moments: count, momentum, velocity spread and the
 *      collisional (virial) part of the stress tensor (Sec. 4, stress-tensor
 *      equation), plus global momentum, kinetic energy and max |v|^2.
 *
 * Random numbers: Philox4x32-10 keyed by the 64-bit seed, with counter
 * (step, id_A, id_B, instance << 8 | draw), id_A < id_B, so every draw is a
 * pure function of (seed, step, instance, pair); Marsaglia's method turns
 * two uniforms into the isotropic direction.
 *
 * Conventions:
 *   - Every function returns TPKMC_OK (0) or a negative TPKMC_E* code.
 *     Argument errors are detected on the host before anything is launched.
 *     Conditions met on the device (pair-list overflow, non-finite input,
 *     a particle faster than one c-bin per step) set bits of a sticky status
 *     word read with tpkmc_status.  No C++ exception or abort crosses the ABI.
 *   - All particle and output pointers are DEVICE pointers owned by the
 *     caller (for example torch tensors); the handle owns only its scratch,
 *     allocated once in tpkmc_create.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*, NULL = default stream) and the calls return without waiting.
 *     One handle serves one stream at a time.
 *   - The time step is the caller's dt, or with TPKMC_ADAPTIVE_DT the
 *     rule of Sec. 3 (dt = c-bin width / v_max), evaluated on the device.
 *   - Precision is fixed per handle: TPKMC_FP64 takes double particle
 *     arrays and reproduces the CPU oracle's pair decisions bit for bit;
 *     TPKMC_FP32 takes float arrays; its runs are not bit-reproducible
 *     (exact FP32 ties of the closest distance go to the lower record, and
 *     the record order inside a c-bin follows atomic ordering).  Moments and
 *     global sums are FP64 in both modes.
 */
#ifndef TPKMC_H
#define TPKMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPKMC_ABI_VERSION 2

enum {
    TPKMC_OK = 0,
    TPKMC_EINVAL = -1,       /* bad argument, checked before any launch      */
    TPKMC_ENOMEM = -2,       /* device allocation failed (tpkmc_create)      */
    TPKMC_EHIP = -3,         /* a HIP runtime call failed                    */
    TPKMC_ECAPACITY = -4,    /* input exceeds the capacities of the handle   */
    TPKMC_EUNSUPPORTED = -5  /* valid but not supported by the library       */
};

enum { TPKMC_FP64 = 0, TPKMC_FP32 = 1 };

/* Boundary per axis.  REFLECT mirrors position and velocity component at
 * the wall; PERIODIC wraps (pair tests use the minimum image); ABSORB marks
 * the particle dead (alive = 0) once it leaves [lo, hi).  Pair tests ignore
 * walls (straight lines). */
enum { TPKMC_BC_REFLECT = 0, TPKMC_BC_PERIODIC = 1, TPKMC_BC_ABSORB = 2 };

/* tpkmc_params.flags */
enum {
    TPKMC_EMIT_PAIRS = 1u,     /* write accepted pairs to outputs.pairs       */
    TPKMC_ALLOW_REORDER = 2u,  /* leave all particle arrays (id and alive
                                  included) in c-bin order instead of the
                                  caller's order                            */
    TPKMC_ADAPTIVE_DT = 4u,    /* time step of Sec. 3: dt = dx / v_max, with
                                  v_max the largest speed of the alive finite
                                  particles at the start of the step and dx
                                  the smallest c-bin width over the axes with
                                  more than one c-bin; params.dt is the upper
                                  bound (also taken when v_max = 0).  Computed
                                  on the device, so graph replays adapt too;
                                  the dt used is globals slot 7.            */
    TPKMC_PLANAR = 8u,         /* two-dimensional gas in the x-y plane (the 2D
                                  runs of Sec. 4, f = 2): the grid has one
                                  c-bin along z and the caller gives every
                                  particle the same z and vz = 0, which the
                                  step keeps; sigma is then a length, the
                                  width 2 D of the strip one disk sweeps
                                  relative to another (D^2 = sigma^2 / 4),
                                  and directions are isotropic in the plane */
    TPKMC_RANK_TIME = 16u,     /* criterion 3 by time: among the candidates,
                                  the one whose effective radii touch first
                                  (the earlier overlap time t_o1 of Sec. 2.4)
                                  instead of the smallest d_min; the paper
                                  names both choices and uses the distance */
    TPKMC_PAIR_RANDOM = 32u    /* random partners inside each c-bin, the usual
                                  DSMC rule that Sec. 2.3 sets against the
                                  point of closest approach, in place of
                                  criteria 1-3.  The c-bin's particles are
                                  ordered by (key, id), key = word 0 of
                                  Philox4x32-10 (counter (step, id, id,
                                  instance * 2^8 + 255), key = seed), and
                                  positions (0, 1), (2, 3), ... pair up.  A
                                  pair {A, B} (A the lower id) of a c-bin of
                                  n_c particles collides when
                                  u < (((n_c - 1) sigma) g) dt / V_c, in
                                  double: g = |v_A - v_B|, V_c the c-bin
                                  volume (area in the plane), u the 53-bit
                                  uniform of words 0 and 1 of Philox with
                                  counter (step, id_A, id_B,
                                  instance * 2^8 + 255).  Colliders scatter
                                  at the start of the step (no point of
                                  closest approach; the virial takes the
                                  separation then) and move with the new
                                  velocity.  Counters: tests = pairs formed,
                                  cand = have_best = particles in a formed
                                  pair, pairs = colliding pairs.  Not with
                                  TPKMC_RANK_TIME.  In every mode the
                                  scattering direction draws at most 255
                                  times, so the counters ending in 255 are
                                  these draws' alone. */
};

/* Bits of the device status word (sticky until read). */
enum {
    TPKMC_STATUS_PAIR_OVERFLOW = 1, /* more pairs than outputs.pair_cap       */
    TPKMC_STATUS_NONFINITE = 2,     /* an alive particle had a NaN/Inf value  */
    TPKMC_STATUS_FAST = 4           /* |v_a| dt > c-bin width on some axis    */
};

/* Counters (uint64[8] per instance). */
enum {
    TPKMC_CNT_ALIVE = 0,      /* alive particles with finite state, after    */
    TPKMC_CNT_PAIRS = 1,      /* accepted pairs                              */
    TPKMC_CNT_TESTS = 2,      /* algorithmic unordered neighbourhood pairs:
                                 sum_c n_c(n_c-1)/2 + sum_{c'>c adjacent}
                                 n_c n_c'                                   */
    TPKMC_CNT_CAND = 3,       /* ordered (i, j) passing all three criteria   */
    TPKMC_CNT_FAST = 4,       /* particles with |v_a| dt > w_a (before)      */
    TPKMC_CNT_NONFINITE = 5,  /* alive particles with a NaN/Inf value        */
    TPKMC_CNT_ABSORBED = 6,   /* particles absorbed in this step             */
    TPKMC_CNT_HAVE_BEST = 7   /* particles with at least one candidate       */
};

/* Globals (double[8] per instance), over alive finite particles after the
 * step: 0..2 sum m v_a, 3 sum m|v|^2/2, 4 max |v|^2, 5 sum of virial trace
 * terms, 6 sum m, 7 the time step this step used. */
enum { TPKMC_G_PX = 0, TPKMC_G_EKIN = 3, TPKMC_G_VMAX2 = 4, TPKMC_G_VIRIAL = 5, TPKMC_G_MASS = 6,
       TPKMC_G_DT = 7 };

/* Per-o-bin moments (double[nobin * 12] per instance, o-bin index
 * bx + nobin[0] * (by + nobin[1] * bz) of the post-step position):
 *  0 count; 1..3 sum m v_a; 4..6 sum m (v_a - vbar_a)^2 with vbar the bin's
 *  mass-weighted mean velocity; 7..9 sum over colliders of (1/2) s_a dp_a /
 *  dt with s the separation from the partner at closest approach and dp the
 *  momentum change; 10 number of colliders; 11 sum m (count x mass for a
 *  scalar mass, rounded once).  Pressure of a bin of
 *  volume V: p = (sum_a [4+a] + sum_a [7+a]) / (3 V); temperature
 *  T = sum_a [4+a] / (3 count).
 *  The sums are exact and independent of the order of the particles: each
 *  term is rounded once to an integer multiple of 2^-50 times the power of
 *  two just above the largest term of its kind in that o-bin and step, the
 *  integers are added exactly, and the total is rounded to double; equal
 *  inputs give bit-identical moments whatever the launch shape, batch or
 *  particle order.  Velocities enter relative to a per-o-bin shift (the
 *  bin's previous mean), so the spread is not the difference of large
 *  sums. */
#define TPKMC_MOMENT_STRIDE 12

typedef struct tpkmc_handle tpkmc_handle;

typedef struct {
    int64_t max_particles;  /* capacity: particles (sum over instances)      */
    int64_t max_cells;      /* capacity: sum over instances of (c-bins + 1)  */
    int64_t max_obins;      /* capacity: sum over instances of o-bins        */
    int32_t max_instances;  /* capacity: instances per call (>= 1)           */
    int32_t precision;      /* TPKMC_FP64 or TPKMC_FP32                      */
    int32_t device;         /* HIP device ordinal                            */
    uint32_t flags;         /* reserved, must be 0                           */
} tpkmc_config;

/* Box [lo, hi) per axis with ncell c-bins (partner search) and nobin
 * o-bins (moments) per axis.  Cell index cx + ncell[0]*(cy + ncell[1]*cz),
 * cx = floor((x - lo) ncell / (hi - lo)) clamped into [0, ncell-1]. */
typedef struct {
    double lo[3], hi[3];
    int32_t ncell[3];
    int32_t bc[3];          /* TPKMC_BC_* per axis                           */
    int32_t nobin[3];
    int32_t pad;
} tpkmc_grid;

typedef struct {
    double sigma;           /* cross section; D^2 = sigma / pi (sigma^2 / 4
                               with TPKMC_PLANAR)                            */
    double mass;            /* particle mass (> 0)                           */
    double dt;              /* time step (> 0); its upper bound with
                               TPKMC_ADAPTIVE_DT                             */
    uint64_t seed;          /* Philox key                                    */
    uint64_t step;          /* step number (low 32 bits enter the counter)   */
    uint32_t instance;      /* instance number (< 2^24)                      */
    uint32_t flags;         /* TPKMC_EMIT_PAIRS | TPKMC_ALLOW_REORDER |
                               TPKMC_ADAPTIVE_DT | TPKMC_PLANAR |
                               TPKMC_RANK_TIME | TPKMC_PAIR_RANDOM (not
                               with TPKMC_RANK_TIME)                         */
} tpkmc_params;

/* Structure-of-arrays particle state, device pointers, n entries each.
 * x..vz are double* (FP64 handle) or float* (FP32 handle).  id: unique
 * uint32 per particle (read; permuted only with ALLOW_REORDER).  alive:
 * uint8 0/1, or NULL for all alive (then no axis may be ABSORB).  mass:
 * NULL (every particle has params.mass) or one mass per particle, of the
 * handle's real type, for a mixture.  Scattering then keeps the
 * mass-weighted centre-of-mass velocity and the relative speed, and moments
 * and global sums weight each particle by its mass.  A mass that is not
 * finite and positive makes the particle non-finite.  The masses are
 * permuted with ALLOW_REORDER. */
typedef struct {
    int64_t n;
    void *x, *y, *z, *vx, *vy, *vz;
    uint32_t* id;
    uint8_t* alive;
    void* mass;
} tpkmc_particles;

/* Output device pointers; any may be NULL (that output is skipped).
 * pairs: uint32[2 * pair_cap], rows (id_A, id_B) with id_A < id_B in
 * unspecified order; pairs beyond pair_cap are counted, not written, and
 * set TPKMC_STATUS_PAIR_OVERFLOW.  counters: uint64[8 * n_inst];
 * globals: double[8 * n_inst]; moments: double[TPKMC_MOMENT_STRIDE * sum of
 * o-bins], the instances' o-bin blocks concatenated in instance order. */
typedef struct {
    uint32_t* pairs;
    int64_t pair_cap;
    uint64_t* counters;
    double* moments;
    double* globals;
} tpkmc_outputs;

/* One independent instance of a batch: particles [offset, offset + count)
 * of the concatenated arrays, with its own grid and parameters.  Slices of
 * different instances must not overlap. */
typedef struct {
    int64_t offset, count;
    tpkmc_grid grid;
    tpkmc_params params;
} tpkmc_instance;

/* ABI version (TPKMC_ABI_VERSION). */
int tpkmc_version(void);

/* Static description of a return code. */
const char* tpkmc_strerror(int code);

/* Allocates a handle and all its device scratch on cfg->device (memory is
 * sized from the capacities: about 73 B per particle in FP32, 113 B in FP64,
 * 8 B per c-bin, 152 B per o-bin).  *out is NULL on failure. */
int tpkmc_create(const tpkmc_config* cfg, tpkmc_handle** out);

/* Waits for the handle's work, frees everything.  NULL is a no-op. */
int tpkmc_destroy(tpkmc_handle* h);

/* One collision step of one instance (steps 1-6 above), in place. */
int tpkmc_step(tpkmc_handle* h, const tpkmc_grid* g, const tpkmc_params* p,
               const tpkmc_particles* s, const tpkmc_outputs* o, void* hip_stream);

/* Size in bytes of the static device scratch of tpkmc_step_noalloc: one
 * array per GPU the library runs on, held until the process ends. */
#define TPKMC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of tpkmc_step for one instance without a handle.  It calls no hipMalloc,
 * hipFree, host-pinned allocation or other allocating routine; its scratch
 * lives in a static device array of TPKMC_NOALLOC_SCRATCH_BYTES per GPU.
 *   precision: TPKMC_FP64 (double particle arrays) or TPKMC_FP32 (float);
 *   device:    HIP device ordinal (made current on the calling thread); the
 *              stream must belong to it;
 *   g, p, s, o, hip_stream: as for tpkmc_step; the search runs in the
 *              default launch shape (2 records per lane, 64 lanes), so the
 *              results equal those of tpkmc_step on a new handle.
 * Returns TPKMC_ECAPACITY, before anything is launched, when the step's
 * scratch exceeds the array: about 105 B per particle in FP64 (113 with
 * per-particle masses), 69 B in FP32 (73), plus 4 B per c-bin and 152 B per
 * o-bin, so at most about 0.6M particles in FP64 and 0.9M in FP32.
 * Every call on a GPU uses that GPU's one array, and the array keeps the
 * last call's contents (the call clears what must start at zero), so calls
 * that overlap in time on one GPU race: order them on one stream.  There
 * is no status word: the device conditions show in the counters
 * (TPKMC_CNT_NONFINITE, TPKMC_CNT_FAST, and TPKMC_CNT_PAIRS > pair_cap for
 * an overflowing pair list). */
int tpkmc_step_noalloc(int32_t precision, int32_t device, const tpkmc_grid* g, const tpkmc_params* p,
                       const tpkmc_particles* s, const tpkmc_outputs* o, void* hip_stream);

/* One step of n_inst independent instances in a single set of launches;
 * s describes the concatenated arrays.  Outputs are per instance as above;
 * EMIT_PAIRS of any instance writes into the one shared pair list. */
int tpkmc_step_batched(tpkmc_handle* h, const tpkmc_particles* s,
                       const tpkmc_instance* inst, int32_t n_inst,
                       const tpkmc_outputs* o, void* hip_stream);

/* nsteps steps of a batch: the step is captured once as a HIP graph and
 * replayed nsteps times; each instance's step number advances on the device
 * from inst[k].params.step.  Outputs hold the last step's values.  On the
 * handle's first run without a launch shape chosen by tpkmc_autotune or
 * tpkmc_set_search, it first tunes the search on this batch (as
 * tpkmc_autotune, which synchronises the stream; every shape gives the same
 * results). */
int tpkmc_run(tpkmc_handle* h, const tpkmc_particles* s,
              const tpkmc_instance* inst, int32_t n_inst, int32_t nsteps,
              const tpkmc_outputs* o, void* hip_stream);

/* Chooses the results-neutral knobs of the partner search on this batch
 * and keeps them for later steps of this handle:
 *  - c-bins split by speed (S10 of the search's design).  Two particles of
 *    speed at most v_c that meet the criteria of Sec. 2.4 within a step start
 *    at most D + 2 v_c dt apart, so on c-bins at least that wide the stencil
 *    holds every such pair.  Per instance, with v_c = 2 times the
 *    root-mean-square speed v_rms of its live particles on this state (6
 *    v_rms when the particles above 2 v_rms hold more than half of the
 *    kinetic energy, as in a point blast), the slow
 *    particles (|v| <= v_c, decided every step) are binned on c-bins refined
 *    per axis to the largest count that keeps a factor 1 + 1/64 over that
 *    reach, when that is at least 1.25 times the configured count (3 or more
 *    on periodic axes; never with TPKMC_PAIR_RANDOM, whose draw depends on
 *    the c-bin), with at most one c-bin per two particles; the fast ones keep
 *    the configured c-bins and are tested against every particle of their
 *    configured neighbourhood.  The split applies to the instance at the
 *    same batch position while its grid, sigma, dt and flags stay those it
 *    was tuned with; at any later speeds, pairs, states and all outputs
 *    other than the search's work counters (TPKMC_CNT_TESTS,
 *    TPKMC_CNT_CAND) equal those of the configured c-bins.  The time step
 *    and the fast-particle check keep the configured c-bins.  May grow the
 *    handle's c-bin storage.
 *  - the launch shape (work-group size and particles per work-item): timed,
 *    the default kept unless another is at least 5% faster;
 *  - the order in which the search's work-groups are dealt to the XCDs:
 *    chunks of 16 work-groups dealt round-robin over the XCDs (the default:
 *    balance when the work per work-group varies along the c-bin order, as
 *    across a batch of instances or in a dense shocked region), contiguous
 *    ranges per XCD (neighbouring work-groups share an L2), or chunks of 1
 *    or 128; another order is timed in the chosen shape and kept when at
 *    least 5% faster.
 * Runs the binning and search kernels only; the particle state is not
 * modified.  Synchronises the stream. */
int tpkmc_autotune(tpkmc_handle* h, const tpkmc_particles* s,
                   const tpkmc_instance* inst, int32_t n_inst, void* hip_stream);

/* The search's work-group order in use: 0 for contiguous ranges per XCD,
 * S > 0 for chunks of S work-groups dealt round-robin. */
int tpkmc_search_order(tpkmc_handle* h, int32_t* order);

/* Sets that order (0, or a chunk of 1..4096 work-groups); results do not
 * depend on it.  tpkmc_set_search resets it to the default, 16. */
int tpkmc_set_search_order(tpkmc_handle* h, int32_t order);

/* The slow particles' c-bins per axis that tpkmc_autotune chose for batch
 * position k of the batch it last tuned (the configured counts where it kept
 * them).  EINVAL if k is not a tuned position. */
int tpkmc_tuned_cells(tpkmc_handle* h, int32_t k, int32_t ncell[3]);

/* The speed bound v_c of the slow particles at batch position k (0 where
 * the c-bins are not split).  EINVAL if k is not a tuned position. */
int tpkmc_tuned_speed(tpkmc_handle* h, int32_t k, double* speed);

/* Diagnostic: the arithmetic mix of the partner search on a state, for the
 * roofline of the search.  counts (host, uint64[3]) receives, summed over
 * the instances, the algorithmic unordered pair tests (TPKMC_CNT_TESTS),
 * those with s0 = r.u < 0 (approaching) and those with s0 < 0 < s1 =
 * s0 + |u|^2 dt (criterion 1 of Sec. 2.4).  A pair test costs 11 FLOP to
 * decide s0 (r, u, r.u), 7 more for |u|^2 and s1 when s0 < 0, and 12 more
 * for t_poca, the separation there and d_min^2 when both hold.  Bins the
 * state and runs a counting build of the search (never the one tpkmc_step
 * runs); the state and all outputs are left as they were.  Synchronises the
 * stream. */
int tpkmc_search_mix(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* inst, int32_t n_inst,
                     uint64_t* counts, void* hip_stream);

/* Launch shape of the partner search: one lane per `group` consecutive
 * c-bin-ordered records (1, 2 or 4) and `block` lanes per work-group (64,
 * 128 or 256, at most 256 / group).  Every shape gives the same pairs, state
 * and counters.  The default is group 2, block 64; tpkmc_autotune keeps it
 * unless another shape is at least 3% faster; tpkmc_set_search fixes one
 * (EINVAL outside these lists). */
int tpkmc_set_search(tpkmc_handle* h, int32_t group, int32_t block);
int tpkmc_get_search(tpkmc_handle* h, int32_t* group, int32_t* block);

/* Synchronises the handle's last stream, returns the status word in
 * *device_status and clears it. */
int tpkmc_status(tpkmc_handle* h, int32_t* device_status);

/* Phase timing: when enabled, every step records HIP events around each
 * kernel on the step's stream.  tpkmc_profile_read synchronises, writes
 * the summed milliseconds and launch counts of up to n phases
 * (0 clear, 1 key, 2 scan, 3 scatter, 4 search, 5 move, 6 finalize) and
 * resets the sums. */
int tpkmc_profile_enable(tpkmc_handle* h, int32_t on);
int tpkmc_profile_read(tpkmc_handle* h, double* ms, int64_t* launches, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
