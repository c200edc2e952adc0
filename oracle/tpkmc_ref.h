/*
 * tpkmc_ref.h -- plain FP64 CPU oracle for the test-particle kinetic Monte
 * Carlo collision step of Sagert et al., "Hydrodynamic Shock Wave Studies
 * within a Kinetic Monte Carlo Approach" (arXiv:1210.8084).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library;
 * nothing in the product path may link, load or call it.  It shares no code,
 * header, table or helper with the GPU sources.  It is deliberately slow and
 * written to be read against the paper: every arithmetic expression is
 * evaluated in IEEE double, left to right, each product rounded (the build
 * uses -ffp-contract=off), with correctly rounded division and sqrt.
 *
 * All pointers are host pointers.  Nothing is allocated that outlives a call.
 * Functions return 0 on success and a negative value on bad arguments.
 */
#ifndef TPKMC_REF_H
#define TPKMC_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_BC_REFLECT = 0, REF_BC_PERIODIC = 1, REF_BC_ABSORB = 2 };

/* Partner-search modes of ref_step / ref_best:
 *  REF_MODE_BINNED : the particle's c-bin and its neighbour c-bins (Sec. 3),
 *                    enumerated cell by cell;
 *  REF_MODE_BRUTE  : every other particle, kept only when the adjacency
 *                    predicate between the two c-bins holds (the O(N^2)
 *                    search of Sec. 3 restricted to the same neighbourhood);
 *  REF_MODE_ALL    : every other particle, no neighbourhood restriction. */
enum { REF_MODE_BINNED = 0, REF_MODE_BRUTE = 1, REF_MODE_ALL = 2 };

typedef struct {
    double  lo[3], hi[3];   /* box [lo, hi) per axis                          */
    int32_t ncell[3];       /* c-bins per axis (>= 1)                         */
    int32_t bc[3];          /* REF_BC_* per axis                              */
    int32_t nobin[3];       /* o-bins per axis (>= 1)                         */
    int32_t pad;
} ref_grid;

typedef struct {
    double   sigma;         /* cross section; D^2 = sigma / pi (Sec. 2.4)      */
    double   mass;          /* particle mass (single species)                 */
    double   dt;            /* time step                                      */
    uint64_t seed;          /* Philox key                                     */
    uint64_t step;          /* step number (low 32 bits enter the counter)    */
    uint32_t instance;      /* instance number (< 2^24)                       */
    uint32_t flags;         /* REF_ADAPTIVE_DT | REF_PLANAR | REF_RANK_TIME | REF_PAIR_RANDOM */
} ref_params;

/* ref_params.flags.  REF_ADAPTIVE_DT: the step length follows the rule of
 * Sec. 3, dt = dx / v_max, with v_max the largest speed of the alive,
 * finite particles at the start of the step and dx the smallest c-bin width
 * over the axes that have more than one c-bin; params.dt is then an upper
 * bound (it is also taken when v_max = 0 or no axis has two c-bins).  Full
 * steps (ref_step, ref_step_sample) and the searches (ref_best,
 * ref_best_sample) apply it; ref_pair_test uses params.dt as given. */
enum { REF_ADAPTIVE_DT = 1 };

/* ref_params.flags.  REF_PLANAR: a two-dimensional gas (Sec. 4: every test
 * is also run in 2D, with f = 2 velocity degrees of freedom).  Particles
 * move in the x-y plane: the grid must have one c-bin along z, and the
 * caller gives every particle the same z and vz = 0, which the step then
 * keeps.  The cross section is a length, sigma = 2 D (the width of the strip
 * a disk of diameter D sweeps relative to another), so D^2 = sigma^2 / 4 in
 * place of sigma / pi, and the scattering direction is isotropic in the
 * plane. */
enum { REF_PLANAR = 2 };

/* ref_params.flags.  REF_RANK_TIME: criterion 3 takes, among the candidates,
 * the one with the earliest contact of the effective radii (the earlier
 * overlap time t_o1 of Sec. 2.4) instead of the smallest d_min; the paper
 * names both choices and uses the distance.  Ties go to the lower id, and
 * best_d2 outputs stay the d_min^2 of the chosen partner. */
enum { REF_RANK_TIME = 4 };

/* ref_params.flags.  REF_PAIR_RANDOM: random partners inside each c-bin,
 * the usual DSMC rule that Sec. 2.3 sets against the point of closest
 * approach, in place of criteria 1-3 (the criteria select no pair in this
 * mode):
 *  - every usable particle of a c-bin gets the key w0 of Philox4x32-10 with
 *    counter (step, id, id, instance * 2^8 + 255) and the seed as key; the
 *    c-bin's particles are ordered by (key, id), and positions (0, 1),
 *    (2, 3), ... form pairs (an odd last particle has none);
 *  - a pair {A, B} (A the lower id) of a c-bin holding n_c particles
 *    collides when u < (((n_c - 1) sigma) g) dt / V_c, with g = |v_A - v_B|,
 *    V_c the c-bin volume (w_x w_y w_z; w_x w_y in the plane, where sigma is
 *    a length) and u the 53-bit uniform of the words w0, w1 of Philox with
 *    counter (step, id_A, id_B, instance * 2^8 + 255).  Each particle of the
 *    c-bin then collides with probability n sigma g dt on average, the
 *    kinetic-theory rate;
 *  - a colliding pair scatters as in Sec. 3 and then moves with the new
 *    velocity for the whole step (no point of closest approach); its virial
 *    term takes the separation at the start of the step.
 * Counters: TESTS = pairs formed, CAND = HAVE_BEST = particles in a formed
 * pair, PAIRS = colliding pairs.  Not combinable with REF_RANK_TIME; the
 * searches (ref_best, ref_best_sample) and ref_step_sample reject it.  In
 * every mode the scattering direction draws at most 255 times, so that the
 * counter ending in 255 belongs to the key and acceptance draws alone. */
enum { REF_PAIR_RANDOM = 8 };

/* Phases of ref_step whose wall times ref_last_phase_ms reports, in ms, for
 * the last ref_step of the process (instrumentation for the benchmark's CPU
 * baseline; the random-partner mode books its pairing under SEARCH). */
enum { REF_PHASE_BIN = 0, REF_PHASE_SEARCH, REF_PHASE_PAIR, REF_PHASE_SCATTER, REF_PHASE_MOVE,
       REF_PHASE_MOMENTS, REF_NPHASES };
void ref_last_phase_ms(double out[REF_NPHASES]);

/* Counters written by ref_step (uint64[8]). */
enum {
    REF_CNT_ALIVE = 0,      /* alive particles after the step                 */
    REF_CNT_PAIRS = 1,      /* accepted (unambiguous) pairs                   */
    REF_CNT_TESTS = 2,      /* algorithmic unordered neighbourhood pairs      */
    REF_CNT_CAND = 3,       /* ordered (i, j) that passed all three criteria  */
    REF_CNT_FAST = 4,       /* particles with |v_a| dt > w_a on some axis     */
    REF_CNT_NONFINITE = 5,  /* alive particles with a non-finite coordinate   */
    REF_CNT_ABSORBED = 6,   /* particles absorbed this step                   */
    REF_CNT_HAVE_BEST = 7   /* particles with at least one candidate          */
};

/* Globals written by ref_step (double[8]). */
enum {
    REF_G_PX = 0, REF_G_PY = 1, REF_G_PZ = 2, /* sum m v_a                     */
    REF_G_EKIN = 3,                           /* sum m |v|^2 / 2               */
    REF_G_VMAX2 = 4,                          /* max |v|^2                     */
    REF_G_VIRIAL = 5,                         /* sum of virial trace terms     */
    REF_G_MASS = 6,                           /* sum m                         */
    REF_G_DT = 7                              /* time step the step used       */
};

/* Per-o-bin moments written by ref_step (double[nobin * 11]). */
enum {
    REF_M_COUNT = 0,
    REF_M_PX = 1,           /* 1..3: sum m v_a                                */
    REF_M_CXX = 4,          /* 4..6: sum m (v_a - vbar_a)^2, vbar = bin mean  */
    REF_M_VIRX = 7,         /* 7..9: sum (1/2) r_a dp_a / dt over colliders   */
    REF_M_NCOLL = 10,
    REF_M_MASS = 11,        /* sum m                                          */
    REF_M_STRIDE = 12
};

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Isotropic unit vector for the pair (idA < idB) at (seed, step, instance);
 * returns the number of Philox draws used (1..256). */
int ref_direction(uint64_t seed, uint64_t step, uint32_t instance,
                  uint32_t idA, uint32_t idB, double n[3]);

/* In-plane isotropic unit vector (n[2] = 0) for the pair, from the same
 * Philox draws: an accepted point (x1, x2) of the unit disk, 0 < s < 1,
 * gives the doubled angle n = ((x1^2 - x2^2) / s, 2 x1 x2 / s).  Returns the
 * number of draws used. */
int ref_direction_planar(uint64_t seed, uint64_t step, uint32_t instance,
                         uint32_t idA, uint32_t idB, double n[3]);

/* c-bin of a point (bin indices per axis and flattened index). */
int32_t ref_cell_of(const ref_grid* g, double x, double y, double z, int32_t c[3]);

/* Distinct neighbour c-bins of cell c (itself included); returns the count. */
int ref_stencil(const ref_grid* g, int32_t c, int32_t out[27]);

/* The three-criterion test for the ordered pair (i, j) with states
 * (ri, vi), (rj, vj).  Returns 1 and fills d2, tp when j is a candidate. */
int ref_pair_test(const ref_grid* g, const ref_params* p,
                  const double ri[3], const double vi[3],
                  const double rj[3], const double vj[3],
                  double* d2, double* tp);

/* Closest-candidate index per particle (-1 if none) and its d^2. */
int ref_best(const ref_grid* g, const ref_params* p, int64_t n,
             const double* x, const double* y, const double* z,
             const double* vx, const double* vy, const double* vz,
             const uint32_t* id, const uint8_t* alive, int mode, int nthreads,
             int64_t* best, double* best_d2);

/* Same as ref_best but only for the particles listed in sample[0..ns). */
int ref_best_sample(const ref_grid* g, const ref_params* p, int64_t n,
                    const double* x, const double* y, const double* z,
                    const double* vx, const double* vy, const double* vz,
                    const uint32_t* id, const uint8_t* alive,
                    int64_t ns, const int64_t* sample, int nthreads,
                    int64_t* best, double* best_d2);

/* Algorithmic unordered neighbourhood pair count:
 * sum_c [ n_c (n_c - 1) / 2 + sum_{c' in N(c), c' > c} n_c n_c' ]. */
uint64_t ref_count_tests(const ref_grid* g, int64_t n,
                         const double* x, const double* y, const double* z,
                         const double* vx, const double* vy, const double* vz,
                         const uint8_t* alive);

/* Post-step state of the listed particles only, as ref_step (binned mode)
 * would leave it: out_state[6k..6k+5] = x y z vx vy vz, out_partner[k] =
 * index of the accepted partner or -1, out_alive[k] = alive after the step.
 * Cost: two neighbourhood searches per listed particle. */
int ref_step_sample(const ref_grid* g, const ref_params* p, int64_t n,
                    const double* x, const double* y, const double* z,
                    const double* vx, const double* vy, const double* vz,
                    const uint32_t* id, const uint8_t* alive, const double* mass,
                    int64_t ns, const int64_t* sample, int nthreads,
                    double* out_state, int64_t* out_partner, uint8_t* out_alive);

/* Time step a step of this state would use: params.dt, or the adaptive
 * rule above when params.flags has REF_ADAPTIVE_DT.  Negative on bad
 * arguments. */
double ref_step_dt(const ref_grid* g, const ref_params* p, int64_t n,
                   const double* x, const double* y, const double* z,
                   const double* vx, const double* vy, const double* vz,
                   const uint8_t* alive);

/* Particle masses: mass may be NULL (every particle has params.mass) or
 * hold one finite positive mass per particle (a mixture).  Scattering then
 * keeps the mass-weighted centre-of-mass velocity and the relative speed
 * (Sec. 3 for the equal-mass case, plain elastic kinematics otherwise), and
 * moments and global sums weight each particle by its own mass.  A particle
 * whose mass is not finite and positive counts as non-finite.
 *
 * One full collision step, in place, in caller order.
 * pairs (may be NULL): (idA, idB) with idA < idB, at most pair_cap entries.
 * moments (may be NULL): double[nobin * 11].  globals: double[8] or NULL.
 * counters: uint64[8] or NULL.  alive may be NULL (all alive), except when
 * an axis is ABSORB (then the call is rejected). */
int ref_step(const ref_grid* g, const ref_params* p, int64_t n,
             double* x, double* y, double* z,
             double* vx, double* vy, double* vz,
             const uint32_t* id, uint8_t* alive, const double* mass, int mode, int nthreads,
             uint32_t* pairs, int64_t pair_cap,
             uint64_t* counters, double* moments, double* globals);

#ifdef __cplusplus
}
#endif
#endif
