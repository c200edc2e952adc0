/*
 * tpkmc_ref.c -- plain FP64 CPU oracle of the collision step of the
 * test-particle kinetic Monte Carlo method (Sagert et al., arXiv:1210.8084).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU baseline of the benchmark; never by the GPU library.  It shares no
 * code with the GPU sources.  Build with -ffp-contract=off (no FMA), so that
 * every product below is rounded on its own.
 *
 * One step, in the order of Sec. 3 (flow chart, Fig. 2):
 *   1. sort particles into c-bins                      (Sec. 3)
 *   2. partner search over the bin and its neighbours  (Sec. 3, Fig. 1)
 *      with the three criteria: negative crossing number chi (Sec. 2.4,
 *      crossing-number equation), real overlap times t_o (Sec. 2.4, the
 *      overlap-time quadratic), smallest distance between final partners
 *   3. keep only unambiguous partners                  (end of Sec. 3)
 *   4. isotropic elastic scattering in the centre-of-mass frame (Sec. 3)
 *   5. position update split at t_poca, free streaming otherwise (Sec. 3)
 *   6. walls, then o-bin moments (Sec. 4, bulk velocity, stress tensor,
 *      pressure and temperature equations)
 */
#include "tpkmc_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the description in Salmon, Moraes, Dror and Shaw,     */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two  */
/* 32x32->64 multiplications; the high halves are XORed with the other two   */
/* words and the round key, the words are permuted, and the key is bumped by */
/* the Weyl constants (golden ratio and sqrt(3)-1 in 32-bit fixed point).    */
/* ------------------------------------------------------------------------ */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform double in [0, 1) from two 32-bit words: 27 + 26 = 53 bits. */
static double unit_double(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* The outgoing directions are random and opposite (Sec. 3); the random unit
 * vector is drawn with Marsaglia's 1972 rejection method, which needs only a
 * square root.  The counter names the pair and the draw. */
int ref_direction(uint64_t seed, uint64_t step, uint32_t instance,
                  uint32_t idA, uint32_t idB, double n[3])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (uint32_t attempt = 0; attempt < 255u; ++attempt) {
        uint32_t ctr[4] = { (uint32_t)step, idA, idB, (instance << 8) | attempt };
        uint32_t w[4];
        ref_philox4x32_10(ctr, key, w);
        double u1 = unit_double(w[0], w[1]);
        double u2 = unit_double(w[2], w[3]);
        double x1 = 2.0 * u1 - 1.0;
        double x2 = 2.0 * u2 - 1.0;
        double s = x1 * x1 + x2 * x2;
        if (s < 1.0) {
            double q = sqrt(1.0 - s);
            n[0] = (2.0 * x1) * q;
            n[1] = (2.0 * x2) * q;
            n[2] = 1.0 - 2.0 * s;
            return (int)attempt + 1;
        }
    }
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    return 255;
}

int ref_direction_planar(uint64_t seed, uint64_t step, uint32_t instance,
                         uint32_t idA, uint32_t idB, double n[3])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (uint32_t attempt = 0; attempt < 255u; ++attempt) {
        uint32_t ctr[4] = { (uint32_t)step, idA, idB, (instance << 8) | attempt };
        uint32_t w[4];
        ref_philox4x32_10(ctr, key, w);
        double x1 = 2.0 * unit_double(w[0], w[1]) - 1.0;
        double x2 = 2.0 * unit_double(w[2], w[3]) - 1.0;
        double s = x1 * x1 + x2 * x2;
        if (s < 1.0 && s > 0.0) {
            /* The angle of (x1, x2) is uniform; doubling it keeps it uniform
             * and needs no square root. */
            n[0] = (x1 * x1 - x2 * x2) / s;
            n[1] = (2.0 * x1 * x2) / s;
            n[2] = 0.0;
            return (int)attempt + 1;
        }
    }
    n[0] = 1.0; n[1] = 0.0; n[2] = 0.0;
    return 255;
}

/* ------------------------------------------------------------------------ */
/* Grid                                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double L[3], w[3], inv_w[3], halfL[3], inv_wo[3];
    double D2;
    double cellvol;         /* c-bin volume (area in the plane) */
    int rank_time;          /* criterion 3 ranks by the contact time t_o1 */
    int pair_random;        /* random partners inside each c-bin */
    int32_t n[3], bc[3], no[3];
    int64_t C, B;
} derived;

static int derive(const ref_grid* g, const ref_params* p, derived* G)
{
    if (!g) return -1;
    G->C = 1; G->B = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->ncell[a] < 1 || g->nobin[a] < 1) return -1;
        if (!(g->hi[a] > g->lo[a])) return -1;
        if (g->bc[a] < 0 || g->bc[a] > 2) return -1;
        G->n[a] = g->ncell[a];
        G->no[a] = g->nobin[a];
        G->bc[a] = g->bc[a];
        G->L[a] = g->hi[a] - g->lo[a];
        G->w[a] = G->L[a] / (double)g->ncell[a];
        G->inv_w[a] = (double)g->ncell[a] / G->L[a];
        G->inv_wo[a] = (double)g->nobin[a] / G->L[a];
        G->halfL[a] = 0.5 * G->L[a];
        G->C *= g->ncell[a];
        G->B *= g->nobin[a];
    }
    G->rank_time = p && (p->flags & REF_RANK_TIME) != 0;
    G->pair_random = p && (p->flags & REF_PAIR_RANDOM) != 0;
    if (G->rank_time && G->pair_random) return -1;
    G->cellvol = (G->w[0] * G->w[1]) * G->w[2];
    if (p) {
        if (!(p->sigma >= 0.0) || !(p->dt > 0.0) || !(p->mass > 0.0)) return -1;
        if (p->instance >= (1u << 24)) return -1;
        /* sigma = 4 pi r_eff^2 and d_min <= r_eff,A + r_eff,B = 2 r_eff
         * (Sec. 2.4), so the largest accepted d_min^2 is sigma / pi.  In
         * the plane the cross section is the length 2 D. */
        if (p->flags & REF_PLANAR) {
            if (g->ncell[2] != 1) return -1;
            double D = 0.5 * p->sigma;
            G->D2 = D * D;
            G->cellvol = G->w[0] * G->w[1];
        } else {
            G->D2 = p->sigma / M_PI;
        }
    } else {
        G->D2 = 0.0;
    }
    return 0;
}

/* Bin along one axis: floor((x - lo) / w), clamped into [0, n-1]. */
static int32_t axis_bin(double x, double lo, double inv_w, int32_t n)
{
    double t = (x - lo) * inv_w;
    if (!(t >= 0.0)) return 0;
    if (t >= (double)n) return n - 1;
    return (int32_t)t;
}

int32_t ref_cell_of(const ref_grid* g, double x, double y, double z, int32_t c[3])
{
    derived G;
    if (derive(g, NULL, &G)) return -1;
    int32_t cx = axis_bin(x, g->lo[0], G.inv_w[0], G.n[0]);
    int32_t cy = axis_bin(y, g->lo[1], G.inv_w[1], G.n[1]);
    int32_t cz = axis_bin(z, g->lo[2], G.inv_w[2], G.n[2]);
    if (c) { c[0] = cx; c[1] = cy; c[2] = cz; }
    return cx + G.n[0] * (cy + G.n[1] * cz);
}

/* The bin itself and its 8 (2D) / 26 (3D) neighbours (Sec. 3): every cell
 * whose index differs by at most one on each axis, wrapping on periodic
 * axes, dropped outside the grid otherwise, listed once each. */
static int stencil(const derived* G, int64_t c, int64_t out[27])
{
    int32_t cx = (int32_t)(c % G->n[0]);
    int32_t cy = (int32_t)((c / G->n[0]) % G->n[1]);
    int32_t cz = (int32_t)(c / ((int64_t)G->n[0] * G->n[1]));
    int count = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int32_t z = cz + dz;
        if (G->bc[2] == REF_BC_PERIODIC) z = ((z % G->n[2]) + G->n[2]) % G->n[2];
        else if (z < 0 || z >= G->n[2]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int32_t y = cy + dy;
            if (G->bc[1] == REF_BC_PERIODIC) y = ((y % G->n[1]) + G->n[1]) % G->n[1];
            else if (y < 0 || y >= G->n[1]) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t x = cx + dx;
                if (G->bc[0] == REF_BC_PERIODIC) x = ((x % G->n[0]) + G->n[0]) % G->n[0];
                else if (x < 0 || x >= G->n[0]) continue;
                int64_t cell = x + (int64_t)G->n[0] * (y + (int64_t)G->n[1] * z);
                int seen = 0;
                for (int k = 0; k < count; ++k)
                    if (out[k] == cell) seen = 1;
                if (!seen) out[count++] = cell;
            }
        }
    }
    return count;
}

int ref_stencil(const ref_grid* g, int32_t c, int32_t out[27])
{
    derived G;
    if (derive(g, NULL, &G)) return -1;
    if (c < 0 || c >= G.C) return -1;
    int64_t tmp[27];
    int k = stencil(&G, c, tmp);
    for (int i = 0; i < k; ++i) out[i] = (int32_t)tmp[i];
    return k;
}

/* Adjacency of two c-bins written as a predicate (used by the brute-force
 * search, independent of the enumeration above). */
static int adjacent(const derived* G, int64_t c1, int64_t c2)
{
    int64_t a[3], b[3];
    a[0] = c1 % G->n[0]; a[1] = (c1 / G->n[0]) % G->n[1]; a[2] = c1 / ((int64_t)G->n[0] * G->n[1]);
    b[0] = c2 % G->n[0]; b[1] = (c2 / G->n[0]) % G->n[1]; b[2] = c2 / ((int64_t)G->n[0] * G->n[1]);
    for (int k = 0; k < 3; ++k) {
        int64_t d = a[k] - b[k];
        if (d < 0) d = -d;
        if (G->bc[k] == REF_BC_PERIODIC && G->n[k] - d < d) d = G->n[k] - d;
        if (d > 1) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The three criteria (Sec. 2.4 and the list in Sec. 3)                      */
/* ------------------------------------------------------------------------ */
/* Relative position with the minimum image on periodic axes. */
static void rel(const derived* G, const double ri[3], const double vi[3],
                const double rj[3], const double vj[3], double r[3], double u[3])
{
    for (int a = 0; a < 3; ++a) {
        r[a] = ri[a] - rj[a];
        if (G->bc[a] == REF_BC_PERIODIC) {
            if (r[a] > G->halfL[a]) r[a] = r[a] - G->L[a];
            else if (r[a] < -G->halfL[a]) r[a] = r[a] + G->L[a];
        }
        u[a] = vi[a] - vj[a];
    }
}

static int test_pair(const derived* G, double dt,
                     const double ri[3], const double vi[3],
                     const double rj[3], const double vj[3],
                     double* d2_out, double* tp_out, double* tc_out)
{
    double r[3], u[3];
    rel(G, ri, vi, rj, vj, r, u);
    /* Criterion 1, chi < 0: with straight-line motion v_rel is constant and
     * r_rel(t + dt) = r + u dt, so chi = s0 * s1 with s0 = r.u and
     * s1 = r.u + |u|^2 dt; chi < 0 <=> s0 < 0 < s1. */
    double s0 = (r[0] * u[0] + r[1] * u[1]) + r[2] * u[2];
    if (!(s0 < 0.0)) return 0;
    double vv = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double s1 = s0 + vv * dt;
    if (!(s1 > 0.0)) return 0;
    /* Time and separation at the point of closest approach (Sec. 3,
     * t_poca equation). */
    double tp = -s0 / vv;
    double q[3];
    for (int a = 0; a < 3; ++a) q[a] = r[a] + tp * u[a];
    double d2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
    /* Criterion 2: the overlap times are real exactly when the discriminant
     * of the quadratic is non-negative, i.e. when d_min^2 <= D^2. */
    if (!(d2 <= G->D2)) return 0;
    *d2_out = d2;
    *tp_out = tp;
    if (tc_out) {
        /* The earlier root of the overlap quadratic of Sec. 2.4 (first
         * contact of the effective radii): t_o1 = (-(u.r) - sqrt((u.r)^2 -
         * |u|^2 (|r|^2 - D^2))) / |u|^2.  The discriminant equals
         * |u|^2 (D^2 - d_min^2) >= 0; a rounding below zero is taken as 0. */
        double rr = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        double disc = s0 * s0 - vv * (rr - G->D2);
        if (!(disc > 0.0)) disc = 0.0;
        *tc_out = (-s0 - sqrt(disc)) / vv;
    }
    return 1;
}

int ref_pair_test(const ref_grid* g, const ref_params* p,
                  const double ri[3], const double vi[3],
                  const double rj[3], const double vj[3],
                  double* d2, double* tp)
{
    derived G;
    if (derive(g, p, &G)) return -1;
    return test_pair(&G, p->dt, ri, vi, rj, vj, d2, tp, NULL);
}

/* ------------------------------------------------------------------------ */
/* Particle views and binning                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const double *x, *y, *z, *vx, *vy, *vz;
    const uint32_t* id;
    const uint8_t* alive;
    const double* mass;     /* per-particle mass, or NULL: params.mass for all */
} view;

/* Finite coordinates and velocities (and a finite positive mass when the
 * particles carry their own). */
static int finite6(const view* V, int64_t i)
{
    return isfinite(V->x[i]) && isfinite(V->y[i]) && isfinite(V->z[i]) &&
           isfinite(V->vx[i]) && isfinite(V->vy[i]) && isfinite(V->vz[i]) &&
           (!V->mass || (isfinite(V->mass[i]) && V->mass[i] > 0.0));
}

/* A particle takes part in the partner search when it is alive and all of
 * its coordinates are finite. */
static int usable(const view* V, int64_t i)
{
    if (V->alive && !V->alive[i]) return 0;
    return finite6(V, i);
}

static void load(const view* V, int64_t i, double r[3], double v[3])
{
    r[0] = V->x[i]; r[1] = V->y[i]; r[2] = V->z[i];
    v[0] = V->vx[i]; v[1] = V->vy[i]; v[2] = V->vz[i];
}

/* Cell lists by a plain counting sort: cell[i] (-1 if not usable),
 * first[c]..first[c+1] indexes member[]. */
typedef struct {
    int64_t* cell;
    int64_t* first;
    int64_t* member;
} bins;

static int make_bins(const derived* G, const ref_grid* g, const view* V, bins* Bn)
{
    Bn->cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V->n > 0 ? V->n : 1));
    Bn->first = (int64_t*)calloc((size_t)G->C + 1, sizeof(int64_t));
    Bn->member = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V->n > 0 ? V->n : 1));
    if (!Bn->cell || !Bn->first || !Bn->member) return -1;
    for (int64_t i = 0; i < V->n; ++i) {
        if (!usable(V, i)) { Bn->cell[i] = -1; continue; }
        int32_t cx = axis_bin(V->x[i], g->lo[0], G->inv_w[0], G->n[0]);
        int32_t cy = axis_bin(V->y[i], g->lo[1], G->inv_w[1], G->n[1]);
        int32_t cz = axis_bin(V->z[i], g->lo[2], G->inv_w[2], G->n[2]);
        Bn->cell[i] = cx + (int64_t)G->n[0] * (cy + (int64_t)G->n[1] * cz);
        Bn->first[Bn->cell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < G->C; ++c) Bn->first[c + 1] += Bn->first[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)G->C);
    if (!fill) return -1;
    memcpy(fill, Bn->first, sizeof(int64_t) * (size_t)G->C);
    for (int64_t i = 0; i < V->n; ++i)
        if (Bn->cell[i] >= 0) Bn->member[fill[Bn->cell[i]]++] = i;
    free(fill);
    return 0;
}

static void free_bins(bins* Bn)
{
    free(Bn->cell); free(Bn->first); free(Bn->member);
}

/* Criterion 3: the closest candidate, ties to the lower id. */
static void consider(const derived* G, double dt, const view* V, int64_t j,
                     const double ri[3], const double vi[3],
                     int64_t* bj, double* bkey, double* bd2, uint64_t* ncand)
{
    double rj[3], vj[3], d2, tp, tc;
    load(V, j, rj, vj);
    if (!test_pair(G, dt, ri, vi, rj, vj, &d2, &tp, G->rank_time ? &tc : NULL)) return;
    *ncand += 1;
    /* Criterion 3: the smallest d_min (or, ranked by time, the earliest
     * contact), ties to the lower id. */
    double key = G->rank_time ? tc : d2;
    if (*bj < 0 || key < *bkey || (key == *bkey && V->id[j] < V->id[*bj])) {
        *bj = j;
        *bkey = key;
        *bd2 = d2;
    }
}

static void best_of(const derived* G, double dt, const view* V, const bins* Bn,
                    int mode, int64_t i, int64_t* bj_out, double* bd2_out, uint64_t* ncand)
{
    int64_t bj = -1;
    double bd2 = 0.0, bkey = 0.0;
    *bj_out = -1; *bd2_out = 0.0;
    if (Bn->cell[i] < 0) return;
    double ri[3], vi[3];
    load(V, i, ri, vi);
    if (mode == REF_MODE_BINNED) {
        int64_t nb[27];
        int k = stencil(G, Bn->cell[i], nb);
        for (int s = 0; s < k; ++s)
            for (int64_t m = Bn->first[nb[s]]; m < Bn->first[nb[s] + 1]; ++m) {
                int64_t j = Bn->member[m];
                if (j != i) consider(G, dt, V, j, ri, vi, &bj, &bkey, &bd2, ncand);
            }
    } else {
        for (int64_t j = 0; j < V->n; ++j) {
            if (j == i || Bn->cell[j] < 0) continue;
            if (mode == REF_MODE_BRUTE && !adjacent(G, Bn->cell[i], Bn->cell[j])) continue;
            consider(G, dt, V, j, ri, vi, &bj, &bkey, &bd2, ncand);
        }
    }
    *bj_out = bj;
    *bd2_out = bd2;
}

static int nthreads_or_default(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static uint64_t search_all(const derived* G, double dt, const view* V, const bins* Bn,
                           int mode, int nthreads, int64_t* best, double* best_d2)
{
    uint64_t total = 0;
    int nt = nthreads_or_default(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total) num_threads(nt)
    for (int64_t i = 0; i < V->n; ++i) {
        uint64_t nc = 0;
        best_of(G, dt, V, Bn, mode, i, &best[i], &best_d2[i], &nc);
        total += nc;
    }
    return total;
}

static int check_common(const derived* G, const ref_grid* g, const ref_params* p, int64_t n,
                        const void* x, const void* y, const void* z,
                        const void* vx, const void* vy, const void* vz, const void* id)
{
    (void)G; (void)g; (void)p;
    if (n < 0) return -1;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !id)) return -1;
    return 0;
}

/* Time step of Sec. 3: dt = dx / v_max, so that no particle crosses more
 * than one c-bin per step; the caller's dt is the upper bound. */
static double step_dt(const derived* G, const ref_params* p, const view* V)
{
    if (!(p->flags & REF_ADAPTIVE_DT)) return p->dt;
    double dx = 0.0;
    for (int a = 0; a < 3; ++a)
        if (G->n[a] > 1 && (dx == 0.0 || G->w[a] < dx)) dx = G->w[a];
    double vmax2 = 0.0;
    for (int64_t i = 0; i < V->n; ++i) {
        if (V->alive && !V->alive[i]) continue;
        if (!finite6(V, i)) continue;
        double v2 = (V->vx[i] * V->vx[i] + V->vy[i] * V->vy[i]) + V->vz[i] * V->vz[i];
        if (v2 > vmax2) vmax2 = v2;
    }
    if (dx == 0.0 || vmax2 == 0.0) return p->dt;
    double t = dx / sqrt(vmax2);
    return t < p->dt ? t : p->dt;
}

/* Copy of the parameters with the step's dt filled in. */
static void with_step_dt(const derived* G, const ref_params* p, const view* V, ref_params* q)
{
    *q = *p;
    q->dt = step_dt(G, p, V);
}

double ref_step_dt(const ref_grid* g, const ref_params* p, int64_t n,
                   const double* x, const double* y, const double* z,
                   const double* vx, const double* vy, const double* vz,
                   const uint8_t* alive)
{
    derived G;
    if (derive(g, p, &G)) return -1.0;
    if (n < 0 || (n > 0 && (!x || !y || !z || !vx || !vy || !vz))) return -1.0;
    static const uint32_t no_id = 0;
    view V = { n, x, y, z, vx, vy, vz, &no_id, alive, NULL };
    return step_dt(&G, p, &V);
}

int ref_best(const ref_grid* g, const ref_params* p, int64_t n,
             const double* x, const double* y, const double* z,
             const double* vx, const double* vy, const double* vz,
             const uint32_t* id, const uint8_t* alive, int mode, int nthreads,
             int64_t* best, double* best_d2)
{
    derived G;
    if (derive(g, p, &G)) return -1;
    if (G.pair_random) return -1;
    if (check_common(&G, g, p, n, x, y, z, vx, vy, vz, id)) return -1;
    if (mode < 0 || mode > 2 || (n > 0 && (!best || !best_d2))) return -1;
    view V = { n, x, y, z, vx, vy, vz, id, alive, NULL };
    const double dt = step_dt(&G, p, &V);
    bins Bn;
    if (make_bins(&G, g, &V, &Bn)) { free_bins(&Bn); return -2; }
    search_all(&G, dt, &V, &Bn, mode, nthreads, best, best_d2);
    free_bins(&Bn);
    return 0;
}

int ref_best_sample(const ref_grid* g, const ref_params* p, int64_t n,
                    const double* x, const double* y, const double* z,
                    const double* vx, const double* vy, const double* vz,
                    const uint32_t* id, const uint8_t* alive,
                    int64_t ns, const int64_t* sample, int nthreads,
                    int64_t* best, double* best_d2)
{
    derived G;
    if (derive(g, p, &G)) return -1;
    if (G.pair_random) return -1;
    if (check_common(&G, g, p, n, x, y, z, vx, vy, vz, id)) return -1;
    if (ns < 0 || (ns > 0 && (!sample || !best || !best_d2))) return -1;
    for (int64_t k = 0; k < ns; ++k)
        if (sample[k] < 0 || sample[k] >= n) return -1;
    view V = { n, x, y, z, vx, vy, vz, id, alive, NULL };
    const double dt = step_dt(&G, p, &V);
    bins Bn;
    if (make_bins(&G, g, &V, &Bn)) { free_bins(&Bn); return -2; }
    int nt = nthreads_or_default(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t k = 0; k < ns; ++k) {
        uint64_t nc = 0;
        best_of(&G, dt, &V, &Bn, REF_MODE_BINNED, sample[k], &best[k], &best_d2[k], &nc);
    }
    free_bins(&Bn);
    return 0;
}

uint64_t ref_count_tests(const ref_grid* g, int64_t n,
                         const double* x, const double* y, const double* z,
                         const double* vx, const double* vy, const double* vz,
                         const uint8_t* alive)
{
    derived G;
    if (derive(g, NULL, &G) || n < 0) return 0;
    static const uint32_t no_id = 0;
    view V = { n, x, y, z, vx, vy, vz, &no_id, alive, NULL };
    bins Bn;
    if (make_bins(&G, g, &V, &Bn)) { free_bins(&Bn); return 0; }
    uint64_t total = 0;
    for (int64_t c = 0; c < G.C; ++c) {
        uint64_t nc = (uint64_t)(Bn.first[c + 1] - Bn.first[c]);
        total += nc * (nc - (nc > 0 ? 1 : 0)) / 2;
        int64_t nb[27];
        int k = stencil(&G, c, nb);
        for (int s = 0; s < k; ++s)
            if (nb[s] > c) total += nc * (uint64_t)(Bn.first[nb[s] + 1] - Bn.first[nb[s]]);
    }
    free_bins(&Bn);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Random partners inside a c-bin (REF_PAIR_RANDOM, the usual DSMC rule that */
/* Sec. 2.3 describes).                                                      */
/* ------------------------------------------------------------------------ */
static void philox_words(const ref_params* p, uint32_t c1, uint32_t c2, uint32_t w[4])
{
    uint32_t key[2] = { (uint32_t)p->seed, (uint32_t)(p->seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)p->step, c1, c2, (p->instance << 8) | 255u };
    ref_philox4x32_10(ctr, key, w);
}

typedef struct { uint32_t key, id; int64_t idx; } keyed;

static int by_key_then_id(const void* a, const void* b)
{
    const keyed* x = (const keyed*)a;
    const keyed* y = (const keyed*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

/* best[i] = the random partner of i (or -1); returns the pairs formed. */
static int64_t random_pairs(const derived* G, const ref_params* p, const view* V, const bins* Bn,
                            int64_t* best)
{
    int64_t formed = 0, most = 0;
    for (int64_t i = 0; i < V->n; ++i) best[i] = -1;
    for (int64_t c = 0; c < G->C; ++c)
        if (Bn->first[c + 1] - Bn->first[c] > most) most = Bn->first[c + 1] - Bn->first[c];
    keyed* t = (keyed*)malloc(sizeof(keyed) * (size_t)(most > 0 ? most : 1));
    if (!t) return -1;
    for (int64_t c = 0; c < G->C; ++c) {
        const int64_t m = Bn->first[c + 1] - Bn->first[c];
        for (int64_t k = 0; k < m; ++k) {
            const int64_t i = Bn->member[Bn->first[c] + k];
            uint32_t w[4];
            philox_words(p, V->id[i], V->id[i], w);
            t[k].key = w[0];
            t[k].id = V->id[i];
            t[k].idx = i;
        }
        qsort(t, (size_t)m, sizeof(keyed), by_key_then_id);
        for (int64_t k = 0; k + 1 < m; k += 2) {
            best[t[k].idx] = t[k + 1].idx;
            best[t[k + 1].idx] = t[k].idx;
            formed++;
        }
    }
    free(t);
    return formed;
}

/* Whether the random pair {i, j} of a c-bin with nc particles collides. */
static int random_pair_collides(const derived* G, const ref_params* p, const view* V, int64_t i, int64_t j,
                                int64_t nc)
{
    const int64_t A = V->id[i] < V->id[j] ? i : j, B = A == i ? j : i;
    double rA[3], vA[3], rB[3], vB[3], r[3], u[3];
    load(V, A, rA, vA);
    load(V, B, rB, vB);
    rel(G, rA, vA, rB, vB, r, u);
    double vv = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double g = sqrt(vv);
    double prob = ((((double)(nc - 1) * p->sigma) * g) * p->dt) / G->cellvol;
    uint32_t w[4];
    philox_words(p, V->id[A], V->id[B], w);
    return unit_double(w[0], w[1]) < prob;
}

/* ------------------------------------------------------------------------ */
/* Scattering and position update                                            */
/* ------------------------------------------------------------------------ */
/* Scattering of the accepted pair {i, j} (Sec. 3): A is the lower id, B the
 * higher one; r, u, t_poca are recomputed from A's side.  Writes the new
 * velocities of i and j, t_poca, and their virial terms (separation at the
 * point of closest approach times momentum change, half per particle). */
static void scatter_pair(const derived* G, const ref_params* p, const view* V, int64_t i, int64_t j,
                         double vi_new[3], double vj_new[3], double* tp_out,
                         double vir_i[3], double vir_j[3])
{
    /* Random partners have no point of closest approach: t_poca = 0, the
     * collision happens at the start of the step. */
    const int i_is_A = V->id[i] < V->id[j];
    const int64_t A = i_is_A ? i : j, B = i_is_A ? j : i;
    double rA[3], vA[3], rB[3], vB[3], r[3], u[3], nhat[3], nA[3], nB[3];
    load(V, A, rA, vA);
    load(V, B, rB, vB);
    rel(G, rA, vA, rB, vB, r, u);
    double s0 = (r[0] * u[0] + r[1] * u[1]) + r[2] * u[2];
    double vv = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double tp = G->pair_random ? 0.0 : -s0 / vv;
    if (p->flags & REF_PLANAR)
        ref_direction_planar(p->seed, p->step, p->instance, V->id[A], V->id[B], nhat);
    else
        ref_direction(p->seed, p->step, p->instance, V->id[A], V->id[B], nhat);
    /* Centre-of-mass frame (Sec. 3): the relative speed g is kept and the
     * outgoing velocities are opposite along nhat.  Equal masses: v_cm is the
     * mean and each moves g/2; masses mA, mB: v_cm is mass-weighted and A
     * moves mB g / (mA + mB), B moves mA g / (mA + mB). */
    double gr = sqrt(vv);
    double mA = V->mass ? V->mass[A] : p->mass, mB = V->mass ? V->mass[B] : p->mass;
    if (!V->mass) {
        double h = 0.5 * gr;
        for (int a = 0; a < 3; ++a) {
            double vcm = 0.5 * (vA[a] + vB[a]);
            nA[a] = vcm + h * nhat[a];
            nB[a] = vcm - h * nhat[a];
        }
    } else {
        double M = mA + mB;
        double hA = (mB / M) * gr, hB = (mA / M) * gr;
        for (int a = 0; a < 3; ++a) {
            double vcm = (mA * vA[a] + mB * vB[a]) / M;
            nA[a] = vcm + hA * nhat[a];
            nB[a] = vcm - hB * nhat[a];
        }
    }
    for (int a = 0; a < 3; ++a) {
        double sep = r[a] + tp * u[a];
        double dpA = mA * (nA[a] - vA[a]);
        double dpB = mB * (nB[a] - vB[a]);
        double virA = 0.5 * sep * dpA / p->dt;
        double virB = 0.5 * (-sep) * dpB / p->dt;
        vi_new[a] = i_is_A ? nA[a] : nB[a];
        vj_new[a] = i_is_A ? nB[a] : nA[a];
        vir_i[a] = i_is_A ? virA : virB;
        vir_j[a] = i_is_A ? virB : virA;
    }
    *tp_out = tp;
}

/* Position update (Sec. 3): old velocity up to t_poca and the new one for
 * the rest of the step for a collider (vnew != NULL), straight line
 * otherwise; then the walls, once per axis.  Returns 1 when absorbed. */
static int move_one(const derived* G, const ref_grid* g, double dt, double r[3], double v[3],
                    const double* vnew, double tp)
{
    for (int a = 0; a < 3; ++a) {
        if (vnew) {
            r[a] = (r[a] + v[a] * tp) + vnew[a] * (dt - tp);
            v[a] = vnew[a];
        } else {
            r[a] = r[a] + v[a] * dt;
        }
    }
    int gone = 0;
    for (int a = 0; a < 3; ++a) {
        double lo = g->lo[a], hi = g->hi[a];
        double xn = r[a];
        if (G->bc[a] == REF_BC_REFLECT) {
            if (xn < lo) { r[a] = lo + (lo - xn); v[a] = -v[a]; }
            else if (xn > hi) { r[a] = hi - (xn - hi); v[a] = -v[a]; }
        } else if (G->bc[a] == REF_BC_PERIODIC) {
            if (xn < lo) xn = xn + G->L[a];
            if (xn >= hi) xn = xn - G->L[a];
            r[a] = xn;
        } else {
            if (xn < lo || xn >= hi) gone = 1;
        }
    }
    return gone;
}

int ref_step_sample(const ref_grid* g, const ref_params* p, int64_t n,
                    const double* x, const double* y, const double* z,
                    const double* vx, const double* vy, const double* vz,
                    const uint32_t* id, const uint8_t* alive, const double* mass,
                    int64_t ns, const int64_t* sample, int nthreads,
                    double* out_state, int64_t* out_partner, uint8_t* out_alive)
{
    derived G;
    if (derive(g, p, &G)) return -1;
    if (G.pair_random) return -1;
    if (check_common(&G, g, p, n, x, y, z, vx, vy, vz, id)) return -1;
    if (ns < 0 || (ns > 0 && (!sample || !out_state || !out_partner || !out_alive))) return -1;
    for (int64_t k = 0; k < ns; ++k)
        if (sample[k] < 0 || sample[k] >= n) return -1;
    view V = { n, x, y, z, vx, vy, vz, id, alive, mass };
    ref_params q;
    with_step_dt(&G, p, &V, &q);
    p = &q;
    bins Bn;
    if (make_bins(&G, g, &V, &Bn)) { free_bins(&Bn); return -2; }
    int nt = nthreads_or_default(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t k = 0; k < ns; ++k) {
        int64_t i = sample[k], bi, bb;
        double d2, r[3], v[3], vnew[3], vj_new[3], tp = 0.0, vir_i[3], vir_j[3];
        uint64_t nc = 0;
        load(&V, i, r, v);
        out_partner[k] = -1;
        out_alive[k] = (alive && !alive[i]) ? 0 : 1;
        if (!out_alive[k]) {
            for (int a = 0; a < 3; ++a) { out_state[6 * k + a] = r[a]; out_state[6 * k + 3 + a] = v[a]; }
            continue;
        }
        best_of(&G, p->dt, &V, &Bn, REF_MODE_BINNED, i, &bi, &d2, &nc);
        int mutual = 0;
        if (bi >= 0) {
            best_of(&G, p->dt, &V, &Bn, REF_MODE_BINNED, bi, &bb, &d2, &nc);
            mutual = bb == i;
        }
        if (mutual) {
            scatter_pair(&G, p, &V, i, bi, vnew, vj_new, &tp, vir_i, vir_j);
            out_partner[k] = bi;
        }
        if (move_one(&G, g, p->dt, r, v, mutual ? vnew : NULL, tp)) out_alive[k] = 0;
        for (int a = 0; a < 3; ++a) { out_state[6 * k + a] = r[a]; out_state[6 * k + 3 + a] = v[a]; }
    }
    free_bins(&Bn);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation for the global sums.                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Wall time of the phases of the last ref_step (for the CPU baseline of the */
/* benchmark; instrumentation only).                                         */
/* ------------------------------------------------------------------------ */
static double phase_ms[REF_NPHASES];

static double now_ms(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return 1e3 * (double)t.tv_sec + 1e-6 * (double)t.tv_nsec;
}

void ref_last_phase_ms(double out[REF_NPHASES])
{
    for (int k = 0; k < REF_NPHASES; ++k) out[k] = phase_ms[k];
}

/* ------------------------------------------------------------------------ */
/* One step                                                                  */
/* ------------------------------------------------------------------------ */
int ref_step(const ref_grid* g, const ref_params* p, int64_t n,
             double* x, double* y, double* z,
             double* vx, double* vy, double* vz,
             const uint32_t* id, uint8_t* alive, const double* mass, int mode, int nthreads,
             uint32_t* pairs, int64_t pair_cap,
             uint64_t* counters, double* moments, double* globals)
{
    derived G;
    if (derive(g, p, &G)) return -1;
    if (check_common(&G, g, p, n, x, y, z, vx, vy, vz, id)) return -1;
    if (mode < 0 || mode > 2 || pair_cap < 0) return -1;
    for (int a = 0; a < 3; ++a)
        if (G.bc[a] == REF_BC_ABSORB && !alive) return -1;
    view V = { n, x, y, z, vx, vy, vz, id, alive, mass };
    ref_params q;
    with_step_dt(&G, p, &V, &q);
    p = &q;
    const double dt = p->dt;
    uint64_t cnt[8] = { 0 };
    for (int k = 0; k < REF_NPHASES; ++k) phase_ms[k] = 0.0;
    double t_mark = now_ms(), t_now;
#define REF_PHASE_END(k) (t_now = now_ms(), phase_ms[k] += t_now - t_mark, t_mark = t_now)

    size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t* best = (int64_t*)malloc(sizeof(int64_t) * nn);
    double* best_d2 = (double*)malloc(sizeof(double) * nn);
    int64_t* partner = (int64_t*)malloc(sizeof(int64_t) * nn);
    double* nvel = (double*)malloc(sizeof(double) * 3 * nn);
    double* vir = (double*)calloc(3 * nn, sizeof(double));
    double* tpoca = (double*)malloc(sizeof(double) * nn);
    bins Bn = { 0, 0, 0 };
    int rc = 0;
    if (!best || !best_d2 || !partner || !nvel || !vir || !tpoca) { rc = -2; goto done; }

    /* Diagnostics on the incoming state. */
    for (int64_t i = 0; i < n; ++i) {
        if (alive && !alive[i]) continue;
        if (!finite6(&V, i)) { cnt[REF_CNT_NONFINITE]++; continue; }
        if (fabs(vx[i]) * dt > G.w[0] || fabs(vy[i]) * dt > G.w[1] || fabs(vz[i]) * dt > G.w[2])
            cnt[REF_CNT_FAST]++;
    }

    /* 1. Sort into c-bins. */
    if (make_bins(&G, g, &V, &Bn)) { rc = -2; goto done; }
    REF_PHASE_END(REF_PHASE_BIN);
    if (G.pair_random) {
        /* 2'-3'. Random partners inside each c-bin, each pair its own
         * acceptance draw (REF_PAIR_RANDOM). */
        int64_t formed = random_pairs(&G, p, &V, &Bn, best);
        if (formed < 0) { rc = -2; goto done; }
        cnt[REF_CNT_TESTS] = (uint64_t)formed;
        cnt[REF_CNT_CAND] = cnt[REF_CNT_HAVE_BEST] = 2 * (uint64_t)formed;
        for (int64_t i = 0; i < n; ++i) partner[i] = -1;
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = best[i];
            if (j < 0 || !(id[i] < id[j])) continue;
            int64_t c = Bn.cell[i];
            if (random_pair_collides(&G, p, &V, i, j, Bn.first[c + 1] - Bn.first[c])) {
                partner[i] = j;
                partner[j] = i;
            }
        }
        REF_PHASE_END(REF_PHASE_SEARCH);
        goto scatter;
    }
    for (int64_t c = 0; c < G.C; ++c) {
        uint64_t nc = (uint64_t)(Bn.first[c + 1] - Bn.first[c]);
        cnt[REF_CNT_TESTS] += nc * (nc - (nc > 0 ? 1 : 0)) / 2;
        int64_t nb[27];
        int k = stencil(&G, c, nb);
        for (int s = 0; s < k; ++s)
            if (nb[s] > c) cnt[REF_CNT_TESTS] += nc * (uint64_t)(Bn.first[nb[s] + 1] - Bn.first[nb[s]]);
    }

    /* 2. Closest candidate of every particle. */
    cnt[REF_CNT_CAND] = search_all(&G, dt, &V, &Bn, mode, nthreads, best, best_d2);
    REF_PHASE_END(REF_PHASE_SEARCH);
    for (int64_t i = 0; i < n; ++i)
        if (best[i] >= 0) cnt[REF_CNT_HAVE_BEST]++;

    /* 3. Unambiguous partners: i and j chose each other. */
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = best[i];
        partner[i] = (j >= 0 && best[j] == i) ? j : -1;
    }

    REF_PHASE_END(REF_PHASE_PAIR);

    /* 4. Scattering of every accepted pair, visited once from its lower id. */
scatter:;
    int64_t npairs = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = partner[i];
        if (j < 0 || !(id[i] < id[j])) continue;
        scatter_pair(&G, p, &V, i, j, nvel + 3 * i, nvel + 3 * j, &tpoca[i], vir + 3 * i, vir + 3 * j);
        tpoca[j] = tpoca[i];
        if (pairs && npairs < pair_cap) {
            pairs[2 * npairs] = id[i];
            pairs[2 * npairs + 1] = id[j];
        }
        npairs++;
    }
    cnt[REF_CNT_PAIRS] = (uint64_t)npairs;

    REF_PHASE_END(REF_PHASE_SCATTER);

    /* 5. Positions: split at t_poca for colliders, free streaming otherwise;
     * then the walls. */
    for (int64_t i = 0; i < n; ++i) {
        if (alive && !alive[i]) continue;
        double r[3], v[3];
        load(&V, i, r, v);
        int gone = move_one(&G, g, dt, r, v, partner[i] >= 0 ? nvel + 3 * i : NULL, tpoca[i]);
        x[i] = r[0]; y[i] = r[1]; z[i] = r[2];
        vx[i] = v[0]; vy[i] = v[1]; vz[i] = v[2];
        if (gone) { alive[i] = 0; cnt[REF_CNT_ABSORBED]++; }
    }

    REF_PHASE_END(REF_PHASE_MOVE);

    /* 6. Moments of the post-step state per o-bin, and global sums. */
    nsum gp[3] = { { 0, 0 }, { 0, 0 }, { 0, 0 } }, ge = { 0, 0 }, gv = { 0, 0 }, gm = { 0, 0 };
    double vmax2 = 0.0;
    int64_t* ob = (int64_t*)malloc(sizeof(int64_t) * nn);
    if (!ob) { rc = -2; goto done; }
    if (moments) memset(moments, 0, sizeof(double) * (size_t)G.B * REF_M_STRIDE);
    for (int64_t i = 0; i < n; ++i) {
        ob[i] = -1;
        if (alive && !alive[i]) continue;
        if (!finite6(&V, i)) continue;
        cnt[REF_CNT_ALIVE]++;
        int32_t bx = axis_bin(x[i], g->lo[0], G.inv_wo[0], G.no[0]);
        int32_t by = axis_bin(y[i], g->lo[1], G.inv_wo[1], G.no[1]);
        int32_t bz = axis_bin(z[i], g->lo[2], G.inv_wo[2], G.no[2]);
        ob[i] = bx + (int64_t)G.no[0] * (by + (int64_t)G.no[1] * bz);
        double v2 = (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
        const double m = mass ? mass[i] : p->mass;
        nadd(&gp[0], m * vx[i]);
        nadd(&gp[1], m * vy[i]);
        nadd(&gp[2], m * vz[i]);
        nadd(&ge, 0.5 * m * v2);
        nadd(&gm, m);
        nadd(&gv, (vir[3 * i] + vir[3 * i + 1]) + vir[3 * i + 2]);
        if (v2 > vmax2) vmax2 = v2;
        if (moments) {
            double* M = moments + ob[i] * REF_M_STRIDE;
            M[REF_M_COUNT] += 1.0;
            M[REF_M_MASS] += m;
            M[REF_M_PX] += m * vx[i];
            M[REF_M_PX + 1] += m * vy[i];
            M[REF_M_PX + 2] += m * vz[i];
            M[REF_M_VIRX] += vir[3 * i];
            M[REF_M_VIRX + 1] += vir[3 * i + 1];
            M[REF_M_VIRX + 2] += vir[3 * i + 2];
            if (partner[i] >= 0) M[REF_M_NCOLL] += 1.0;
        }
    }
    if (moments) {
        /* Second pass: spread around the bin's bulk velocity. */
        for (int64_t i = 0; i < n; ++i) {
            if (ob[i] < 0) continue;
            double* M = moments + ob[i] * REF_M_STRIDE;
            const double m = mass ? mass[i] : p->mass;
            double mass_bin = M[REF_M_MASS];
            double vb[3] = { M[REF_M_PX] / mass_bin, M[REF_M_PX + 1] / mass_bin, M[REF_M_PX + 2] / mass_bin };
            double dv0 = vx[i] - vb[0], dv1 = vy[i] - vb[1], dv2 = vz[i] - vb[2];
            M[REF_M_CXX] += m * dv0 * dv0;
            M[REF_M_CXX + 1] += m * dv1 * dv1;
            M[REF_M_CXX + 2] += m * dv2 * dv2;
        }
    }
    free(ob);
    if (globals) {
        globals[REF_G_PX] = nval(&gp[0]);
        globals[REF_G_PY] = nval(&gp[1]);
        globals[REF_G_PZ] = nval(&gp[2]);
        globals[REF_G_EKIN] = nval(&ge);
        globals[REF_G_VMAX2] = vmax2;
        globals[REF_G_VIRIAL] = nval(&gv);
        globals[REF_G_MASS] = nval(&gm);
        globals[REF_G_DT] = dt;
    }
    if (counters) memcpy(counters, cnt, sizeof(cnt));
    REF_PHASE_END(REF_PHASE_MOMENTS);
#undef REF_PHASE_END

done:
    free_bins(&Bn);
    free(best); free(best_d2); free(partner); free(nvel); free(vir); free(tpoca);
    return rc;
}
