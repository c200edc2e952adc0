// Internal declarations shared by the HIP translation units of libtpkmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpkmc.h"

namespace tpkmc {

// Particles per work-group in every per-particle kernel; a work-group never
// spans two instances (see the block table below).
constexpr int kBlock = 256;
constexpr int kWave = 64;

// Slots of the per-work-group partial results (doubles), reduced per
// instance by the finalize kernel.
enum GPart {
    GP_PX = 0, GP_PY, GP_PZ, GP_EKIN, GP_VMAX2, GP_VIR, GP_MASS,
    GP_ALIVE, GP_PAIRS, GP_ABSORBED, GP_TESTS2, GP_CAND, GP_HAVEBEST,
    GP_FAST, GP_NONFINITE, GP_VMAX0, kGPart
};

// Exact o-bin sums, in two passes over the particles.  The move records,
// per o-bin, the exponent E per kind of term of a power of two above every
// term (|x| < 2^E, an integer maximum, so the order does not matter) and the
// counts of particles and colliders.  The moment pass then rounds each term
// once to an integer q, a multiple of 2^(E-50+h) (|q| <= 2^(50-h)), where
// the headroom h = max(0, ceil(log2 n) - 12) grows with the o-bin's n
// particles (none up to 4096): the n integers of a value sum to less than
// 2^62 in magnitude, so every partial and the total fit one int64, and
// integer sums do not depend on the order of the terms.  Kinds: 0 m (v -
// shift) per axis, 1 m (v - shift)^2 per axis, 2 virial terms, 3 mass.  Per
// o-bin: values 0..2 momentum, 3..5 spread, 6..8 virial, 9 mass
// (per-particle masses only); the particle count in the low 32 bits of nc
// and the collider count in its high 32 bits (at most 2^32 - 1 particles
// per o-bin); the four exponents (biased by kExpBias; 0: no nonzero term).
constexpr int kAccVals = 10;
constexpr int kExpBias = 1100;
struct ObAcc {
    long long sum[kAccVals];
    unsigned long long nc;
    int32_t e[4];
    unsigned long long pad[3];
};
static_assert(sizeof(ObAcc) == 128, "one o-bin accumulator is 128 B");
__host__ __device__ inline int acc_headroom(unsigned long long n) {
    const int c = n <= 1 ? 0 : 64 - __builtin_clzll(n - 1);  // ceil(log2 n)
    return c > 12 ? c - 12 : 0;
}
__host__ __device__ constexpr int acc_kind(int k) { return k < 3 ? 0 : k < 6 ? 1 : k < 9 ? 2 : 3; }

// Instance descriptor on the device.  Derived grid quantities are computed
// on the host in double, exactly like the CPU oracle, then cast to `real`.
template <typename real>
struct Inst {
    int64_t off, cnt;         // particle slice [off, off + cnt)
    int64_t cell_off;         // first global c-bin; C bins + 1 sentinel bin
    int64_t obin_off;         // first global o-bin
    int32_t C;                // c-bins of this instance
    int32_t n[3], bc[3];      // c-bins and boundary per axis
    int32_t no[3];            // o-bins per axis
    int32_t blk0, nblk;       // range in the block table
    int32_t chunk0, nchunk;   // range in the chunk table (partials reduction)
    uint32_t seed_lo, seed_hi, step_lo, instance;
    uint32_t flags;           // TPKMC_EMIT_PAIRS | TPKMC_ALLOW_REORDER
    int32_t band_log2;        // y-band height 2^band_log2 of the c-bin order
    real lo[3], hi[3], L[3], halfL[3], inv_w[3], inv_wo[3], w[3];
    real dt, D2, mass;
    double mass_d, dt_d;      // dt_d: this step's time step (set on the device with ADAPTIVE_DT)
    double dt_cap, dx_d;      // caller's dt; smallest c-bin width over axes with > 1 c-bin (0: none)
    double sigma_d, cellvol_d; // cross section; c-bin volume (area in the plane), for random partners
    // Adaptive time step: running maximum of |v|^2 (bit pattern of a
    // non-negative double) and the count of prep work-groups done; the last
    // one to finish resets both.
    unsigned long long run_v2;
    uint32_t prep_done;
    // Split c-bins (kSplit): a particle is slow when its |v|^2 <= vc2; slow
    // particles are binned on the n[] c-bins (the first Cf of the C), the
    // others on the configured ncfg[] c-bins after them, numbered
    // x + ncfg[0] * (y + ncfg[1] * z).  inv_wc: configured c-bins per unit
    // length.  vmax2_d: this step's largest |v|^2 before the move.
    int32_t ncfg[3];
    int32_t Cf;
    real vc2;
    real inv_wc[3];
    double vmax2_d;
};

// Bit of Inst::flags set by the host (outside the public flag bits): the
// c-bins are split by speed (slow particles on refined c-bins, see Inst).
constexpr uint32_t kSplit = 1u << 30;

// Bit of Inst::flags, set by the host (outside the public flag bits): the
// particles carry their own masses.
constexpr uint32_t kHasMass = 1u << 31;

// Block table entry: instance index and first particle of the work-group.
struct Blk {
    int32_t inst;
    int32_t first;
};

// Chunk of at most kChunk consecutive block-table entries of one instance,
// the unit of the first level of the per-instance reduction.
constexpr int kChunk = 256;
struct Chunk {
    int32_t first;
    int32_t count;
};

// Arguments of one step, shared by all kernels of a precision.
template <typename real>
struct StepArgs {
    // caller state (structure of arrays)
    real *x, *y, *z, *vx, *vy, *vz;
    uint32_t* id;
    uint8_t* alive;
    // scratch
    const Inst<real>* inst;
    const Blk* blk;
    int32_t nblk;
    int32_t* rank;            // rank inside its c-bin
    int32_t* start;           // counts, then exclusive prefix (ncells + 1)
    real* rec;                // c-bin ordered records, 8 reals per particle
    real* mass;               // caller's per-particle masses, or null
    real* rmass;              // masses in record order (with mass only)
    int32_t* src;             // record -> caller index
    int32_t* best;            // record -> partner record or -1 (FP64 search)
    int32_t* perm;            // random partners: c-bin-local order -> record
    unsigned long long* bkey; // record -> (d_min^2 bits, partner record) (FP32 search)
    double* gpart;            // [nblk][kGPart]
    double* shift;            // per-o-bin velocity shift (3 per o-bin)
    int32_t order;            // search work-group order: 0 contiguous per XCD, S > 0 chunks of S round-robin
    ObAcc* macc;              // per-o-bin exact sums, or null (no moments)
    real* vir;                // virial terms of each collider (3 per particle, caller index)
    uint8_t* coll;            // 1 if the particle collided this step (caller index)
    unsigned long long* mix;  // search mix counters (tests, s0 < 0, s0 < 0 < s1), or null
    // outputs
    uint32_t* pairs;
    int64_t pair_cap;
    unsigned long long* pair_count;
    double* moments;
};

// Launchers implemented per precision (tpkmc_f32.hip / tpkmc_f64.hip).
template <typename real> void launch_key(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_scatter(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_prep(Inst<real>* inst, const double* gpart, int n_inst, int max_nblk,
                                         hipStream_t s);
template <typename real> void launch_search(const StepArgs<real>& a, int block, int group, hipStream_t s);
template <typename real> void launch_search_mix(const StepArgs<real>& a, int block, int n_inst, bool split,
                                               hipStream_t s);
template <typename real> void launch_search_fast(const StepArgs<real>& a, int n_inst, hipStream_t s);
template <typename real> void launch_move(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_moments(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_random_pairs(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_speed_stats(const StepArgs<real>& a, hipStream_t s);

}  // namespace tpkmc
