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
};

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
template <typename real> void launch_adapt_dt(Inst<real>* inst, const double* gpart, int n_inst, hipStream_t s);
template <typename real> void launch_search(const StepArgs<real>& a, int block, int group, hipStream_t s);
template <typename real> void launch_search_mix(const StepArgs<real>& a, int block, hipStream_t s);
template <typename real> void launch_move(const StepArgs<real>& a, hipStream_t s);
template <typename real> void launch_random_pairs(const StepArgs<real>& a, hipStream_t s);

}  // namespace tpkmc
