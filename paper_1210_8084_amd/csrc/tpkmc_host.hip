// Host side of libtpkmc: the C ABI, argument checking, device scratch, the
// precision-independent kernels (clear, prefix sum, per-instance reduction)
// and the step pipeline, plain or captured as a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "tpkmc_internal.h"

#pragma clang fp contract(off)

using namespace tpkmc;

namespace {

constexpr int kScanItems = 8;                       // per thread
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanItems * kScanBlock;  // per work-group
constexpr int kPhases = 8;
// Default work-group order of the search: chunks of 16 work-groups dealt
// round-robin over the XCDs (StepArgs::order; see the autotuner).
constexpr int kDefaultSearchOrder = 16;

enum Phase { PH_CLEAR = 0, PH_KEY, PH_SCAN, PH_SCATTER, PH_SEARCH, PH_MOVE, PH_FINAL };

// ---------------------------------------------------------------- kernels
__global__ void k_clear(int32_t* start, int64_t ncell, unsigned long long* macc, int64_t nwords,
                        unsigned long long* pair_count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t t = t0; t < ncell; t += stride) start[t] = 0;
    if (macc)
        for (int64_t t = t0; t < nwords; t += stride) macc[t] = 0ull;
    if (t0 == 0) *pair_count = 0ull;
}

// Exclusive prefix sum of n int32 in place: per-tile totals, a single
// work-group scan of the totals, then per-tile scans with the tile offset.
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const int32_t* d, int64_t n, int32_t* tile_sum) {
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (b0 + k < n) s += d[b0 + k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) t += lds[w];
        tile_sum[blockIdx.x] = t;
    }
}

// Exclusive scan across one work-group of `v`; returns the prefix, and the
// total in *total.
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t* lds, int32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    __syncthreads();
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) woff += lds[k];
        tot += lds[k];
    }
    *total = tot;
    return woff + inc - v;
}

__global__ void __launch_bounds__(1024) k_scan_top(int32_t* tile_sum, int64_t ntiles) {
    __shared__ int32_t lds[16];
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < ntiles; c0 += blockDim.x) {
        const int64_t t = c0 + threadIdx.x;
        const int32_t v = t < ntiles ? tile_sum[t] : 0;
        int32_t total;
        const int32_t ex = block_exscan(v, lds, &total);
        if (t < ntiles) tile_sum[t] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(int32_t* d, int64_t n, const int32_t* tile_off) {
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = b0 + k < n ? d[b0 + k] : 0;
        s += v[k];
    }
    int32_t total;
    int32_t run = tile_off[blockIdx.x] + block_exscan(s, lds, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (b0 + k < n) d[b0 + k] = run;
        run += v[k];
    }
}

// Neumaier (compensated) accumulation.
struct NSum {
    double s = 0.0, c = 0.0;
    __device__ void add(double v) {
        const double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
    __device__ double value() const { return s + c; }
};

// Per-instance reduction of the work-group partials, in a fixed order:
// first each chunk of <= kChunk work-groups, then each instance's chunks.
// Sixteen threads per slot (work-groups of 256 threads): thread t of slot k
// folds rows t, t + 16, t + 32, ... (Neumaier sums for the FP slots, max for
// max|v|^2, plain sums for the integer-valued counts), then a butterfly over
// the sixteen lanes combines their partials with a commutative step, so all
// sixteen end with the same total.
constexpr int kSlotLanes = 256 / kGPart;
static_assert(kSlotLanes * kGPart == 256 && (kSlotLanes & (kSlotLanes - 1)) == 0, "slot lanes");

__device__ __forceinline__ void reduce_slots(const double* rows, int nrows, double* out) {
    const int k = threadIdx.x / kSlotLanes, t = threadIdx.x % kSlotLanes;
    double s = 0.0, c = 0.0;
    if (k == GP_VMAX2) {
        for (int r = t; r < nrows; r += kSlotLanes) s = fmax(s, rows[(int64_t)r * kGPart + k]);
        for (int o = 1; o < kSlotLanes; o <<= 1) s = fmax(s, __shfl_xor(s, o));
    } else if (k < GP_ALIVE) {
        NSum a;
        for (int r = t; r < nrows; r += kSlotLanes) a.add(rows[(int64_t)r * kGPart + k]);
        s = a.s;
        c = a.c;
        for (int o = 1; o < kSlotLanes; o <<= 1) {
            const double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
            const double sum = s + s2;
            const double err = fabs(s) >= fabs(s2) ? (s - sum) + s2 : (s2 - sum) + s;
            c = (c + c2) + err;
            s = sum;
        }
    } else {
        for (int r = t; r < nrows; r += kSlotLanes) s += rows[(int64_t)r * kGPart + k];
        for (int o = 1; o < kSlotLanes; o <<= 1) s += __shfl_xor(s, o);
    }
    if (t == 0) out[k] = s + c;
}

__global__ void __launch_bounds__(256) k_reduce_chunks(const Chunk* chunks, const double* gpart, double* cpart) {
    __shared__ double rows[kChunk * kGPart];
    const Chunk c = chunks[blockIdx.x];
    for (int t = threadIdx.x; t < c.count * kGPart; t += blockDim.x)
        rows[t] = gpart[(int64_t)c.first * kGPart + t];
    __syncthreads();
    reduce_slots(rows, c.count, cpart + (int64_t)blockIdx.x * kGPart);
}

template <typename real>
__global__ void __launch_bounds__(256) k_finalize(Inst<real>* inst, const double* cpart, uint64_t* counters,
                                                 double* globals, uint32_t* status,
                                                 const unsigned long long* pair_count, int64_t pair_cap,
                                                 int advance_step) {
    __shared__ double tot[kGPart];
    __shared__ double rows[kChunk * kGPart];
    Inst<real>& I = inst[blockIdx.x];
    // Chunk partials of this instance, staged in LDS kChunk rows at a time
    // (folded in order, so the result does not depend on the launch shape).
    double acc = 0.0;
    NSum ns;
    for (int c0 = 0; c0 < I.nchunk; c0 += kChunk) {
        const int nr = min(kChunk, I.nchunk - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < nr * kGPart; t += blockDim.x)
            rows[t] = cpart[(int64_t)(I.chunk0 + c0) * kGPart + t];
        __syncthreads();
        reduce_slots(rows, nr, tot);
        __syncthreads();
        if (threadIdx.x < kGPart) {
            const int k = threadIdx.x;
            if (k == GP_VMAX2) acc = fmax(acc, tot[k]);
            else if (k < GP_ALIVE) ns.add(tot[k]);
            else acc += tot[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < kGPart) tot[threadIdx.x] = threadIdx.x < GP_ALIVE && threadIdx.x != GP_VMAX2 ? ns.value() : acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int k0 = blockIdx.x;
    if (counters) {
        uint64_t* c = counters + 8 * k0;
        c[TPKMC_CNT_ALIVE] = (uint64_t)tot[GP_ALIVE];
        c[TPKMC_CNT_PAIRS] = (uint64_t)tot[GP_PAIRS];
        c[TPKMC_CNT_TESTS] = (uint64_t)tot[GP_TESTS2] / 2u;
        c[TPKMC_CNT_CAND] = (uint64_t)tot[GP_CAND];
        c[TPKMC_CNT_FAST] = (uint64_t)tot[GP_FAST];
        c[TPKMC_CNT_NONFINITE] = (uint64_t)tot[GP_NONFINITE];
        c[TPKMC_CNT_ABSORBED] = (uint64_t)tot[GP_ABSORBED];
        c[TPKMC_CNT_HAVE_BEST] = (uint64_t)tot[GP_HAVEBEST];
    }
    if (globals) {
        double* g = globals + 8 * k0;
        g[0] = tot[GP_PX];
        g[1] = tot[GP_PY];
        g[2] = tot[GP_PZ];
        g[3] = tot[GP_EKIN];
        g[4] = tot[GP_VMAX2];
        g[5] = tot[GP_VIR];
        g[6] = tot[GP_MASS];
        g[7] = I.dt_d;
    }
    uint32_t st = 0;
    if (tot[GP_NONFINITE] > 0.0) st |= TPKMC_STATUS_NONFINITE;
    if (tot[GP_FAST] > 0.0) st |= TPKMC_STATUS_FAST;
    if (k0 == 0 && (int64_t)*pair_count > pair_cap) st |= TPKMC_STATUS_PAIR_OVERFLOW;
    if (st) atomicOr(status, st);
    if (advance_step) I.step_lo += 1u;
}

// Exact shifted o-bin sums -> the moments of the output: momentum and central
// second moments; the bin mean becomes the shift of the next step, so the
// sums stay small next time.  Each integer sum is rounded once to double (a
// function of the exact sum only) and scaled by its power-of-two quantum.
// Each work-group (256 threads) stages its 256 o-bins' output rows through
// LDS, so the stores are coalesced; every output value is written.
template <typename real>
__global__ void __launch_bounds__(256) k_moments_final(const Inst<real>* inst, const ObAcc* macc, double* moments,
                                                       double* shift) {
    constexpr int kRows = 256;
    __shared__ double rows[kRows * TPKMC_MOMENT_STRIDE];
    const Inst<real>& I = inst[blockIdx.y];
    const int64_t nb = (int64_t)I.no[0] * I.no[1] * I.no[2];
    const int64_t b0 = (int64_t)blockIdx.x * kRows;
    if (b0 >= nb) return;  // whole work-group
    const int nloc = (int)min<int64_t>(kRows, nb - b0);
    if ((int)threadIdx.x < nloc) {
        const int64_t ob = I.obin_off + b0 + threadIdx.x;
        const ObAcc& A = macc[ob];
        double* M = rows + threadIdx.x * TPKMC_MOMENT_STRIDE;
        double* S = shift + ob * 3;
        const unsigned long long cnt = A.nc & 0xffffffffull, coll = A.nc >> 32;
        for (int k = 0; k < TPKMC_MOMENT_STRIDE; ++k) M[k] = 0.0;
        if (cnt > 0) {
            // Quanta 2^(E-50+h) of the four kinds (as in the moment pass); each
            // integer sum is rounded once to double, then scaled exactly.
            const int h = acc_headroom(cnt);
            double inv[4];
            for (int k = 0; k < 4; ++k) {
                const int e = A.e[k] > 0 ? A.e[k] - kExpBias : 0;
                inv[k] = ldexp(1.0, max(e, -969) - 50 + h);
            }
            double v[kAccVals];
            for (int k = 0; k < kAccVals; ++k) v[k] = (double)A.sum[k] * inv[acc_kind(k)];
            // Without per-particle masses the moment pass leaves the mass sum out.
            const double mass = (I.flags & kHasMass) ? v[9] : (double)cnt * I.mass_d;
            M[0] = (double)cnt;
            for (int ax = 0; ax < 3; ++ax) {
                const double s1 = v[ax], s2 = v[3 + ax];
                const double mean_off = s1 / mass;
                M[1 + ax] = s1 + mass * S[ax];
                M[4 + ax] = fmax(s2 - s1 * mean_off, 0.0);
                M[7 + ax] = v[6 + ax];
                S[ax] = S[ax] + mean_off;
            }
            M[10] = (double)coll;
            M[11] = mass;
        }
    }
    __syncthreads();
    double* M0 = moments + (I.obin_off + b0) * TPKMC_MOMENT_STRIDE;
    for (int t = threadIdx.x; t < nloc * TPKMC_MOMENT_STRIDE; t += kRows) M0[t] = rows[t];
}

// Tables of the allocation-free entry point, written on the device so that
// no host staging or copy is needed: its one instance descriptor (passed by
// value as a kernel argument), the block and chunk tables, and the o-bin
// velocity shifts and status word, cleared because the static scratch keeps
// the previous call's contents.
template <typename real>
__global__ void __launch_bounds__(256) k_setup_one(Inst<real> one, Inst<real>* inst, Blk* blk, int nblk,
                                                  Chunk* chunks, int nchunk, double* shift, int64_t nshift,
                                                  uint32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0) {
        *inst = one;
        *status = 0u;
    }
    for (int64_t t = t0; t < nblk; t += stride) blk[t] = Blk{0, (int32_t)(one.off + t * kBlock)};
    for (int64_t t = t0; t < nchunk; t += stride)
        chunks[t] = Chunk{(int32_t)(t * kChunk), (int32_t)min<int64_t>(kChunk, nblk - t * kChunk)};
    for (int64_t t = t0; t < nshift; t += stride) shift[t] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------- handle
// Device scratch of one step: owned by a handle (tpkmc_create), or carved
// out of the static scratch array by the allocation-free entry point.
struct Buffers {
    int32_t *rank, *start, *tiles, *src, *best, *perm;
    void *rec, *rmass, *inst;
    Blk* blk;
    Chunk* chunks;
    unsigned long long* bkey;
    double *gpart, *cpart, *shift;
    ObAcc* macc;      // exact o-bin sums, 128 B per o-bin
    void* vir;        // colliders' virial terms, 3 reals per particle
    uint8_t* coll;    // collided flags, 1 B per particle
    unsigned long long* pair_count;
    uint32_t* status;
    unsigned long long* mix;  // counters of tpkmc_search_mix (handles only)
};

struct ProfRec {
    int phase;
    hipEvent_t a, b;
};

struct tpkmc_handle {
    int device = 0, precision = TPKMC_FP64;
    int64_t max_n = 0, max_cells = 0, max_obins = 0, max_blk = 0;
    int32_t max_inst = 0;
    int64_t max_chunks = 0;
    Buffers b{};  // device scratch, allocated once in tpkmc_create
    hipStream_t last_stream = nullptr;
    hipStream_t own_stream = nullptr;
    int search_block = kWave;
    int search_group = 2;
    int search_order = kDefaultSearchOrder;  // work-group order of the search (StepArgs::order)
    bool shape_chosen = false;  // set by tpkmc_set_search or tpkmc_autotune
    // c-bins chosen by tpkmc_autotune per batch position, each applied while
    // the instance at that position keeps the grid and parameters it was
    // tuned on (the key); capacity of the c-bin counts array.
    struct Cells {
        tpkmc_grid g;
        double sigma, dt;
        uint32_t flags;
        int32_t n[3];   // c-bins of the slow particles (the configured ones: no split)
        double vc;      // speed bound of the slow particles
    };
    std::vector<Cells> cells;
    int64_t cell_cap = 0;
    bool profiling = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    double prof_ms[kPhases] = {};
    int64_t prof_n[kPhases] = {};
    hipGraphExec_t gexec = nullptr;
    // Pinned staging ring for the instance and block tables: a slot is
    // rewritten only after the copy that last read it has run.
    static constexpr int kRing = 8;
    char* stage[kRing] = {};
    hipEvent_t stage_ev[kRing] = {};
    bool stage_used[kRing] = {};
    size_t stage_bytes = 0;
    int stage_next = 0;
};

namespace {

// Host view of one validated call.
// Target size of one band plane of records (see row_of).
constexpr double kBandBytes = 1 << 20;

struct Plan {
    int n_inst = 0;
    int64_t ncell_tot = 0, nob_tot = 0, max_nob = 0;
    int nblk = 0;
    bool adaptive = false;    // some instance takes the adaptive time step
    bool any_search = false;  // some instance takes partners by closest approach
    bool split = false;       // some instance has c-bins split by speed
    bool any_random = false;  // some instance takes random partners
    std::vector<Blk> blk;
    std::vector<Chunk> chunks;
    std::vector<char> inst_bytes;
};

bool bad_ptr(const void* p) { return p == nullptr; }

bool bad_state(const tpkmc_particles* s) {
    return s->n > 0 && (bad_ptr(s->x) || bad_ptr(s->y) || bad_ptr(s->z) || bad_ptr(s->vx) || bad_ptr(s->vy) ||
                        bad_ptr(s->vz) || bad_ptr(s->id));
}

// Validates one instance and fills its device descriptor, except the
// offsets into the c-bin, o-bin, block and chunk tables, which the caller
// sets.  C and B: its c-bins and o-bins.  nref (split c-bins): the slow
// particles' c-bins per axis, vc their speed bound.
template <typename real>
int fill_inst(const tpkmc_particles* s, const tpkmc_instance& q, Inst<real>& d, int64_t& C, int64_t& B,
              const int32_t* nref = nullptr, double vc = 0.0) {
    const tpkmc_grid& g = q.grid;
    const tpkmc_params& p = q.params;
    if (q.offset < 0 || q.count < 0 || q.offset + q.count > s->n) return TPKMC_EINVAL;
    if (!(std::isfinite(p.sigma) && p.sigma >= 0.0)) return TPKMC_EINVAL;
    if (!(std::isfinite(p.mass) && p.mass > 0.0)) return TPKMC_EINVAL;
    if (!(std::isfinite(p.dt) && p.dt > 0.0)) return TPKMC_EINVAL;
    if (p.instance >= (1u << 24)) return TPKMC_EINVAL;
    if (p.flags & ~(uint32_t)(TPKMC_EMIT_PAIRS | TPKMC_ALLOW_REORDER | TPKMC_ADAPTIVE_DT | TPKMC_PLANAR |
                              TPKMC_RANK_TIME | TPKMC_PAIR_RANDOM))
        return TPKMC_EINVAL;
    if ((p.flags & TPKMC_RANK_TIME) && (p.flags & TPKMC_PAIR_RANDOM)) return TPKMC_EINVAL;
    const bool planar = (p.flags & TPKMC_PLANAR) != 0;
    if (planar && g.ncell[2] != 1) return TPKMC_EINVAL;
    std::memset(&d, 0, sizeof(d));
    C = 1;
    B = 1;
    int64_t Cc = 1;
    double dx = 0.0, wd[3];
    for (int a = 0; a < 3; ++a) {
        if (g.ncell[a] < 1 || g.nobin[a] < 1) return TPKMC_EINVAL;
        if (g.ncell[a] > (1 << 24) || g.nobin[a] > (1 << 24)) return TPKMC_EINVAL;
        if (!(std::isfinite(g.lo[a]) && std::isfinite(g.hi[a]) && g.hi[a] > g.lo[a])) return TPKMC_EINVAL;
        if (g.bc[a] < TPKMC_BC_REFLECT || g.bc[a] > TPKMC_BC_ABSORB) return TPKMC_EINVAL;
        if (g.bc[a] == TPKMC_BC_ABSORB && s->alive == nullptr) return TPKMC_EINVAL;
        if (nref && (nref[a] < g.ncell[a] || nref[a] > (1 << 24))) return TPKMC_EINVAL;
        C *= nref ? nref[a] : g.ncell[a];
        Cc *= g.ncell[a];
        B *= g.nobin[a];
        // Derived grid quantities, in double, in the order of the reference.
        // With split c-bins the slow particles are binned on nc c-bins; the
        // fast ones, the time step and the fast-particle check keep the
        // configured ones.
        const double L = g.hi[a] - g.lo[a];
        const int32_t nc = nref ? nref[a] : g.ncell[a];
        d.n[a] = nc;
        d.ncfg[a] = g.ncell[a];
        d.inv_wc[a] = (real)((double)g.ncell[a] / L);
        d.no[a] = g.nobin[a];
        d.bc[a] = g.bc[a];
        d.lo[a] = (real)g.lo[a];
        d.hi[a] = (real)g.hi[a];
        d.L[a] = (real)L;
        d.halfL[a] = (real)(0.5 * L);
        d.w[a] = (real)(L / (double)g.ncell[a]);
        wd[a] = L / (double)g.ncell[a];
        if (g.ncell[a] > 1 && (dx == 0.0 || L / (double)g.ncell[a] < dx)) dx = L / (double)g.ncell[a];
        d.inv_w[a] = (real)((double)nc / L);
        d.inv_wo[a] = (real)((double)g.nobin[a] / L);
    }
    const bool split = nref && (nref[0] != g.ncell[0] || nref[1] != g.ncell[1] || nref[2] != g.ncell[2]);
    const int64_t Cf = C;
    if (split) C = Cf + Cc;
    if (C + 1 > (int64_t)1 << 30 || B > (int64_t)1 << 30) return TPKMC_EINVAL;
    d.off = q.offset;
    d.cnt = q.count;
    d.C = (int32_t)C;
    d.Cf = (int32_t)Cf;
    d.seed_lo = (uint32_t)p.seed;
    d.seed_hi = (uint32_t)(p.seed >> 32);
    d.step_lo = (uint32_t)p.step;
    d.instance = p.instance;
    d.flags = p.flags | (s->mass ? kHasMass : 0u);
    if (split) {
        d.flags |= kSplit;
        d.vc2 = (real)(vc * vc);
    }
    d.dt = (real)p.dt;
    // Largest accepted d_min^2: sigma = pi D^2 in space, sigma = 2 D in
    // the plane (same expressions as the reference).
    const double Dp = 0.5 * p.sigma;
    d.D2 = planar ? (real)(Dp * Dp) : (real)(p.sigma / M_PI);
    d.mass = (real)p.mass;
    d.mass_d = p.mass;
    d.dt_d = p.dt;
    d.dt_cap = p.dt;
    d.dx_d = dx;
    // Random partners: the cross section and the c-bin volume (an area
    // in the plane), in the reference's order.
    d.sigma_d = p.sigma;
    d.cellvol_d = planar ? wd[0] * wd[1] : (wd[0] * wd[1]) * wd[2];
    // Band height of the c-bin order: the largest power of two of rows
    // whose band plane (rows x n_x c-bins of records) stays within
    // kBandBytes, so that one XCD's L2 holds the plane its neighbourhood
    // walk reads twice.  Planar and one-row grids keep a single band.
    d.band_log2 = 30;
    if (d.n[2] > 1 && d.n[1] > 1 && q.count > 0) {
        const double row_bytes = (double)d.n[0] * ((double)q.count / (double)Cf) * 8.0 * sizeof(real);
        int h = 0;
        while (h < 30 && (double)(2 << h) * row_bytes <= (double)kBandBytes) ++h;
        if ((1 << h) < d.n[1]) d.band_log2 = h;
    }
    return TPKMC_OK;
}

// Flags that decide the choice of c-bins (with the grid, sigma and dt).
constexpr uint32_t kCellKey = TPKMC_ADAPTIVE_DT | TPKMC_PLANAR | TPKMC_RANK_TIME | TPKMC_PAIR_RANDOM;

// The c-bins autotune chose for batch position k, if the instance there
// keeps the grid and parameters it was tuned on.
const tpkmc_handle::Cells* tuned_cells(const tpkmc_handle* h, int k, const tpkmc_instance& q) {
    if (k >= (int)h->cells.size()) return nullptr;
    const tpkmc_handle::Cells& c = h->cells[k];
    if (std::memcmp(&c.g, &q.grid, sizeof(tpkmc_grid)) != 0 || c.sigma != q.params.sigma ||
        c.dt != q.params.dt || c.flags != (q.params.flags & kCellKey))
        return nullptr;
    return &c;
}

template <typename real>
int make_plan(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, Plan& P,
              bool configured = false) {
    if (!s || !in || n_inst < 1) return TPKMC_EINVAL;
    if (n_inst > h->max_inst) return TPKMC_ECAPACITY;
    if (s->n < 0) return TPKMC_EINVAL;
    if (s->n > h->max_n) return TPKMC_ECAPACITY;
    if (bad_state(s)) return TPKMC_EINVAL;
    std::vector<std::pair<int64_t, int64_t>> spans;
    std::vector<Inst<real>> I(n_inst);
    P.blk.clear();
    P.chunks.clear();
    P.n_inst = n_inst;
    P.adaptive = false;
    P.any_search = false;
    P.split = false;
    P.any_random = false;
    P.ncell_tot = 0;
    P.nob_tot = 0;
    P.max_nob = 0;
    for (int k = 0; k < n_inst; ++k) {
        const tpkmc_instance& q = in[k];
        Inst<real>& d = I[k];
        int64_t C, B;
        const tpkmc_handle::Cells* tc = configured ? nullptr : tuned_cells(h, k, q);
        const int rc = fill_inst<real>(s, q, d, C, B, tc ? tc->n : nullptr, tc ? tc->vc : 0.0);
        if (rc) return rc;
        if (d.flags & kSplit) P.split = true;
        spans.push_back({q.offset, q.count});
        if (q.params.flags & TPKMC_PAIR_RANDOM) P.any_random = true;
        else P.any_search = true;
        if (q.params.flags & TPKMC_ADAPTIVE_DT) P.adaptive = true;
        d.cell_off = P.ncell_tot;
        d.obin_off = P.nob_tot;
        P.ncell_tot += C + 1;
        P.nob_tot += B;
        P.max_nob = std::max(P.max_nob, B);
        d.blk0 = (int32_t)P.blk.size();
        for (int64_t o = 0; o < q.count; o += kBlock) P.blk.push_back({k, (int32_t)(q.offset + o)});
        d.nblk = (int32_t)P.blk.size() - d.blk0;
        d.chunk0 = (int32_t)P.chunks.size();
        for (int32_t b = 0; b < d.nblk; b += kChunk)
            P.chunks.push_back({d.blk0 + b, std::min<int32_t>(kChunk, d.nblk - b)});
        d.nchunk = (int32_t)P.chunks.size() - d.chunk0;
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k - 1].first + spans[k - 1].second > spans[k].first) return TPKMC_EINVAL;
    if (P.ncell_tot > h->cell_cap) return TPKMC_ECAPACITY;
    if (P.nob_tot > h->max_obins) return TPKMC_ECAPACITY;
    if ((int64_t)P.blk.size() > h->max_blk) return TPKMC_ECAPACITY;
    if ((int64_t)P.chunks.size() > h->max_chunks) return TPKMC_ECAPACITY;
    P.nblk = (int)P.blk.size();
    P.inst_bytes.resize(sizeof(Inst<real>) * n_inst);
    std::memcpy(P.inst_bytes.data(), I.data(), P.inst_bytes.size());
    return TPKMC_OK;
}

int check_outputs(const tpkmc_outputs* o) {
    if (!o) return TPKMC_OK;
    if (o->pairs && o->pair_cap < 0) return TPKMC_EINVAL;
    return TPKMC_OK;
}

hipEvent_t pool_event(tpkmc_handle* h) {
    if (h->pool_used == h->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->pool.push_back(e);
    }
    return h->pool[h->pool_used++];
}

struct PhaseScope {
    tpkmc_handle* h;
    int phase;
    hipStream_t s;
    hipEvent_t b = nullptr;
    PhaseScope(tpkmc_handle* h_, int ph, hipStream_t s_, bool on) : h(h_), phase(ph), s(s_) {
        if (!on) { h = nullptr; return; }
        hipEvent_t a = pool_event(h);
        b = pool_event(h);
        if (!a || !b) { h = nullptr; return; }
        hipEventRecord(a, s);
        h->prof.push_back({phase, a, b});
    }
    ~PhaseScope() {
        if (h) hipEventRecord(b, s);
    }
};

template <typename real>
StepArgs<real> make_args(const Buffers& B, const tpkmc_particles* s, const tpkmc_outputs* o, int nblk) {
    StepArgs<real> a{};
    a.x = (real*)s->x; a.y = (real*)s->y; a.z = (real*)s->z;
    a.vx = (real*)s->vx; a.vy = (real*)s->vy; a.vz = (real*)s->vz;
    a.id = s->id;
    a.alive = s->alive;
    a.inst = (const Inst<real>*)B.inst;
    a.blk = B.blk;
    a.nblk = nblk;
    a.rank = B.rank;
    a.start = B.start;
    a.rec = (real*)B.rec;
    a.mass = (real*)s->mass;
    a.rmass = (real*)B.rmass;
    a.src = B.src;
    a.best = B.best;
    a.perm = B.perm;
    a.bkey = B.bkey;
    a.gpart = B.gpart;
    a.shift = B.shift;
    a.macc = (o && o->moments) ? B.macc : nullptr;
    a.vir = (real*)B.vir;
    a.coll = B.coll;
    a.pairs = o ? o->pairs : nullptr;
    a.pair_cap = (o && o->pairs) ? o->pair_cap : 0;
    a.pair_count = B.pair_count;
    a.mix = B.mix;
    a.moments = o ? o->moments : nullptr;
    return a;
}

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

void enqueue_scan(const Buffers& B, int64_t n, hipStream_t s) {
    const int64_t tiles = scan_tiles(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, B.start, n, B.tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, B.tiles, tiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, B.start, n, B.tiles);
}

// Shape of one launch sequence: what enqueue_step needs of a Plan.
struct Shape {
    int n_inst, nblk, nchunk;
    int64_t ncell_tot, nob_tot, max_nob;
    bool prep, any_search, any_random, split;  // prep: some instance needs the prep kernel
};

Shape shape_of(const Plan& P) {
    return Shape{P.n_inst, P.nblk, (int)P.chunks.size(), P.ncell_tot, P.nob_tot, P.max_nob,
                 P.adaptive || P.split, P.any_search, P.any_random, P.split};
}

// Everything of one step after the tables are on the device.  `h` only
// records phase timings (null: none).
template <typename real>
void enqueue_step(tpkmc_handle* h, const Buffers& B, const StepArgs<real>& a, const tpkmc_outputs* o,
                  const Shape& P, int search_block, int search_group, hipStream_t s, bool prof,
                  int advance_step) {
    const bool mom = o && o->moments;
    const int64_t nwords = mom ? P.nob_tot * (int64_t)(sizeof(ObAcc) / 8) : 0;
    {
        PhaseScope ps(h, PH_CLEAR, s, prof);
        const int64_t work = std::max<int64_t>(P.ncell_tot + 1, nwords);
        const int64_t grid = std::min<int64_t>((work + 255) / 256, 4096);
        hipLaunchKernelGGL(k_clear, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(256), 0, s, B.start,
                           P.ncell_tot + 1, mom ? (unsigned long long*)B.macc : nullptr, nwords, B.pair_count);
    }
    if (P.nblk > 0) {
        PhaseScope ps(h, PH_KEY, s, prof);
        launch_key<real>(a, s);
        if (P.prep) launch_prep<real>((Inst<real>*)B.inst, B.gpart, P.n_inst, P.nblk, s);
    }
    {
        PhaseScope ps(h, PH_SCAN, s, prof);
        enqueue_scan(B, P.ncell_tot + 1, s);
    }
    if (P.nblk > 0) {
        {
            PhaseScope ps(h, PH_SCATTER, s, prof);
            launch_scatter<real>(a, s);
        }
        {
            PhaseScope ps(h, PH_SEARCH, s, prof);
            if (P.any_search) launch_search<real>(a, search_block, search_group, s);
            if (P.split) launch_search_fast<real>(a, P.n_inst, s);
            if (P.any_random) launch_random_pairs<real>(a, s);
        }
        {
            PhaseScope ps(h, PH_MOVE, s, prof);
            launch_move<real>(a, s);
            if (mom) launch_moments<real>(a, s);
        }
    }
    {
        PhaseScope ps(h, PH_FINAL, s, prof);
        if (P.nchunk > 0)
            hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)P.nchunk), dim3(256), 0, s,
                               (const Chunk*)B.chunks, (const double*)B.gpart, B.cpart);
        hipLaunchKernelGGL(k_finalize<real>, dim3(P.n_inst), dim3(256), 0, s, (Inst<real>*)B.inst, B.cpart,
                           o ? o->counters : nullptr, o ? o->globals : nullptr, B.status, B.pair_count,
                           a.pair_cap, advance_step);
        if (mom && P.max_nob > 0) {
            const unsigned gx = (unsigned)((P.max_nob + 255) / 256);
            hipLaunchKernelGGL(k_moments_final<real>, dim3(gx, P.n_inst), dim3(256), 0, s,
                               (const Inst<real>*)B.inst, (const ObAcc*)B.macc, o->moments, B.shift);
        }
    }
}

int upload(tpkmc_handle* h, const Plan& P, hipStream_t s) {
    const size_t ib = P.inst_bytes.size(), bb = sizeof(Blk) * P.blk.size(), cb = sizeof(Chunk) * P.chunks.size();
    if (ib + bb + cb > h->stage_bytes) return TPKMC_ECAPACITY;
    const int k = h->stage_next;
    h->stage_next = (k + 1) % tpkmc_handle::kRing;
    if (h->stage_used[k] && hipEventSynchronize(h->stage_ev[k]) != hipSuccess) return TPKMC_EHIP;
    std::memcpy(h->stage[k], P.inst_bytes.data(), ib);
    if (bb) std::memcpy(h->stage[k] + ib, P.blk.data(), bb);
    if (cb) std::memcpy(h->stage[k] + ib + bb, P.chunks.data(), cb);
    if (hipMemcpyAsync(h->b.inst, h->stage[k], ib, hipMemcpyHostToDevice, s) != hipSuccess) return TPKMC_EHIP;
    if (bb && hipMemcpyAsync(h->b.blk, h->stage[k] + ib, bb, hipMemcpyHostToDevice, s) != hipSuccess)
        return TPKMC_EHIP;
    if (cb && hipMemcpyAsync(h->b.chunks, h->stage[k] + ib + bb, cb, hipMemcpyHostToDevice, s) != hipSuccess)
        return TPKMC_EHIP;
    if (hipEventRecord(h->stage_ev[k], s) != hipSuccess) return TPKMC_EHIP;
    h->stage_used[k] = true;
    return TPKMC_OK;
}

template <typename real>
int step_impl(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst,
              const tpkmc_outputs* o, hipStream_t st) {
    Plan P;
    int rc = make_plan<real>(h, s, in, n_inst, P);
    if (rc) return rc;
    if ((rc = check_outputs(o))) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    if ((rc = upload(h, P, st))) return rc;
    StepArgs<real> a = make_args<real>(h->b, s, o, P.nblk);
    a.order = h->search_order;
    enqueue_step<real>(h, h->b, a, o, shape_of(P), h->search_block, h->search_group, st, h->profiling, 0);
    h->last_stream = st;
    return hipGetLastError() == hipSuccess ? TPKMC_OK : TPKMC_EHIP;
}

template <typename real>
int tune_impl(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, hipStream_t st);

template <typename real>
int run_impl(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, int nsteps,
             const tpkmc_outputs* o, hipStream_t caller) {
    if (nsteps < 0) return TPKMC_EINVAL;
    Plan P;
    int rc = make_plan<real>(h, s, in, n_inst, P, true);  // validation before anything runs
    if (rc) return rc;
    if ((rc = check_outputs(o))) return rc;
    if (nsteps == 0) return TPKMC_OK;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    // Graphs are captured on a non-default stream; order it after the caller.
    hipStream_t st = caller ? caller : h->own_stream;
    hipEvent_t ev = nullptr;
    if (!caller) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return TPKMC_EHIP;
        hipEventRecord(ev, nullptr);
        hipStreamWaitEvent(st, ev, 0);
    }
    // First use without a chosen launch shape: tune it on this batch (the
    // state is not modified; every shape gives the same results).
    if (!h->shape_chosen && (rc = tune_impl<real>(h, s, in, n_inst, st))) return rc;
    if ((rc = make_plan<real>(h, s, in, n_inst, P))) return rc;  // with the tuned c-bins
    if ((rc = upload(h, P, st))) return rc;
    StepArgs<real> a = make_args<real>(h->b, s, o, P.nblk);
    a.order = h->search_order;
    if (h->gexec) {
        hipStreamSynchronize(h->last_stream ? h->last_stream : st);
        hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return TPKMC_EHIP;
    enqueue_step<real>(nullptr, h->b, a, o, shape_of(P), h->search_block, h->search_group, st, false, 1);
    if (hipStreamEndCapture(st, &graph) != hipSuccess || !graph) return TPKMC_EHIP;
    if (hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(graph);
        return TPKMC_EHIP;
    }
    hipGraphDestroy(graph);
    for (int k = 0; k < nsteps; ++k)
        if (hipGraphLaunch(h->gexec, st) != hipSuccess) return TPKMC_EHIP;
    if (!caller) {
        hipEventRecord(ev, st);
        hipStreamWaitEvent(nullptr, ev, 0);
        hipEventDestroy(ev);
    }
    h->last_stream = st;
    return hipGetLastError() == hipSuccess ? TPKMC_OK : TPKMC_EHIP;
}

template <typename T>
int dalloc(T** p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void**)p, sizeof(T) * (size_t)count) == hipSuccess ? 0 : -1;
}

// Grows the c-bin counts array (and its scan tiles) to hold `need` c-bins.
int grow_cells(tpkmc_handle* h, int64_t need) {
    if (need <= h->cell_cap) return TPKMC_OK;
    if (need >= ((int64_t)1 << 30)) return TPKMC_ECAPACITY;
    if (hipDeviceSynchronize() != hipSuccess) return TPKMC_EHIP;
    if (h->gexec) {
        hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    hipFree(h->b.start);
    hipFree(h->b.tiles);
    h->b.start = nullptr;
    h->b.tiles = nullptr;
    const int64_t tiles = (need + 1 + kScanTile - 1) / kScanTile + 1;
    if (dalloc(&h->b.start, need + 1) || dalloc(&h->b.tiles, tiles)) {
        h->cell_cap = 0;
        return TPKMC_ENOMEM;
    }
    h->cell_cap = need;
    return TPKMC_OK;
}

// Split c-bins (range S10 of the partner search).  Two particles of speed at
// most v_c that meet the criteria of Sec. 2.4 within the step start at most
// D + 2 v_c dt apart, so the slow particles (|v| <= v_c) can be binned on
// c-bins down to that width without losing a pair, and every pair of them
// that meets the criteria lies in neighbouring configured c-bins too.  The
// fast particles keep the configured c-bins and neighbourhood (the search's
// fast particle pass), so the step's results are the configured grid's
// whatever the speeds do later; only the search's work changes.  The bound
// is v_c = 2 v_rms over the instance's live particles, set for the gas as it
// will be once thermalised: an isolated gas keeps its root-mean-square speed
// (its energy is conserved) while its largest speed grows with the tail of
// the distribution, and a Maxwellian has 0.7% of its particles above 2 v_rms
// in three dimensions (1.8% in two), few enough that the finer c-bins of
// the rest more than pay for their searches.  Where the particles above
// 2 v_rms hold more than half of the kinetic energy (a Maxwellian: 3.5% in
// three dimensions, 9% in two, 26% in one), the gas is far from thermal (a
// point blast): collisions share that energy out and lift many more
// particles above 2 v_rms later in the run.  There the bound is 6 v_rms,
// above which at most 1/36 of the particles can ever be, as long as the
// energy is conserved (Markov's inequality on |v|^2; the 16M Sedov blast:
// 3.11 ms/step, against 3.17 with sqrt(20) v_rms and 3.35 unsplit).  Per
// instance (not with random partners,
// whose draw depends on the c-bin) and per axis, the slow particles' c-bins
// are the largest count whose width keeps a factor 1 + 1/64 over that reach
// (the rounding of the binning and of the pair test), used when it is at
// least 1.25 times the configured count (3 or more on periodic axes, never
// on a planar z), with at most one c-bin per two particles.
constexpr double kSpeedBound = 2.0;      // thermal gases
constexpr double kSpeedBoundHot = 6.0;   // far from thermal
constexpr double kReachMargin = 1.0 + 1.0 / 64.0;
constexpr double kMinRefine = 1.25;
constexpr double kHotEnergy = 0.5;
template <typename real>
int choose_cells(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, hipStream_t st) {
    h->cells.clear();
    Plan P;
    int rc = make_plan<real>(h, s, in, n_inst, P, true);
    if (rc) return rc;
    std::vector<Inst<real>> I(n_inst);
    std::memcpy(I.data(), P.inst_bytes.data(), P.inst_bytes.size());
    std::vector<double> v2sum(n_inst, 0.0), nlive(n_inst, 0.0), hot(n_inst, 0.0);
    if (P.nblk > 0) {
        // Two passes: the root-mean-square speeds, then the energy held above
        // each instance's bound.
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                for (int k = 0; k < n_inst; ++k) {
                    const double vc = nlive[k] > 0.0 ? kSpeedBound * sqrt(v2sum[k] / nlive[k]) : 0.0;
                    I[k].vc2 = (real)(vc * vc);
                }
                std::memcpy(P.inst_bytes.data(), I.data(), P.inst_bytes.size());
            }
            if ((rc = upload(h, P, st))) return rc;
            tpkmc_outputs none{};
            StepArgs<real> a = make_args<real>(h->b, s, &none, P.nblk);
            launch_speed_stats<real>(a, st);
            std::vector<double> gp((size_t)P.nblk * kGPart);
            if (hipMemcpyAsync(gp.data(), h->b.gpart, sizeof(double) * gp.size(), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return TPKMC_EHIP;
            // Summed in block order, so the same state always gives the same c-bins.
            for (int b = 0; b < P.nblk; ++b) {
                const int k = P.blk[b].inst;
                if (pass == 0) {
                    v2sum[k] += gp[(size_t)b * kGPart + GP_PX];
                    nlive[k] += gp[(size_t)b * kGPart + GP_PY];
                } else {
                    hot[k] += gp[(size_t)b * kGPart + GP_PZ];
                }
            }
        }
    }
    int64_t total = 0;
    for (int k = 0; k < n_inst; ++k) {
        const tpkmc_instance& q = in[k];
        tpkmc_handle::Cells c{q.grid, q.params.sigma, q.params.dt, q.params.flags & kCellKey,
                              {q.grid.ncell[0], q.grid.ncell[1], q.grid.ncell[2]}, 0.0};
        const bool thermal = !(hot[k] > kHotEnergy * v2sum[k]);
        const double vc = nlive[k] > 0.0 ? (thermal ? kSpeedBound : kSpeedBoundHot) * sqrt(v2sum[k] / nlive[k]) : 0.0;
        const double reach = sqrt((double)I[k].D2) + 2.0 * vc * q.params.dt;
        const bool planar = (q.params.flags & TPKMC_PLANAR) != 0;
        int64_t cfg = 1;
        for (int a = 0; a < 3; ++a) cfg *= q.grid.ncell[a];
        if (!(q.params.flags & TPKMC_PAIR_RANDOM) && q.count > 0 && reach > 0.0 && std::isfinite(reach)) {
            const int64_t cap = std::max<int64_t>(cfg, q.count / 2);
            int32_t lo[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = (int32_t)std::ceil(kMinRefine * q.grid.ncell[a]);
                if (q.grid.bc[a] == TPKMC_BC_PERIODIC) lo[a] = std::max(lo[a], 3);
                if (planar && a == 2) continue;
                const double L = q.grid.hi[a] - q.grid.lo[a];
                const double nmax = std::floor(L / (kReachMargin * reach));
                if (nmax < (double)lo[a] || nmax > (double)(1 << 24)) continue;
                c.n[a] = (int32_t)nmax;
            }
            // At most `cap` c-bins: shrink the most refined axis first.
            for (;;) {
                int64_t prod = (int64_t)c.n[0] * c.n[1] * c.n[2];
                if (prod <= cap) break;
                int a = -1;
                double best = 1.0;
                for (int b = 0; b < 3; ++b) {
                    const double f = (double)c.n[b] / q.grid.ncell[b];
                    if (f > best) { best = f; a = b; }
                }
                if (a < 0) break;
                const int32_t m = (int32_t)std::floor(c.n[a] * 0.9);
                c.n[a] = m >= lo[a] ? m : q.grid.ncell[a];
            }
        }
        const int64_t nslow = (int64_t)c.n[0] * c.n[1] * c.n[2];
        if (nslow != cfg) c.vc = vc;
        total += (nslow != cfg ? nslow + cfg : cfg) + 1;
        h->cells.push_back(c);
    }
    if (total > h->cell_cap && (rc = grow_cells(h, total))) {
        h->cells.clear();
        return rc;
    }
    return TPKMC_OK;
}

template <typename real>
int tune_impl(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, hipStream_t st) {
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    int rc = choose_cells<real>(h, s, in, n_inst, st);
    if (rc) return rc;
    Plan P;
    rc = make_plan<real>(h, s, in, n_inst, P);
    if (rc) return rc;
    if (P.nblk == 0) return TPKMC_OK;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    if ((rc = upload(h, P, st))) return rc;
    tpkmc_outputs none{};
    StepArgs<real> a = make_args<real>(h->b, s, &none, P.nblk);
    a.order = 0;  // shapes are timed in the default work-group order
    // Bin once (clear, key, prefix, scatter); then time only the search.
    hipLaunchKernelGGL(k_clear, dim3(1024), dim3(256), 0, st, h->b.start, P.ncell_tot + 1,
                       (unsigned long long*)nullptr, (int64_t)0, h->b.pair_count);
    launch_key<real>(a, st);
    if (P.adaptive || P.split) launch_prep<real>((Inst<real>*)h->b.inst, h->b.gpart, P.n_inst, P.nblk, st);
    enqueue_scan(h->b, P.ncell_tot + 1, st);
    launch_scatter<real>(a, st);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // Results-neutral launch shapes: records per lane (1, 2, 4) and lanes per
    // work-group (64, 128, 256).  The default shape (2 records per lane, 64
    // lanes, the fastest on sparse bins) is timed first and is replaced only
    // by a shape at least 5% faster, so that near-ties do not flip the choice
    // from run to run (on the 16M Sedov blast 128 lanes time up to 4% faster
    // on the initial state and 4% slower later in the run).
    float best_ms = 1e30f;
    int best_block = kWave, best_group = 2;
    std::vector<std::pair<int, int>> shapes = {{2, kWave}};
    for (int grp : {1, 2, 4})
        for (int bs : {256, 128, 64})
            if (bs <= kBlock / grp && !(grp == 2 && bs == kWave)) shapes.push_back({grp, bs});
    // Warm the caches and clocks first: the first shape timed would
    // otherwise look slower than it is.
    for (int r = 0; r < 4; ++r) launch_search<real>(a, kWave, 2, st);
    for (const auto& sh : shapes) {
        const int grp = sh.first, bs = sh.second;
        launch_search<real>(a, bs, grp, st);  // warm-up
        hipEventRecord(e0, st);
        for (int r = 0; r < 3; ++r) launch_search<real>(a, bs, grp, st);
        hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { rc = TPKMC_EHIP; break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < 0.95f * best_ms) { best_ms = ms; best_block = bs; best_group = grp; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    // Work-group order of the search (results-neutral): chunks of 16
    // work-groups dealt round-robin over the XCDs (the default), contiguous
    // ranges per XCD, or chunks of 1 or 128; another order is kept only when
    // at least 5% faster, timed in the chosen shape.  The default balances
    // the XCDs by construction: where the work concentrates as a run goes on
    // (the shocked core of an implosion, the shell of a blast), contiguous
    // ranges leave it to one or two XCDs, which the initial state does not
    // show (on the Noh 8M implosion 9.7 against 6.8 ms per step).
    int best_order = kDefaultSearchOrder;
    if (!rc) {
        hipEvent_t f0, f1;
        hipEventCreate(&f0);
        hipEventCreate(&f1);
        float base_ms = 1e30f;
        for (int order : {kDefaultSearchOrder, 0, 1, 128}) {
            a.order = order;
            launch_search<real>(a, best_block, best_group, st);  // warm-up
            hipEventRecord(f0, st);
            for (int r = 0; r < 3; ++r) launch_search<real>(a, best_block, best_group, st);
            hipEventRecord(f1, st);
            if (hipEventSynchronize(f1) != hipSuccess) { rc = TPKMC_EHIP; break; }
            float ms = 0.f;
            hipEventElapsedTime(&ms, f0, f1);
            if (order == kDefaultSearchOrder) base_ms = best_ms = ms;
            else if (ms < 0.95f * best_ms && ms < 0.95f * base_ms) { best_ms = ms; best_order = order; }
        }
        hipEventDestroy(f0);
        hipEventDestroy(f1);
        a.order = 0;
    }
    h->search_block = best_block;
    h->search_group = best_group;
    h->search_order = best_order;
    h->shape_chosen = true;
    h->last_stream = st;
    return hipGetLastError() == hipSuccess ? TPKMC_OK : TPKMC_EHIP;
}

// The search's arithmetic mix on a state: bins it (clear, key, prefix,
// scatter) and runs the counting build of the search, which leaves the state
// and the step's outputs untouched.
template <typename real>
int mix_impl(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* in, int n_inst, uint64_t* counts,
             hipStream_t st) {
    if (!counts) return TPKMC_EINVAL;
    Plan P;
    int rc = make_plan<real>(h, s, in, n_inst, P);
    if (rc) return rc;
    counts[0] = counts[1] = counts[2] = 0;
    if (P.nblk == 0) return TPKMC_OK;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    if ((rc = upload(h, P, st))) return rc;
    tpkmc_outputs none{};
    StepArgs<real> a = make_args<real>(h->b, s, &none, P.nblk);
    a.order = h->search_order;
    hipLaunchKernelGGL(k_clear, dim3(1024), dim3(256), 0, st, h->b.start, P.ncell_tot + 1,
                       (unsigned long long*)nullptr, (int64_t)0, h->b.pair_count);
    launch_key<real>(a, st);
    if (P.adaptive || P.split) launch_prep<real>((Inst<real>*)h->b.inst, h->b.gpart, P.n_inst, P.nblk, st);
    enqueue_scan(h->b, P.ncell_tot + 1, st);
    launch_scatter<real>(a, st);
    if (hipMemsetAsync(h->b.mix, 0, 3 * sizeof(unsigned long long), st) != hipSuccess) return TPKMC_EHIP;
    launch_search_mix<real>(a, h->search_block, P.n_inst, P.split, st);
    if (hipMemcpyAsync(counts, h->b.mix, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return TPKMC_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return TPKMC_EHIP;
    for (int k = 0; k < 3; ++k) counts[k] /= 2u;  // the device counts each unordered pair twice
    h->last_stream = st;
    return hipGetLastError() == hipSuccess ? TPKMC_OK : TPKMC_EHIP;
}


void free_all(tpkmc_handle* h) {
    for (int k = 0; k < tpkmc_handle::kRing; ++k) {
        if (h->stage[k]) hipHostFree(h->stage[k]);
        if (h->stage_ev[k]) hipEventDestroy(h->stage_ev[k]);
    }
    hipFree(h->b.rank); hipFree(h->b.start); hipFree(h->b.tiles);
    hipFree(h->b.src); hipFree(h->b.best); hipFree(h->b.perm); hipFree(h->b.rec); hipFree(h->b.rmass); hipFree(h->b.inst);
    hipFree(h->b.blk); hipFree(h->b.chunks); hipFree(h->b.bkey); hipFree(h->b.cpart); hipFree(h->b.gpart); hipFree(h->b.shift); hipFree(h->b.macc); hipFree(h->b.vir); hipFree(h->b.coll); hipFree(h->b.pair_count); hipFree(h->b.status); hipFree(h->b.mix);
}

// ---------------------------------------------------------------- static scratch
// Scratch of the allocation-free entry point: one array per GPU, held until
// the process ends.  Host code never uses the name `scratch` as an address
// (on the host it is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[TPKMC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char* scratch_ptr[kMaxDevices] = {};

int scratch_of(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return TPKMC_EHIP;
        scratch_ptr[device] = (unsigned char*)p;
    }
    *out = scratch_ptr[device];
    return TPKMC_OK;
}

// Carves the buffers of one instance out of the region starting at `base`
// (256-byte aligned pieces) and returns the bytes they span; with base 0 it
// only measures.
template <typename real>
size_t carve(uintptr_t base, int64_t n, int64_t ncell_tot, int64_t nob, int nblk, int nchunk, bool masses,
             Buffers& B) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        const uintptr_t p = base + off;
        off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        return (void*)p;
    };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    B.rank = (int32_t*)take(4 * nn);
    B.src = (int32_t*)take(4 * nn);
    B.best = (int32_t*)take(4 * nn);
    B.perm = (int32_t*)take(4 * nn);
    B.rec = take(8 * sizeof(real) * nn);
    B.rmass = masses ? take(sizeof(real) * nn) : nullptr;
    B.bkey = std::is_same<real, float>::value ? (unsigned long long*)take(8 * nn) : nullptr;
    B.start = (int32_t*)take(4 * (size_t)(ncell_tot + 1));
    B.tiles = (int32_t*)take(4 * (size_t)(scan_tiles(ncell_tot + 1) + 1));
    B.inst = take(sizeof(Inst<real>));
    B.blk = (Blk*)take(sizeof(Blk) * (size_t)nblk);
    B.gpart = (double*)take(sizeof(double) * kGPart * (size_t)nblk);
    B.chunks = (Chunk*)take(sizeof(Chunk) * (size_t)nchunk);
    B.cpart = (double*)take(sizeof(double) * kGPart * (size_t)nchunk);
    B.shift = (double*)take(sizeof(double) * 3 * (size_t)std::max<int64_t>(nob, 1));
    B.macc = (ObAcc*)take(sizeof(ObAcc) * (size_t)std::max<int64_t>(nob, 1));
    B.vir = take(3 * sizeof(real) * nn);
    B.coll = (uint8_t*)take(nn);
    B.pair_count = (unsigned long long*)take(sizeof(unsigned long long));
    B.status = (uint32_t*)take(sizeof(uint32_t));
    return off;
}

template <typename real>
int step_noalloc_impl(int device, const tpkmc_grid* g, const tpkmc_params* p, const tpkmc_particles* s,
                      const tpkmc_outputs* o, hipStream_t st) {
    if (!g || !p || !s || s->n < 0 || bad_state(s)) return TPKMC_EINVAL;
    int rc = check_outputs(o);
    if (rc) return rc;
    tpkmc_instance q;
    q.offset = 0;
    q.count = s->n;
    q.grid = *g;
    q.params = *p;
    Inst<real> d;
    int64_t C = 0, B = 0;
    if ((rc = fill_inst<real>(s, q, d, C, B))) return rc;
    // Records are addressed with 32-bit byte offsets in the FP32 search.
    if (s->n >= ((int64_t)1 << 27)) return TPKMC_ECAPACITY;
    const int nblk = (int)((s->n + kBlock - 1) / kBlock);
    const int nchunk = (nblk + kChunk - 1) / kChunk;
    const int64_t ncell_tot = C + 1;
    d.cell_off = 0;
    d.obin_off = 0;
    d.blk0 = 0;
    d.nblk = nblk;
    d.chunk0 = 0;
    d.nchunk = nchunk;
    Buffers Bf{};
    if (carve<real>(0, s->n, ncell_tot, B, nblk, nchunk, s->mass != nullptr, Bf) > TPKMC_NOALLOC_SCRATCH_BYTES)
        return TPKMC_ECAPACITY;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return TPKMC_EHIP;
    if (device < 0 || device >= ndev || device >= kMaxDevices) return TPKMC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TPKMC_EHIP;
    unsigned char* base = nullptr;
    if ((rc = scratch_of(device, &base))) return rc;
    carve<real>((uintptr_t)base, s->n, ncell_tot, B, nblk, nchunk, s->mass != nullptr, Bf);
    const int64_t nshift = 3 * std::max<int64_t>(B, 1);
    const int64_t work = std::max<int64_t>(std::max<int64_t>(nblk, nchunk), nshift);
    const unsigned sgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 1024));
    hipLaunchKernelGGL(k_setup_one<real>, dim3(sgrid), dim3(256), 0, st, d, (Inst<real>*)Bf.inst, Bf.blk, nblk,
                       Bf.chunks, nchunk, Bf.shift, nshift, Bf.status);
    const bool random = (p->flags & TPKMC_PAIR_RANDOM) != 0;
    Shape P{};
    P.n_inst = 1;
    P.nblk = nblk;
    P.nchunk = nchunk;
    P.ncell_tot = ncell_tot;
    P.nob_tot = B;
    P.max_nob = B;
    P.prep = (p->flags & TPKMC_ADAPTIVE_DT) != 0;
    P.any_search = !random;
    P.any_random = random;
    P.split = false;
    StepArgs<real> a = make_args<real>(Bf, s, o, nblk);
    enqueue_step<real>(nullptr, Bf, a, o, P, kWave, 2, st, false, 0);
    return hipGetLastError() == hipSuccess ? TPKMC_OK : TPKMC_EHIP;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

int tpkmc_version(void) { return TPKMC_ABI_VERSION; }

const char* tpkmc_strerror(int code) {
    switch (code) {
        case TPKMC_OK: return "success";
        case TPKMC_EINVAL: return "invalid argument";
        case TPKMC_ENOMEM: return "device allocation failed";
        case TPKMC_EHIP: return "HIP runtime error";
        case TPKMC_ECAPACITY: return "input exceeds the capacity of the handle or of the static scratch";
        case TPKMC_EUNSUPPORTED: return "unsupported";
        default: return "unknown error code";
    }
}

int tpkmc_create(const tpkmc_config* cfg, tpkmc_handle** out) {
    if (!out) return TPKMC_EINVAL;
    *out = nullptr;
    // Records are addressed with 32-bit byte offsets in the FP32 search.
    const int64_t max_n = cfg && cfg->precision == TPKMC_FP32 ? ((int64_t)1 << 27) : ((int64_t)1 << 31);
    if (!cfg || cfg->max_particles < 0 || cfg->max_particles >= max_n || cfg->max_cells < 1 ||
        cfg->max_cells >= ((int64_t)1 << 30) || cfg->max_obins < 0 || cfg->max_obins >= ((int64_t)1 << 30) ||
        cfg->max_instances < 1 || cfg->flags != 0 ||
        (cfg->precision != TPKMC_FP64 && cfg->precision != TPKMC_FP32))
        return TPKMC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return TPKMC_EINVAL;
    if (hipSetDevice(cfg->device) != hipSuccess) return TPKMC_EHIP;
    tpkmc_handle* h = new (std::nothrow) tpkmc_handle();
    if (!h) return TPKMC_ENOMEM;
    h->device = cfg->device;
    h->precision = cfg->precision;
    h->max_n = cfg->max_particles;
    h->max_cells = cfg->max_cells;
    h->cell_cap = cfg->max_cells;
    h->max_obins = cfg->max_obins;
    h->max_inst = cfg->max_instances;
    h->max_blk = cfg->max_particles / kBlock + cfg->max_instances + 1;
    h->max_chunks = h->max_blk / kChunk + cfg->max_instances + 1;
    const size_t rs = cfg->precision == TPKMC_FP64 ? sizeof(double) : sizeof(float);
    const size_t inst_sz = cfg->precision == TPKMC_FP64 ? sizeof(Inst<double>) : sizeof(Inst<float>);
    const int64_t tiles = (cfg->max_cells + 1 + kScanTile - 1) / kScanTile + 1;
    int bad = 0;
    bad |= dalloc(&h->b.rank, h->max_n);
    bad |= dalloc(&h->b.start, h->max_cells + 1);
    bad |= dalloc(&h->b.tiles, tiles);
    bad |= dalloc(&h->b.src, h->max_n);
    bad |= dalloc(&h->b.best, h->max_n);
    bad |= dalloc(&h->b.perm, h->max_n);
    bad |= hipMalloc(&h->b.rec, rs * 8 * (size_t)std::max<int64_t>(h->max_n, 1)) != hipSuccess;
    bad |= hipMalloc(&h->b.rmass, rs * (size_t)std::max<int64_t>(h->max_n, 1)) != hipSuccess;
    bad |= hipMalloc(&h->b.inst, inst_sz * (size_t)h->max_inst) != hipSuccess;
    bad |= dalloc(&h->b.blk, h->max_blk);
    bad |= dalloc(&h->b.gpart, h->max_blk * kGPart);
    bad |= dalloc(&h->b.chunks, h->max_chunks);
    bad |= dalloc(&h->b.cpart, h->max_chunks * kGPart);
    if (cfg->precision == TPKMC_FP32) bad |= dalloc(&h->b.bkey, h->max_n);
    bad |= dalloc(&h->b.shift, 3 * std::max<int64_t>(h->max_obins, 1));
    bad |= dalloc(&h->b.macc, std::max<int64_t>(h->max_obins, 1));
    bad |= hipMalloc(&h->b.vir, rs * 3 * (size_t)std::max<int64_t>(h->max_n, 1)) != hipSuccess;
    bad |= dalloc(&h->b.coll, std::max<int64_t>(h->max_n, 1));
    bad |= dalloc(&h->b.pair_count, 1);
    bad |= dalloc(&h->b.mix, 3);
    bad |= dalloc(&h->b.status, 1);
    h->stage_bytes = inst_sz * (size_t)h->max_inst + sizeof(Blk) * (size_t)h->max_blk +
                     sizeof(Chunk) * (size_t)h->max_chunks;
    for (int k = 0; k < tpkmc_handle::kRing && !bad; ++k) {
        bad |= hipHostMalloc((void**)&h->stage[k], h->stage_bytes, hipHostMallocDefault) != hipSuccess;
        bad |= hipEventCreateWithFlags(&h->stage_ev[k], hipEventDisableTiming) != hipSuccess;
    }
    if (!bad) {
        bad |= hipMemset(h->b.shift, 0, sizeof(double) * 3 * (size_t)std::max<int64_t>(h->max_obins, 1)) != hipSuccess;
        bad |= hipMemset(h->b.status, 0, sizeof(uint32_t)) != hipSuccess;
        bad |= hipMemset(h->b.gpart, 0, sizeof(double) * kGPart * (size_t)h->max_blk) != hipSuccess;
        bad |= hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess;
        bad |= hipDeviceSynchronize() != hipSuccess;
    }
    if (bad) {
        free_all(h);
        if (h->own_stream) hipStreamDestroy(h->own_stream);
        delete h;
        hipGetLastError();
        return TPKMC_ENOMEM;
    }
    *out = h;
    return TPKMC_OK;
}

int tpkmc_destroy(tpkmc_handle* h) {
    if (!h) return TPKMC_OK;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    for (hipEvent_t e : h->pool) hipEventDestroy(e);
    free_all(h);
    if (h->own_stream) hipStreamDestroy(h->own_stream);
    delete h;
    return TPKMC_OK;
}

int tpkmc_step(tpkmc_handle* h, const tpkmc_grid* g, const tpkmc_params* p, const tpkmc_particles* s,
               const tpkmc_outputs* o, void* stream) {
    if (!h || !g || !p || !s) return TPKMC_EINVAL;
    tpkmc_instance one;
    one.offset = 0;
    one.count = s->n;
    one.grid = *g;
    one.params = *p;
    return tpkmc_step_batched(h, s, &one, 1, o, stream);
}

int tpkmc_step_noalloc(int32_t precision, int32_t device, const tpkmc_grid* g, const tpkmc_params* p,
                       const tpkmc_particles* s, const tpkmc_outputs* o, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (precision == TPKMC_FP64) return step_noalloc_impl<double>(device, g, p, s, o, st);
    if (precision == TPKMC_FP32) return step_noalloc_impl<float>(device, g, p, s, o, st);
    return TPKMC_EINVAL;
}

int tpkmc_step_batched(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* inst, int32_t n_inst,
                       const tpkmc_outputs* o, void* stream) {
    if (!h) return TPKMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return h->precision == TPKMC_FP64 ? step_impl<double>(h, s, inst, n_inst, o, st)
                                      : step_impl<float>(h, s, inst, n_inst, o, st);
}

int tpkmc_run(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* inst, int32_t n_inst,
              int32_t nsteps, const tpkmc_outputs* o, void* stream) {
    if (!h) return TPKMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return h->precision == TPKMC_FP64 ? run_impl<double>(h, s, inst, n_inst, nsteps, o, st)
                                      : run_impl<float>(h, s, inst, n_inst, nsteps, o, st);
}

int tpkmc_autotune(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* inst, int32_t n_inst,
                   void* stream) {
    if (!h) return TPKMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return h->precision == TPKMC_FP64 ? tune_impl<double>(h, s, inst, n_inst, st)
                                      : tune_impl<float>(h, s, inst, n_inst, st);
}

int tpkmc_search_order(tpkmc_handle* h, int32_t* order) {
    if (!h || !order) return TPKMC_EINVAL;
    *order = h->search_order;
    return TPKMC_OK;
}

int tpkmc_set_search_order(tpkmc_handle* h, int32_t order) {
    if (!h || order < 0 || order > 4096) return TPKMC_EINVAL;
    h->search_order = order;
    return TPKMC_OK;
}

int tpkmc_tuned_cells(tpkmc_handle* h, int32_t k, int32_t ncell[3]) {
    if (!h || !ncell || k < 0 || k >= (int32_t)h->cells.size()) return TPKMC_EINVAL;
    for (int a = 0; a < 3; ++a) ncell[a] = h->cells[k].n[a];
    return TPKMC_OK;
}

int tpkmc_tuned_speed(tpkmc_handle* h, int32_t k, double* speed) {
    if (!h || !speed || k < 0 || k >= (int32_t)h->cells.size()) return TPKMC_EINVAL;
    *speed = h->cells[k].vc;
    return TPKMC_OK;
}

int tpkmc_search_mix(tpkmc_handle* h, const tpkmc_particles* s, const tpkmc_instance* inst, int32_t n_inst,
                     uint64_t* counts, void* stream) {
    if (!h) return TPKMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return h->precision == TPKMC_FP64 ? mix_impl<double>(h, s, inst, n_inst, counts, st)
                                      : mix_impl<float>(h, s, inst, n_inst, counts, st);
}

int tpkmc_set_search(tpkmc_handle* h, int32_t group, int32_t block) {
    if (!h) return TPKMC_EINVAL;
    if (block != 64 && block != 128 && block != 256) return TPKMC_EINVAL;
    if (group != 1 && group != 2 && group != 4) return TPKMC_EINVAL;
    if (block > kBlock / group) return TPKMC_EINVAL;
    h->search_group = group;
    h->search_block = block;
    h->search_order = kDefaultSearchOrder;
    h->shape_chosen = true;
    return TPKMC_OK;
}

int tpkmc_get_search(tpkmc_handle* h, int32_t* group, int32_t* block) {
    if (!h || !group || !block) return TPKMC_EINVAL;
    *group = h->search_group;
    *block = h->search_block;
    return TPKMC_OK;
}

int tpkmc_status(tpkmc_handle* h, int32_t* device_status) {
    if (!h || !device_status) return TPKMC_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    if (hipStreamSynchronize(h->last_stream) != hipSuccess) return TPKMC_EHIP;
    uint32_t v = 0;
    if (hipMemcpy(&v, h->b.status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return TPKMC_EHIP;
    if (hipMemset(h->b.status, 0, sizeof(v)) != hipSuccess) return TPKMC_EHIP;
    *device_status = (int32_t)v;
    return TPKMC_OK;
}

int tpkmc_profile_enable(tpkmc_handle* h, int32_t on) {
    if (!h) return TPKMC_EINVAL;
    h->profiling = on != 0;
    return TPKMC_OK;
}

int tpkmc_profile_read(tpkmc_handle* h, double* ms, int64_t* launches, int32_t n) {
    if (!h || n < 0 || (n > 0 && (!ms || !launches))) return TPKMC_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return TPKMC_EHIP;
    if (!h->prof.empty()) {
        if (hipEventSynchronize(h->prof.back().b) != hipSuccess) return TPKMC_EHIP;
        for (const ProfRec& r : h->prof) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && r.phase >= 0 && r.phase < kPhases) {
                h->prof_ms[r.phase] += t;
                h->prof_n[r.phase] += 1;
            }
        }
        h->prof.clear();
        h->pool_used = 0;
    }
    for (int k = 0; k < n; ++k) {
        ms[k] = k < kPhases ? h->prof_ms[k] : 0.0;
        launches[k] = k < kPhases ? h->prof_n[k] : 0;
    }
    for (int k = 0; k < kPhases; ++k) { h->prof_ms[k] = 0.0; h->prof_n[k] = 0; }
    return TPKMC_OK;
}

}  // extern "C"
