// Device kernels of the collision step, templated on the precision of the
// particle state (float or double).  Included by tpkmc_f32.hip and
// tpkmc_f64.hip; the FP64 unit is compiled without FMA contraction so that
// every expression below rounds exactly like the plain C reference.
//
// Work layout.  Every per-particle kernel runs over a block table: each
// work-group owns kBlock consecutive particles of ONE instance, so a batch of
// independent instances is one launch and per-work-group partial sums belong
// to one instance.  Particles are bucketed by c-bin with a counting sort
// (key -> prefix -> scatter) into 8-real records; because the c-bin index is
// x-fastest, the three c-bins of one x-row of a neighbourhood are contiguous
// records, so the 27-cell neighbourhood is at most 9 (18 with a periodic
// x-seam) contiguous record ranges.
#pragma once

#include <type_traits>

#include "tpkmc_internal.h"

namespace tpkmc {

// ---------------------------------------------------------------- records
// Record layout: x y z id | vx vy vz flags (8 reals).  flags bit 0 = alive.
template <typename real> struct Rec;

template <> struct Rec<float> {
    // Position and velocity of record i through a 32-bit byte offset (the
    // host keeps 32 * records below 2^32).
    static __device__ __forceinline__ void load6(const float* r, uint32_t i, float& x, float& y, float& z,
                                                 float& vx, float& vy, float& vz) {
        const char* b = reinterpret_cast<const char*>(r) + i * 32u;
        const float4 a = *reinterpret_cast<const float4*>(b);
        const float4 c = *reinterpret_cast<const float4*>(b + 16);
        x = a.x; y = a.y; z = a.z; vx = c.x; vy = c.y; vz = c.z;
    }
    static __device__ __forceinline__ float from_u32(uint32_t v) { return __uint_as_float(v); }
    static __device__ __forceinline__ uint32_t to_u32(float v) { return __float_as_uint(v); }
    static __device__ __forceinline__ void store(float* r, int64_t i, float x, float y, float z, uint32_t id,
                                                 float vx, float vy, float vz, uint32_t fl) {
        float4* p = reinterpret_cast<float4*>(r + 8 * i);
        p[0] = make_float4(x, y, z, from_u32(id));
        p[1] = make_float4(vx, vy, vz, from_u32(fl));
    }
    static __device__ __forceinline__ void load(const float* r, int64_t i, float& x, float& y, float& z,
                                                uint32_t& id, float& vx, float& vy, float& vz, uint32_t& fl) {
        const float4* p = reinterpret_cast<const float4*>(r + 8 * i);
        float4 a = p[0], b = p[1];
        x = a.x; y = a.y; z = a.z; id = to_u32(a.w);
        vx = b.x; vy = b.y; vz = b.z; fl = to_u32(b.w);
    }
};

template <> struct Rec<double> {
    static __device__ __forceinline__ double from_u32(uint32_t v) { return __longlong_as_double((long long)v); }
    static __device__ __forceinline__ uint32_t to_u32(double v) { return (uint32_t)__double_as_longlong(v); }
    static __device__ __forceinline__ void store(double* r, int64_t i, double x, double y, double z, uint32_t id,
                                                 double vx, double vy, double vz, uint32_t fl) {
        double2* p = reinterpret_cast<double2*>(r + 8 * i);
        p[0] = make_double2(x, y);
        p[1] = make_double2(z, from_u32(id));
        p[2] = make_double2(vx, vy);
        p[3] = make_double2(vz, from_u32(fl));
    }
    static __device__ __forceinline__ void load(const double* r, int64_t i, double& x, double& y, double& z,
                                                uint32_t& id, double& vx, double& vy, double& vz, uint32_t& fl) {
        const double2* p = reinterpret_cast<const double2*>(r + 8 * i);
        double2 a = p[0], b = p[1], c = p[2], d = p[3];
        x = a.x; y = a.y; z = b.x; id = to_u32(b.y);
        vx = c.x; vy = c.y; vz = d.x; fl = to_u32(d.y);
    }
};

// Loads of a record whose index is the same in every lane of the wave: through
// the constant address space the compiler issues scalar loads (one per wave,
// into SGPRs); the records are never written while the search runs.
template <typename real> struct RecU;
template <typename real> struct RecU {
    typedef __attribute__((address_space(4))) const real cr;
    static __device__ __forceinline__ void load(const real* r, int32_t i, real& x, real& y, real& z, uint32_t& id,
                                                real& vx, real& vy, real& vz) {
        const cr* p = (const cr*)(r) + 8 * (int64_t)i;
        x = p[0]; y = p[1]; z = p[2];
        id = Rec<real>::to_u32(p[3]);
        vx = p[4]; vy = p[5]; vz = p[6];
    }
};

// ---------------------------------------------------------------- helpers
// Bin along one axis: floor((x - lo) * n / L) clamped into [0, n - 1].
template <typename real>
__device__ __forceinline__ int axis_bin(real x, real lo, real inv_w, int n) {
    real t = (x - lo) * inv_w;
    if (!(t >= real(0))) return 0;
    if (t >= real(n)) return n - 1;
    return (int)t;
}

// Row (y, z) of c-bins as its index in the c-bin order, in units of rows
// (the c-bin index is x + n_x * row).  The order is band-major: the y axis is
// cut into bands of 2^band_log2 rows, and within a band the rows run z-major.
// A sweep over consecutive c-bins (one XCD's share of the work-groups) thus
// stays inside one band while it walks through the planes.  The records of the
// next plane, which the neighbourhood walk reads again one plane later, are
// then a band plane away instead of a whole plane.  With one band this is the
// plain y + n_y z.
template <typename real>
__device__ __forceinline__ int row_of(const Inst<real>& I, int y, int z) {
    const int h = I.band_log2;
    const int y0 = (y >> h) << h;                 // first row of y's band
    const int rows = min(1 << h, I.n[1] - y0);    // rows in that band
    return y0 * I.n[2] + (y - y0) + rows * z;
}

template <typename real>
__device__ __forceinline__ bool finite3(real a, real b, real c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ __forceinline__ uint64_t lanes_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Cross-lane moves of a double through the VALU's data-parallel primitives
// (DPP) instead of the LDS permute unit; every lane of the wave must be
// active.  Quad permutations: lane q of each group of four reads lane P[q]
// of its group, encoded P[0] | P[1] << 2 | P[2] << 4 | P[3] << 6.  Row
// shifts (0x100 + n): lane r of each row of 16 lanes reads lane r + n of
// the row (lanes past the row's end read nothing defined and must not use
// the value).  Row rotations (0x120 + n) rotate each row by n.
constexpr int kQuadXor1 = 1 | 0 << 2 | 3 << 4 | 2 << 6;
constexpr int kQuadXor2 = 2 | 3 << 2 | 0 << 4 | 1 << 6;
constexpr int kRowShl1 = 0x101;
constexpr int kRowShl2 = 0x102;
constexpr int kRowShl4 = 0x104;
constexpr int kRowShl8 = 0x108;
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum (or maximum) of a double over the 64 lanes, in a fixed order: pairs,
// quads and rows through DPP, then the four row totals.  Every lane must be
// active; the result is returned in every lane.
template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v) {
    auto op = [](double x, double y) { return MAX ? fmax(x, y) : x + y; };
    v = op(v, dpp_move<kQuadXor1>(v));
    v = op(v, dpp_move<kQuadXor2>(v));
    v = op(v, dpp_move<kRowRor4>(v));
    v = op(v, dpp_move<kRowRor8>(v));
    return op(op(lane_value(v, 0), lane_value(v, 16)), op(lane_value(v, 32), lane_value(v, 48)));
}

// Sum of a double over the work-group (blockDim.x <= 1024), result in all threads.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += lds[k];
    return t;
}

__device__ __forceinline__ double block_max(double v, double* lds) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = lds[0];
    for (int k = 1; k < nw; ++k) t = fmax(t, lds[k]);
    return t;
}

// Sums (max for index kmax) of N values over the work-group in one LDS pass;
// the totals land in v[] of thread 0.  lds holds 16 * N doubles.
template <int N>
__device__ __forceinline__ void block_reduce(double v[N], int kmax, double* lds) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(v[k], o);
            v[k] = k == kmax ? fmax(v[k], u) : v[k] + u;
        }
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[w * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 1; q < nw; ++q)
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = k == kmax ? fmax(v[k], lds[q * N + k]) : v[k] + lds[q * N + k];
}

// Work-groups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD (own L2) receives a contiguous range of the table, where neighbouring
// work-groups share neighbour c-bins.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int nx = 8;
    const int xcd = bid % nx, local = bid / nx;
    const int per = nb / nx, rem = nb % nx;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// The other order: chunks of S consecutive work-groups dealt round-robin over
// the XCDs (S = 1 keeps the dispatch order).  Contiguous ranges keep what
// neighbouring work-groups share in one L2, but when the work per
// work-group varies along the table (a batch of instances of different
// densities) they leave some XCDs with much more work than others; chunks
// trade some of that locality for balance.  Full rounds of 8 S work-groups
// are permuted; the last, partial round keeps the dispatch order.
__device__ __forceinline__ int xcd_chunk_remap(int bid, int nb, int S) {
    const int round = 8 * S;
    const int r = bid / round, m = bid - r * round;
    if ((r + 1) * round > nb) return bid;
    return r * round + (m & 7) * S + (m >> 3);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Isotropic unit vector of the pair (idA < idB) from a point (x1, x2) drawn
// uniformly in the unit disk by rejection, two 53-bit uniforms per Philox
// draw (at most 255 draws: the counter ending in 255 is kept for the random
// partners' draws); computed in double in both precisions.  In space: Marsaglia's map
// (2 x1 q, 2 x2 q, 1 - 2 s), q = sqrt(1 - s).  In the plane: the doubled
// angle ((x1^2 - x2^2) / s, 2 x1 x2 / s, 0), which needs s > 0.
__device__ __forceinline__ void pair_direction(uint32_t k0, uint32_t k1, uint32_t step, uint32_t instance,
                                               uint32_t idA, uint32_t idB, bool planar, double n[3]) {
    for (uint32_t attempt = 0; attempt < 255u; ++attempt) {
        uint32_t c[4] = {step, idA, idB, (instance << 8) | attempt};
        philox4x32_10(c, k0, k1);
        const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
        const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * (1.0 / 9007199254740992.0);
        const double x1 = 2.0 * u1 - 1.0;
        const double x2 = 2.0 * u2 - 1.0;
        const double s = x1 * x1 + x2 * x2;
        if (planar) {
            if (s < 1.0 && s > 0.0) {
                n[0] = (x1 * x1 - x2 * x2) / s;
                n[1] = (2.0 * x1 * x2) / s;
                n[2] = 0.0;
                return;
            }
        } else if (s < 1.0) {
            const double q = sqrt(1.0 - s);
            n[0] = (2.0 * x1) * q;
            n[1] = (2.0 * x2) * q;
            n[2] = 1.0 - 2.0 * s;
            return;
        }
    }
    n[0] = planar ? 1.0 : 0.0; n[1] = 0.0; n[2] = planar ? 0.0 : 1.0;
}

// |v|^2 in double, summed in axis order with every product rounded (the
// order the time-step rule and the global maximum are defined in).
__device__ __forceinline__ double speed2(double vx, double vy, double vz) {
#pragma clang fp contract(off)
    return (vx * vx + vy * vy) + vz * vz;
}

// ---------------------------------------------------------------- 1. key
// |v|^2 in the state's precision with fixed fused operations, so that the key
// and scatter kernels class a particle as slow or fast alike.
template <typename real>
__device__ __forceinline__ real speed2_r(real vx, real vy, real vz) {
    return fma(vz, vz, fma(vy, vy, vx * vx));
}

// c-bin key of caller-order particle p: its c-bin, or the instance's trailing
// bin for a dead or non-finite particle.  With split c-bins a fast particle
// (|v|^2 above the instance's bound) takes its configured c-bin, numbered
// after the slow particles' refined ones.  The key and scatter kernels both
// evaluate it on the same loaded values, so the key is never stored.
template <typename real>
__device__ __forceinline__ int cbin_key(const StepArgs<real>& a, const Inst<real>& I, int64_t p, real x, real y,
                                        real z, real vx, real vy, real vz, bool alive, bool& fin) {
    fin = finite3(x, y, z) && finite3(vx, vy, vz);
    if (a.mass) {
        const real m = a.mass[p];
        fin = fin && m > real(0) && m < real(INFINITY);
    }
    if (!(alive && fin)) return (int)(I.cell_off + I.C);
    if ((I.flags & kSplit) && !(speed2_r(vx, vy, vz) <= I.vc2)) {
        const int cx = axis_bin(x, I.lo[0], I.inv_wc[0], I.ncfg[0]);
        const int cy = axis_bin(y, I.lo[1], I.inv_wc[1], I.ncfg[1]);
        const int cz = axis_bin(z, I.lo[2], I.inv_wc[2], I.ncfg[2]);
        return (int)I.cell_off + I.Cf + cx + I.ncfg[0] * (cy + I.ncfg[1] * cz);
    }
    const int cx = axis_bin(x, I.lo[0], I.inv_w[0], I.n[0]);
    const int cy = axis_bin(y, I.lo[1], I.inv_w[1], I.n[1]);
    const int cz = axis_bin(z, I.lo[2], I.inv_w[2], I.n[2]);
    return (int)I.cell_off + cx + I.n[0] * row_of(I, cy, cz);
}

// The key kernel runs one wave per block-table entry, each lane taking
// kKeyRec particles kWave apart, so that every lane has all its loads, and
// then all its atomics, in flight at once.  With dense c-bins (long runs,
// few atomics) the kernel is otherwise bound by the latency of those two
// dependent steps: measured 1.07 -> 0.50 ms on the 4M-particle Sod tube and
// 0.18 -> 0.10 ms on the 8M Noh implosion; the sparse 16M Sedov blast, bound
// by the throughput of its one atomic per c-bin, is unchanged.  The same
// layout made the scatter kernel slower on the Sedov blast (0.226 -> 0.247 ms),
// so that one keeps a particle per lane.
constexpr int kKeyRec = kBlock / kWave;

// c-bin count of every caller-order particle and its rank inside the c-bin.
// Consecutive particles of the same c-bin (the common case for sorted input)
// take one atomic for the whole run, also across the wave's rounds.
template <typename real>
__global__ void __launch_bounds__(kWave) k_key(StepArgs<real> a) {
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int lane = threadIdx.x;
    const int64_t end = I.off + I.cnt;
    const bool want_v2 = (I.flags & (TPKMC_ADAPTIVE_DT | kSplit)) != 0;
    real x[kKeyRec], y[kKeyRec], z[kKeyRec], vx[kKeyRec], vy[kKeyRec], vz[kKeyRec];
    bool alive[kKeyRec];
#pragma unroll
    for (int r = 0; r < kKeyRec; ++r) {
        const int64_t p = (int64_t)bt.first + r * kWave + lane;
        x[r] = y[r] = z[r] = vx[r] = vy[r] = vz[r] = real(0);
        alive[r] = false;
        if (p < end) {
            alive[r] = a.alive ? a.alive[p] != 0 : true;
            x[r] = a.x[p]; y[r] = a.y[p]; z[r] = a.z[p];
            vx[r] = a.vx[p]; vy[r] = a.vy[p]; vz[r] = a.vz[p];
        }
    }
    // The wave's kKeyRec * 64 particles in caller order, q = r * 64 + lane,
    // fall into runs of one c-bin (in c-bin order after the first step, one
    // run per c-bin and wave); a run may span rounds.  Its first particle
    // takes one atomic for the whole run.
    int key[kKeyRec], base[kKeyRec];
    uint64_t heads[kKeyRec];
    double nonfin = 0.0, v2 = 0.0;
    int carry = -1;  // key of the previous round's last lane (keys are >= 0)
#pragma unroll
    for (int r = 0; r < kKeyRec; ++r) {
        const int64_t p = (int64_t)bt.first + r * kWave + lane;
        const bool in = p < end;
        bool fin = true;
        key[r] = in ? cbin_key(a, I, p, x[r], y[r], z[r], vx[r], vy[r], vz[r], alive[r], fin) : 0;
        if (in && alive[r] && fin) {
            if (want_v2) v2 = fmax(v2, speed2((double)vx[r], (double)vy[r], (double)vz[r]));
        } else if (in) {
            nonfin += (alive[r] && !fin) ? 1.0 : 0.0;
        }
        int prev = __shfl_up(key[r], 1);
        if (lane == 0) prev = carry;
        heads[r] = __ballot(in && prev != key[r]);
        carry = __builtin_amdgcn_readlane(key[r], kWave - 1);
    }
    const int nvalid = (int)min<int64_t>(end - (int64_t)bt.first, (int64_t)kKeyRec * kWave);
    int hq[kKeyRec];  // linear index of the run head of each of the lane's particles
#pragma unroll
    for (int r = 0; r < kKeyRec; ++r) {
        const int q = r * kWave + lane;
        const uint64_t below = heads[r] & lanes_le(lane);
        int h = below ? r * kWave + 63 - __clzll((long long)below) : 0;
        if (!below)
            for (int rr = r - 1; rr >= 0; --rr)
                if (heads[rr]) { h = rr * kWave + 63 - __clzll((long long)heads[rr]); break; }
        hq[r] = h;
        base[r] = 0;
        if (q < nvalid && h == q) {
            const uint64_t above = heads[r] & ~lanes_le(lane);
            int nq = above ? r * kWave + __ffsll((long long)above) - 1 : nvalid;
            if (!above)
                for (int rr = r + 1; rr < kKeyRec; ++rr)
                    if (heads[rr]) { nq = min(nvalid, rr * kWave + __ffsll((long long)heads[rr]) - 1); break; }
            base[r] = atomicAdd(&a.start[key[r]], nq - q);
        }
    }
#pragma unroll
    for (int r = 0; r < kKeyRec; ++r) {
        const int q = r * kWave + lane;
        const int hr = hq[r] / kWave, hl = hq[r] % kWave;
        int b = 0;
#pragma unroll
        for (int rr = 0; rr <= r; ++rr) {
            const int t = __shfl(base[rr], hl);
            if (rr == hr) b = t;
        }
        if (q < nvalid) a.rank[(int64_t)bt.first + q] = b + (q - hq[r]);
    }
    nonfin = wave_reduce<false>(nonfin);
    v2 = wave_reduce<true>(v2);
    if (lane == 0) {
        double* gp = a.gpart + (int64_t)blockIdx.x * kGPart;
        gp[GP_NONFINITE] = nonfin;
        gp[GP_VMAX0] = v2;
        gp[GP_FAST] = 0.0;  // counted by the scatter kernel, once dt is known
        // The search kernel may accumulate into these with atomics.
        gp[GP_TESTS2] = 0.0;
        gp[GP_CAND] = 0.0;
    }
}

// ---------------------------------------------------------------- 3. scatter
// Caller-order particle -> its c-bin-ordered record.  The permutation back to
// the caller's order is kept only when the state is written back in that
// order (without TPKMC_ALLOW_REORDER).
template <typename real>
__global__ void __launch_bounds__(kBlock) k_scatter(StepArgs<real> a) {
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t p = (int64_t)bt.first + threadIdx.x;
    bool fast = false;
    if (p < I.off + I.cnt) {
        const int64_t base = I.off - a.start[I.cell_off];
        const bool alive = a.alive ? a.alive[p] != 0 : true;
        const real x = a.x[p], y = a.y[p], z = a.z[p], vx = a.vx[p], vy = a.vy[p], vz = a.vz[p];
        bool fin;
        const int k = cbin_key(a, I, p, x, y, z, vx, vy, vz, alive, fin);
        const int64_t dst = base + a.start[k] + a.rank[p];
        const uint32_t fl = alive ? 1u : 0u;
        Rec<real>::store(a.rec, dst, x, y, z, a.id[p], vx, vy, vz, fl);
        if (!(I.flags & TPKMC_ALLOW_REORDER)) a.src[dst] = (int32_t)p;
        if (a.bkey) a.bkey[dst] = ~0ull;
        if (a.mass) a.rmass[dst] = a.mass[p];
        // Diagnostic: a particle faster than one c-bin per step on some axis.
        const real dt = I.dt;
        fast = alive && fin &&
               (fabs(vx) * dt > I.w[0] || fabs(vy) * dt > I.w[1] || fabs(vz) * dt > I.w[2]);
    }
    const uint64_t fm = __ballot(fast);
    if (fm && (threadIdx.x & 63) == __ffsll((long long)fm) - 1)
        atomicAdd(a.gpart + (int64_t)blockIdx.x * kGPart + GP_FAST, (double)__popcll(fm));
}

// ---------------------------------------------------------------- 4. search
// Per-instance constants of the pair test, held in registers.
template <typename real>
struct Geo {
    real L[3], halfL[3], invL[3];
    real dt, D2;
    bool per[3];
    __device__ __forceinline__ explicit Geo(const Inst<real>& I) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[a] = I.L[a];
            halfL[a] = I.halfL[a];
            invL[a] = real(1) / I.L[a];
            per[a] = I.bc[a] == TPKMC_BC_PERIODIC;
        }
        dt = I.dt;
        D2 = I.D2;
    }
};

// Minimum image on a periodic axis, written as selects (same value as the
// reference's if / else-if).
template <typename real>
__device__ __forceinline__ real min_image(real r, real L, real halfL) {
    const real up = r - L, dn = r + L;
    return r > halfL ? up : (r < -halfL ? dn : r);
}

// The three criteria for the ordered pair (i, j): chi < 0 within the step
// (s0 = r.u < 0 < s1 = r.u + |u|^2 dt), then d_min^2 <= D^2.  Returns d_min^2,
// or -1 when j is not a candidate.  j == i (or an exact twin) has r.u = 0 and
// is rejected by the first criterion.
//
// Most pairs fail, and a branch taken by any lane of a wave costs the whole
// wave, so the rejection is decided without branches and without a division:
// d_min^2 |u|^2 = |r x u|^2, hence d_min^2 <= D^2  <=>  |r x u|^2 <= D^2 |u|^2.
//  - FP32: that form decides; d_min^2 = |r x u|^2 / |u|^2 only for candidates.
//  - FP64: that form, with FMAs and a margin far above the rounding of either
//    form, only discards pairs that are certainly not candidates; the rest go
//    through the reference's own expressions (t_poca = -s0/|u|^2, PoCA
//    separation r + t_poca u), so decisions and d_min^2 are bit-identical.
template <typename real, int PM>
__device__ __forceinline__ void rel_vectors(const Geo<real>& G, real xi, real yi, real zi, real vxi, real vyi,
                                            real vzi, real xj, real yj, real zj, real vxj, real vyj, real vzj,
                                            real& rx, real& ry, real& rz, real& ux, real& uy, real& uz) {
    rx = xi - xj; ry = yi - yj; rz = zi - zj;
    if constexpr (PM < 0) {
        if (G.per[0]) rx = min_image(rx, G.L[0], G.halfL[0]);
        if (G.per[1]) ry = min_image(ry, G.L[1], G.halfL[1]);
        if (G.per[2]) rz = min_image(rz, G.L[2], G.halfL[2]);
    } else {
        if constexpr ((PM & 1) != 0) rx = min_image(rx, G.L[0], G.halfL[0]);
        if constexpr ((PM & 2) != 0) ry = min_image(ry, G.L[1], G.halfL[1]);
        if constexpr ((PM & 4) != 0) rz = min_image(rz, G.L[2], G.halfL[2]);
    }
    ux = vxi - vxj; uy = vyi - vyj; uz = vzi - vzj;
}

// Two-stage screening, both stages without divergent branches:
//  stage 1, criterion 1 (s0 < 0 < s1), on every pair;
//  stage 2, |r x u|^2 <= D^2 |u|^2, only when some lane of the wave passed
//  stage 1 (a wave-uniform branch, so cold regions where no pair of the wave
//  meets within the step skip it).
template <typename real> struct Screen {
    real rx, ry, rz, ux, uy, uz, s0, vv;
};

// PM: the periodic axes as a mask known at compile time (bit a for axis a),
// or -1 to read them from the instance at run time.
template <typename real, int PM> struct PairTest;

template <int PM> struct PairTest<float, PM> {
    static __device__ __forceinline__ bool stage1(const Geo<float>& G, float xi, float yi, float zi, float vxi,
                                                  float vyi, float vzi, float xj, float yj, float zj, float vxj,
                                                  float vyj, float vzj, Screen<float>& S) {
        float rx = xi - xj, ry = yi - yj, rz = zi - zj;
        // Nearest image: r - L rint(r / L) (ties at exactly L/2 keep r).
        if constexpr (PM < 0) {
            if (G.per[0]) rx = fmaf(-G.L[0], rintf(rx * G.invL[0]), rx);
            if (G.per[1]) ry = fmaf(-G.L[1], rintf(ry * G.invL[1]), ry);
            if (G.per[2]) rz = fmaf(-G.L[2], rintf(rz * G.invL[2]), rz);
        } else {
            if constexpr ((PM & 1) != 0) rx = fmaf(-G.L[0], rintf(rx * G.invL[0]), rx);
            if constexpr ((PM & 2) != 0) ry = fmaf(-G.L[1], rintf(ry * G.invL[1]), ry);
            if constexpr ((PM & 4) != 0) rz = fmaf(-G.L[2], rintf(rz * G.invL[2]), rz);
        }
        const float ux = vxi - vxj, uy = vyi - vyj, uz = vzi - vzj;
        const float s0 = fmaf(rz, uz, fmaf(ry, uy, rx * ux));
        const float vv = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
        const float s1 = fmaf(vv, G.dt, s0);
        S.rx = rx; S.ry = ry; S.rz = rz; S.ux = ux; S.uy = uy; S.uz = uz; S.s0 = s0; S.vv = vv;
        return (s0 < 0.0f) & (s1 > 0.0f);
    }
    static __device__ __forceinline__ bool stage2(const Geo<float>& G, const Screen<float>& S) {
        const float cx = fmaf(S.ry, S.uz, -S.rz * S.uy);
        const float cy = fmaf(S.rz, S.ux, -S.rx * S.uz);
        const float cz = fmaf(S.rx, S.uy, -S.ry * S.ux);
        const float c2 = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
        return c2 <= G.D2 * S.vv;
    }
    // d_min^2 of a pair that passed both stages (always a candidate in FP32).
    static __device__ __forceinline__ float finish(const Geo<float>&, const Screen<float>& S) {
        const float cx = fmaf(S.ry, S.uz, -S.rz * S.uy);
        const float cy = fmaf(S.rz, S.ux, -S.rx * S.uz);
        const float cz = fmaf(S.rx, S.uy, -S.ry * S.ux);
        return fmaf(cz, cz, fmaf(cy, cy, cx * cx)) / S.vv;
    }
    // First contact of the effective radii: the earlier root of
    // |u|^2 t^2 + 2 (u.r) t + |r|^2 - D^2 = 0 (a rounding below zero of the
    // discriminant is taken as 0).
    static __device__ __forceinline__ float contact(const Geo<float>& G, const Screen<float>& S) {
        const float rr = fmaf(S.rz, S.rz, fmaf(S.ry, S.ry, S.rx * S.rx));
        float disc = fmaf(S.s0, S.s0, -S.vv * (rr - G.D2));
        disc = disc > 0.0f ? disc : 0.0f;
        return (-S.s0 - sqrtf(disc)) / S.vv;
    }
};

template <int PM> struct PairTest<double, PM> {
    static __device__ __forceinline__ bool stage1(const Geo<double>& G, double xi, double yi, double zi, double vxi,
                                                  double vyi, double vzi, double xj, double yj, double zj, double vxj,
                                                  double vyj, double vzj, Screen<double>& S) {
        double rx, ry, rz, ux, uy, uz;
        rel_vectors<double, PM>(G, xi, yi, zi, vxi, vyi, vzi, xj, yj, zj, vxj, vyj, vzj, rx, ry, rz, ux, uy, uz);
        // Exactly the reference's s0 and s1 (no contraction in this unit).
        const double s0 = (rx * ux + ry * uy) + rz * uz;
        const double vv = (ux * ux + uy * uy) + uz * uz;
        const double s1 = s0 + vv * G.dt;
        S.rx = rx; S.ry = ry; S.rz = rz; S.ux = ux; S.uy = uy; S.uz = uz; S.s0 = s0; S.vv = vv;
        return (s0 < 0.0) & (s1 > 0.0);
    }
    // Conservative: |r x u|^2 <= D^2 |u|^2 with a margin far above the
    // rounding of either form, so no pair the reference accepts is lost.
    static __device__ __forceinline__ bool stage2(const Geo<double>& G, const Screen<double>& S) {
        const double cx = fma(S.ry, S.uz, -S.rz * S.uy);
        const double cy = fma(S.rz, S.ux, -S.rx * S.uz);
        const double cz = fma(S.rx, S.uy, -S.ry * S.ux);
        const double c2 = fma(cz, cz, fma(cy, cy, cx * cx));
        const double rr = fma(S.rz, S.rz, fma(S.ry, S.ry, S.rx * S.rx));
        return c2 <= fma(G.D2 * S.vv, 1.0 + 1e-6, 1e-12 * rr * S.vv);
    }
    // The reference's expressions; -1 when the exact d_min^2 exceeds D^2.
    static __device__ __forceinline__ double finish(const Geo<double>& G, const Screen<double>& S) {
        const double tp = -S.s0 / S.vv;
        const double px = S.rx + tp * S.ux, py = S.ry + tp * S.uy, pz = S.rz + tp * S.uz;
        const double d2 = (px * px + py * py) + pz * pz;
        return d2 <= G.D2 ? d2 : -1.0;
    }
    // First contact time, with the reference's expression and order.
    static __device__ __forceinline__ double contact(const Geo<double>& G, const Screen<double>& S) {
        const double rr = (S.rx * S.rx + S.ry * S.ry) + S.rz * S.rz;
        double disc = S.s0 * S.s0 - S.vv * (rr - G.D2);
        if (!(disc > 0.0)) disc = 0.0;
        return (-S.s0 - sqrt(disc)) / S.vv;
    }
};

// Order-preserving map of a float onto uint32 (negative values included).
__device__ __forceinline__ uint32_t sortable(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Neighbour index along one axis (offset d in -1..1): whether it exists and
// is not a repeat of another offset (periodic axes with 1 or 2 bins), and the
// wrapped index.
__device__ __forceinline__ bool axis_nb(int c, int d, int n, bool periodic, int& out) {
    int v = c + d;
    if (periodic) {
        if (n == 1 && d != 0) return false;
        if (n == 2 && d == 1) return false;
        v = v < 0 ? v + n : (v >= n ? v - n : v);
    } else if (v < 0 || v >= n) {
        return false;
    }
    out = v;
    return true;
}

// x-extent of the neighbourhood as at most two contiguous bin ranges; the
// first always contains cx.
__device__ __forceinline__ int x_ranges(int cx, int n, bool periodic, int xa[2], int xb[2]) {
    if (periodic && n > 3 && cx == 0) { xa[0] = 0; xb[0] = 1; xa[1] = n - 1; xb[1] = n - 1; return 2; }
    if (periodic && n > 3 && cx == n - 1) { xa[0] = n - 2; xb[0] = n - 1; xa[1] = 0; xb[1] = 0; return 2; }
    if (periodic && n <= 3) { xa[0] = 0; xb[0] = n - 1; return 1; }
    xa[0] = cx > 0 ? cx - 1 : 0;
    xb[0] = cx < n - 1 ? cx + 1 : n - 1;
    return 1;
}

template <typename real>
__device__ __forceinline__ int x_lo_of(int32_t f, const StepArgs<real>& a, const Inst<real>& I, int n0, bool per0) {
    real x, y, z, vx, vy, vz;
    uint32_t id;
    RecU<real>::load(a.rec, f, x, y, z, id, vx, vy, vz);
    int xa[2], xb[2];
    x_ranges(axis_bin(x, I.lo[0], I.inv_w[0], I.n[0]), n0, per0, xa, xb);
    return xa[0];
}

template <typename real>
__device__ __forceinline__ int cy_of(real y, const Inst<real>& I) { return axis_bin(y, I.lo[1], I.inv_w[1], I.n[1]); }
template <typename real>
__device__ __forceinline__ int cz_of(real z, const Inst<real>& I) { return axis_bin(z, I.lo[2], I.inv_w[2], I.n[2]); }

// Visits the record ranges of the neighbourhood of record i (bin cx, cy, cz).
// HALF: only pairs (i, j) not visited from j's side -- bins of larger index
// and, in i's own bin, records after i -- so every unordered pair is met once.
// COARSE: the fast particles of split c-bins, on the configured c-bins n[]
// (rows y + n_y z after the slow particles' c-bins).
// One of the nine rows (k = 3 (dz + 1) + dy + 1) of that neighbourhood.
template <bool HALF, bool COARSE = false, typename real, typename F>
__device__ __forceinline__ void neighbourhood_row(const int32_t* start, const Inst<real>& I, int64_t base,
                                                  const int n[3], const bool per[3], int cx, int cy, int cz,
                                                  int32_t i, int k, F&& visit) {
    const int64_t cell_off = COARSE ? I.cell_off + I.Cf : I.cell_off;
    int y, z;
    if (!axis_nb(cz, k / 3 - 1, n[2], per[2], z)) return;
    if (!axis_nb(cy, k % 3 - 1, n[1], per[1], y)) return;
    const int own_row = COARSE ? cy + n[1] * cz : row_of(I, cy, cz);
    const int row_idx = COARSE ? y + n[1] * z : row_of(I, y, z);
    if (HALF && row_idx < own_row) return;
    const bool own = row_idx == own_row;
    int xa[2], xb[2];
    const int nxr = x_ranges(cx, n[0], per[0], xa, xb);
    const int64_t row = cell_off + (int64_t)n[0] * row_idx;
    for (int r = 0; r < nxr; ++r) {
        int32_t j0 = (int32_t)(base + start[row + xa[r]]);
        const int32_t j1 = (int32_t)(base + start[row + xb[r] + 1]);
        if (HALF && own) {
            if (r == 0) j0 = i + 1;           // range holding cx: after i
            else if (xa[r] < cx) continue;    // wrapped bins below cx
        }
        visit(j0, j1);
    }
}

template <bool HALF, bool COARSE = false, typename real, typename F>
__device__ __forceinline__ void for_neighbourhood(const int32_t* start, const Inst<real>& I, int64_t base,
                                                  const int n[3], const bool per[3], int cx, int cy, int cz,
                                                  int32_t i, F&& visit) {
    for (int k = 0; k < 9; ++k) neighbourhood_row<HALF, COARSE>(start, I, base, n, per, cx, cy, cz, i, k, visit);
}

// Records per chunk of a wave's staging buffer in LDS (the staged lane mode
// of the FP32 search, search_staged): kStageCap quads (x, y, z, vx), then
// kStageCap pairs (vy, vz) in 16-byte slots, so that one address serves
// both reads (the pair kStageCap slots further on) and the loop reads 24 B
// per neighbour at a 16-byte stride.  Measured on the 16M Sedov search:
// 1.34 ms reading two quads per neighbour, 1.27 with the pairs packed at an
// 8-byte stride (two addresses), 1.24 with quad and pair interleaved in
// 32-byte slots (one address, four times the LDS bank conflicts), 1.23
// with this layout.
constexpr int kStageCap = 128;
constexpr int kStageBytesPerWave = kStageCap * 32;
static_assert(kStageBytesPerWave % 16 == 0, "each wave's buffer starts on a quad");

// Closest-candidate search with register blocking: one lane owns up to G
// consecutive records and tests every neighbour record it loads against all
// of them, so a load serves up to G pair tests.  The lane walks the union of
// its records' neighbourhoods row by row; record k only takes the records in
// its own range of that row.  It serves the wave-uniform mode of both
// precisions and the lane mode of FP64; the FP32 lane mode is search_staged.
//
// HALF (FP32): every unordered pair is tested once -- bins of larger index
// and, in a record's own bin, the records after it -- and a candidate lowers
// both particles' 64-bit keys (d_min^2 bits, partner record) with atomicMin,
// which is order independent; exact ties of d_min^2 go to the lower record.
// Ordered (FP64): each record scans its whole neighbourhood and keeps the
// smallest d_min^2, ties to the lower id, with the reference's arithmetic, so
// the choice does not depend on the order of records inside a bin.
//
// MIX (a diagnostic build, never the timed one) also counts the pairs the
// step tests that approach (s0 < 0) and that meet criterion 1 (s0 < 0 < s1),
// which fix the pair test's arithmetic per pair.
template <typename real, bool HALF, int PM, int G, bool UNIFORM, bool MIX = false>
__device__ __forceinline__ void search_group(const StepArgs<real>& a, const Inst<real>& I, int64_t base,
                                             int32_t i0, int nrec, int32_t wave_first, int wave_ub,
                                             double& tests, double& cand, uint32_t& n_s0, uint32_t& n_c1) {
    const Geo<real> G_(I);
    const int n[3] = {I.n[0], I.n[1], I.n[2]};
    real xi[G], yi[G], zi[G], vxi[G], vyi[G], vzi[G];
    int cxk[G];
    int cy = 0, cz = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        uint32_t idk, flk;
        const int32_t ik = k < nrec ? i0 + k : i0;
        Rec<real>::load(a.rec, ik, xi[k], yi[k], zi[k], idk, vxi[k], vyi[k], vzi[k], flk);
        cxk[k] = axis_bin(xi[k], I.lo[0], I.inv_w[0], I.n[0]);
        if (k == 0) {
            cy = axis_bin(yi[0], I.lo[1], I.inv_w[1], I.n[1]);
            cz = axis_bin(zi[0], I.lo[2], I.inv_w[2], I.n[2]);
        }
    }
    if constexpr (UNIFORM) {
        // Same row for the whole wave (checked by the caller).
        cy = __builtin_amdgcn_readfirstlane(cy);
        cz = __builtin_amdgcn_readfirstlane(cz);
    }
    // The records share a row (y, z bins) and single x-ranges?  Otherwise
    // search them one at a time.
    bool joint = true;
    int xa[G], xb[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        int ta[2], tb[2];
        const int nr = x_ranges(cxk[k], n[0], G_.per[0], ta, tb);
        xa[k] = ta[0];
        xb[k] = tb[0];
        if (k < nrec) {
            joint &= nr == 1;
            if (k > 0) {
                joint &= axis_bin(yi[k], I.lo[1], I.inv_w[1], I.n[1]) == cy;
                joint &= axis_bin(zi[k], I.lo[2], I.inv_w[2], I.n[2]) == cz;
            }
        }
    }
    unsigned long long mine[G];
    int32_t bj[G];
    real bd2[G];
    uint32_t bid[G];
    int32_t seen = 0, nc = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) { mine[k] = ~0ull; bj[k] = -1; bd2[k] = real(0); bid[k] = 0; }

    // Bookkeeping of a pair that passed both screening stages (rare).  The
    // ranking key of criterion 3 is d_min^2, or with TPKMC_RANK_TIME the
    // first contact time.
    const bool by_time = (I.flags & TPKMC_RANK_TIME) != 0;
    auto hit = [&](int k, int32_t j, uint32_t idj, const Screen<real>& S) {
        const real d2 = PairTest<real, PM>::finish(G_, S);
        if (d2 >= real(0)) {
            ++nc;
            const real key = by_time ? PairTest<real, PM>::contact(G_, S) : d2;
            if constexpr (HALF) {
                const unsigned long long hi = (unsigned long long)sortable((float)key) << 32;
                atomicMin(a.bkey + j, hi | (uint32_t)(i0 + k));
                const unsigned long long kk = hi | (uint32_t)j;
                mine[k] = kk < mine[k] ? kk : mine[k];
            } else {
                if (bj[k] < 0 || key < bd2[k] || (key == bd2[k] && idj < bid[k])) {
                    bj[k] = j; bd2[k] = key; bid[k] = idj;
                }
            }
        }
    };
    // Tests record j (loaded) against the lane's records k with take[k] set.
    auto screen = [&](int32_t j, uint32_t idj, real xj, real yj, real zj, real vxj, real vyj, real vzj,
                      const bool take[G]) {
        Screen<real> S[G];
        bool p1[G];
        bool any1 = false;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            // Evaluated on every lane, masked afterwards: no branch.
            p1[k] = PairTest<real, PM>::stage1(G_, xi[k], yi[k], zi[k], vxi[k], vyi[k], vzi[k], xj, yj, zj, vxj,
                                                vyj, vzj, S[k]) & take[k];
            any1 |= p1[k];
            if constexpr (MIX) {
                n_s0 += (take[k] && S[k].s0 < real(0)) ? 1u : 0u;
                n_c1 += p1[k] ? 1u : 0u;
            }
        }
        if (__builtin_amdgcn_ballot_w64(any1) == 0) return;
        bool p2[G];
        bool any2 = false;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            p2[k] = p1[k] && PairTest<real, PM>::stage2(G_, S[k]);
            any2 |= p2[k];
        }
        if (!any2) return;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (p2[k]) hit(k, j, idj, S[k]);
    };
    auto visit = [&](int32_t j, const bool take[G]) {
        real xj, yj, zj, vxj, vyj, vzj;
        uint32_t idj = 0;
        if constexpr (UNIFORM) {
            RecU<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj);
        } else if constexpr (HALF) {
            // FP32 keys carry the record index, not the id: skip that word.
            Rec<float>::load6(a.rec, (uint32_t)j, xj, yj, zj, vxj, vyj, vzj);
        } else {
            uint32_t flj;
            Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
        }
        screen(j, idj, xj, yj, zj, vxj, vyj, vzj, take);
    };

    if (UNIFORM || joint) {
        // UNIFORM: every lane of the wave shares the row and walks the union
        // of the wave's ranges (first record's lower end, wave_ub upper end)
        // in lock-step, so j is the same in all lanes.
        const int own_row = row_of(I, cy, cz);
        const int ua = UNIFORM ? __builtin_amdgcn_readfirstlane(x_lo_of(wave_first, a, I, n[0], G_.per[0])) : xa[0];
        int ub = xb[0];
#pragma unroll
        for (int k = 1; k < G; ++k)
            if (k < nrec) ub = xb[k];
        if (UNIFORM) ub = wave_ub;
        for (int rr = 0; rr < 9; ++rr) {
            int y, z;
            if (!axis_nb(cz, rr / 3 - 1, n[2], G_.per[2], z)) continue;
            if (!axis_nb(cy, rr % 3 - 1, n[1], G_.per[1], y)) continue;
            const int row_idx = row_of(I, y, z);
            if (HALF && row_idx < own_row) continue;
            const bool own = HALF && row_idx == own_row;
            const int64_t row = I.cell_off + (int64_t)n[0] * row_idx;
            int32_t lo[G], hi[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                lo[k] = own ? i0 + k + 1 : (int32_t)(base + a.start[row + xa[k]]);
                hi[k] = (int32_t)(base + a.start[row + xb[k] + 1]);
                if (k >= nrec || hi[k] < lo[k]) { lo[k] = 0; hi[k] = 0; }
                seen += hi[k] > lo[k] ? hi[k] - lo[k] : 0;
            }
            int32_t u0 = own ? (UNIFORM ? wave_first : i0) + 1 : (int32_t)(base + a.start[row + ua]);
            int32_t u1 = (int32_t)(base + a.start[row + ub + 1]);
            int32_t jm = u0;  // from jm on, the range masks need no test
            bool split = false;
            if constexpr (UNIFORM) {
                u0 = __builtin_amdgcn_readfirstlane(u0);
                u1 = __builtin_amdgcn_readfirstlane(u1);
                // When every non-empty range ends at u1, all of them are open
                // from the largest lower end on, which the last lane holds
                // (records are in c-bin order); checked for every lane.
                int32_t lo_last = lo[0];
#pragma unroll
                for (int k = 1; k < G; ++k)
                    if (k < nrec) lo_last = lo[k];
                const int last = 63 - __clzll((long long)__ballot(true));
                jm = __builtin_amdgcn_readlane(lo_last, last);
                bool open = true;
#pragma unroll
                for (int k = 0; k < G; ++k) open &= hi[k] <= lo[k] || (hi[k] == u1 && lo[k] <= jm);
                split = __ballot(!open) == 0 && jm >= u0 && jm <= u1;
            }
            const int32_t um = split ? jm : u1;
            for (int32_t j = u0; j < um; ++j) {
                bool take[G];
#pragma unroll
                for (int k = 0; k < G; ++k) take[k] = (uint32_t)(j - lo[k]) < (uint32_t)(hi[k] - lo[k]);
                visit(j, take);
            }
            if (split) {  // wave-uniform
                bool take[G];
#pragma unroll
                for (int k = 0; k < G; ++k) take[k] = hi[k] > lo[k];
                int32_t j = jm;
                if constexpr (G == 1) {
                    // Two neighbours per iteration, one vote: the second's
                    // loads are in flight with the first's, as a second
                    // record per lane would do for G = 2.
                    for (; j + 1 < u1; j += 2) {
                        real xa_, ya_, za_, vxa, vya, vza, xb_, yb_, zb_, vxb, vyb, vzb;
                        uint32_t ida, idb;
                        RecU<real>::load(a.rec, j, xa_, ya_, za_, ida, vxa, vya, vza);
                        RecU<real>::load(a.rec, j + 1, xb_, yb_, zb_, idb, vxb, vyb, vzb);
                        Screen<real> SA, SB;
                        const bool pa = PairTest<real, PM>::stage1(G_, xi[0], yi[0], zi[0], vxi[0], vyi[0], vzi[0],
                                                                   xa_, ya_, za_, vxa, vya, vza, SA) & take[0];
                        const bool pb = PairTest<real, PM>::stage1(G_, xi[0], yi[0], zi[0], vxi[0], vyi[0], vzi[0],
                                                                   xb_, yb_, zb_, vxb, vyb, vzb, SB) & take[0];
                        if constexpr (MIX) {
                            n_s0 += (take[0] && SA.s0 < real(0)) ? 1u : 0u;
                            n_s0 += (take[0] && SB.s0 < real(0)) ? 1u : 0u;
                            n_c1 += (pa ? 1u : 0u) + (pb ? 1u : 0u);
                        }
                        if (__builtin_amdgcn_ballot_w64(pa | pb) == 0) continue;
                        if (pa && PairTest<real, PM>::stage2(G_, SA)) hit(0, j, ida, SA);
                        if (pb && PairTest<real, PM>::stage2(G_, SB)) hit(0, j + 1, idb, SB);
                    }
                }
                for (; j < u1; ++j) visit(j, take);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k >= nrec) continue;
            const int32_t ik = i0 + k;
            for_neighbourhood<HALF>(a.start, I, base, n, G_.per, cxk[k], cy_of(yi[k], I), cz_of(zi[k], I),
                                    ik, [&](int32_t j0, int32_t j1) {
                seen += j1 > j0 ? j1 - j0 : 0;
                for (int32_t j = j0; j < j1; ++j) {
                    bool take[G];
#pragma unroll
                    for (int kk = 0; kk < G; ++kk) take[kk] = kk == k;
                    visit(j, take);
                }
            });
        }
    }
    if constexpr (!HALF) {
        // Split c-bins: ordered scans also take the fast particles of each
        // record's configured neighbourhood (binned apart from the slow ones).
        if (I.flags & kSplit) {
            const int nc[3] = {I.ncfg[0], I.ncfg[1], I.ncfg[2]};
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (k >= nrec) continue;
                const int ccx = axis_bin(xi[k], I.lo[0], I.inv_wc[0], nc[0]);
                const int ccy = axis_bin(yi[k], I.lo[1], I.inv_wc[1], nc[1]);
                const int ccz = axis_bin(zi[k], I.lo[2], I.inv_wc[2], nc[2]);
                for_neighbourhood<false, true>(a.start, I, base, nc, G_.per, ccx, ccy, ccz, i0 + k,
                                               [&](int32_t j0, int32_t j1) {
                    seen += j1 > j0 ? j1 - j0 : 0;
                    for (int32_t j = j0; j < j1; ++j) {
                        bool take[G];
#pragma unroll
                        for (int kk = 0; kk < G; ++kk) take[kk] = kk == k;
                        real xj, yj, zj, vxj, vyj, vzj;
                        uint32_t idj, flj;
                        Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
                        screen(j, idj, xj, yj, zj, vxj, vyj, vzj, take);
                    }
                });
            }
        }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
        if (k >= nrec) continue;
        if constexpr (HALF) {
            if (mine[k] != ~0ull) atomicMin(a.bkey + i0 + k, mine[k]);
        } else {
            a.best[i0 + k] = bj[k];
        }
    }
    // Ordered scans see every pair twice and count the record itself once.
    tests = HALF ? (double)seen : 0.5 * (double)(seen - nrec);
    cand = HALF ? 2.0 * (double)nc : (double)nc;
}

// Lane mode of the FP32 half scans, staged through LDS.  A wave that owns
// 64 G consecutive records takes them in G passes of 64, one record per lane
// (record wbase + 64 p + lane in pass p), so that its registers are those of
// one record whatever G is; G > 1 pays off in the wave-uniform mode instead.
// In each pass, the lanes whose records share one row walk every neighbour
// row together: the wave copies the union of their ranges in that row, a
// contiguous run of records, into its LDS buffer in chunks of kStageCap, and
// each lane reads its own part of each chunk from there.  A neighbour record
// is then fetched from memory once per wave instead of once per lane whose
// range holds it.  Records whose x-neighbourhood wraps around a periodic
// axis walk their own rows with global loads.  The pairs tested, the
// arithmetic and the combination of the keys are those of search_group, so
// the results are too.  Called by every lane of a wave holding a live slow
// record; stop ends the slow records.
template <int PM, int G, bool MIX>
__device__ __forceinline__ void search_staged(const StepArgs<float>& a, const Inst<float>& I, int64_t base,
                                              int32_t wbase, int32_t stop, double& tests, double& cand,
                                              uint32_t& n_s0, uint32_t& n_c1) {
    const Geo<float> G_(I);
    const int n[3] = {I.n[0], I.n[1], I.n[2]};
    extern __shared__ float4 tpkmc_stage[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float4* const sp = tpkmc_stage + wave * (kStageBytesPerWave / 16);
    const int lane = (int)(threadIdx.x & 63);
    const bool by_time = (I.flags & TPKMC_RANK_TIME) != 0;
    int32_t seen = 0, nc = 0;
    for (int p = 0; p < G; ++p) {
        const int32_t i = wbase + p * kWave + lane;
        const bool valid = i < stop;
        if (__ballot(valid) == 0) break;  // uniform: later passes start further on
        float xi, yi, zi, vxi, vyi, vzi;
        Rec<float>::load6(a.rec, (uint32_t)(valid ? i : wbase), xi, yi, zi, vxi, vyi, vzi);
        const int cx = axis_bin(xi, I.lo[0], I.inv_w[0], n[0]);
        const int cy = axis_bin(yi, I.lo[1], I.inv_w[1], n[1]);
        const int cz = axis_bin(zi, I.lo[2], I.inv_w[2], n[2]);
        int xa[2], xb[2];
        const bool joint = valid && x_ranges(cx, n[0], G_.per[0], xa, xb) == 1;
        unsigned long long mine = ~0ull;
        auto screen = [&](int32_t j, float xj, float yj, float zj, float vxj, float vyj, float vzj, bool take) {
            Screen<float> S;
            // Criterion 1 as two votes on the compares themselves, so that
            // the wave's decision stays in scalar masks.
            (void)PairTest<float, PM>::stage1(G_, xi, yi, zi, vxi, vyi, vzi, xj, yj, zj, vxj, vyj, vzj, S);
            const bool a0 = take & (S.s0 < 0.0f);
            const bool a1 = fmaf(S.vv, G_.dt, S.s0) > 0.0f;
            const uint64_t m = __builtin_amdgcn_ballot_w64(a0) & __builtin_amdgcn_ballot_w64(a1);
            const bool p1 = a0 & a1;
            if constexpr (MIX) {
                n_s0 += (take && S.s0 < 0.0f) ? 1u : 0u;
                n_c1 += p1 ? 1u : 0u;
            }
            if (m == 0) return;
            if (p1 && PairTest<float, PM>::stage2(G_, S)) {
                const float d2 = PairTest<float, PM>::finish(G_, S);
                if (d2 >= 0.0f) {
                    ++nc;
                    const float key = by_time ? PairTest<float, PM>::contact(G_, S) : d2;
                    const unsigned long long hi = (unsigned long long)sortable(key) << 32;
                    // An empty barrier on j keeps the compiler from carrying
                    // a 64-bit key pointer through the whole loop for this
                    // rare path.
                    int32_t jh = j;
                    asm volatile("" : "+v"(jh));
                    atomicMin(a.bkey + jh, hi | (uint32_t)i);
                    const unsigned long long kk = hi | (uint32_t)j;
                    mine = kk < mine ? kk : mine;
                }
            }
        };
        // Two neighbours j and j + 1 of the staged chunk, one vote: the two
        // tests are independent, so their LDS reads and arithmetic overlap
        // (the loop takes neighbours in pairs; measured on the 16M Sedov
        // search 1.23 -> 1.18 ms, the Noh and Sod searches 2-3% faster).
        auto screen2 = [&](int32_t j, const float4& pa, const float2& va, const float4& pb, const float2& vb) {
            Screen<float> SA, SB;
            (void)PairTest<float, PM>::stage1(G_, xi, yi, zi, vxi, vyi, vzi, pa.x, pa.y, pa.z, pa.w, va.x, va.y, SA);
            (void)PairTest<float, PM>::stage1(G_, xi, yi, zi, vxi, vyi, vzi, pb.x, pb.y, pb.z, pb.w, vb.x, vb.y, SB);
            const bool qa0 = SA.s0 < 0.0f, qa1 = fmaf(SA.vv, G_.dt, SA.s0) > 0.0f;
            const bool qb0 = SB.s0 < 0.0f, qb1 = fmaf(SB.vv, G_.dt, SB.s0) > 0.0f;
            const uint64_t m = (__builtin_amdgcn_ballot_w64(qa0) & __builtin_amdgcn_ballot_w64(qa1)) |
                               (__builtin_amdgcn_ballot_w64(qb0) & __builtin_amdgcn_ballot_w64(qb1));
            const bool pa1 = qa0 & qa1, pb1 = qb0 & qb1;
            if constexpr (MIX) {
                n_s0 += (qa0 ? 1u : 0u) + (qb0 ? 1u : 0u);
                n_c1 += (pa1 ? 1u : 0u) + (pb1 ? 1u : 0u);
            }
            if (m == 0) return;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const Screen<float>& S = h ? SB : SA;
                if ((h ? pb1 : pa1) && PairTest<float, PM>::stage2(G_, S)) {
                    const float d2 = PairTest<float, PM>::finish(G_, S);
                    if (d2 >= 0.0f) {
                        ++nc;
                        const float key = by_time ? PairTest<float, PM>::contact(G_, S) : d2;
                        const unsigned long long hk = (unsigned long long)sortable(key) << 32;
                        int32_t jh = j + h;  // see screen
                        asm volatile("" : "+v"(jh));
                        atomicMin(a.bkey + jh, hk | (uint32_t)i);
                        const unsigned long long kk = hk | (uint32_t)(j + h);
                        mine = kk < mine ? kk : mine;
                    }
                }
            }
        };
        // Lanes taking part in the copies: all of the wave's.
        const int own_row_l = row_of(I, cy, cz);
        uint64_t pending = __ballot(joint);
        while (pending) {
            // One group of lanes per row.  Records are in c-bin order, so the
            // group's lanes are consecutive and their x-bins non-decreasing:
            // the first lane holds the union's lower end, the last its upper.
            const int lead = __ffsll((long long)pending) - 1;
            const int R = __builtin_amdgcn_readlane(own_row_l, lead);
            const bool in = joint && own_row_l == R;
            const uint64_t gm = __ballot(in);
            pending &= ~gm;
            const int last = 63 - __clzll((long long)gm);
            const int gcy = __builtin_amdgcn_readlane(cy, lead);
            const int gcz = __builtin_amdgcn_readlane(cz, lead);
            const int ga = __builtin_amdgcn_readlane(xa[0], lead);
            const int gb = __builtin_amdgcn_readlane(xb[0], last);
            const int32_t gi = __builtin_amdgcn_readlane(i, lead);
            for (int rr = 0; rr < 9; ++rr) {
                int y, z;
                if (!axis_nb(gcz, rr / 3 - 1, n[2], G_.per[2], z)) continue;
                if (!axis_nb(gcy, rr % 3 - 1, n[1], G_.per[1], y)) continue;
                const int row_idx = row_of(I, y, z);
                if (row_idx < R) continue;  // half scans: rows of larger index, and own
                const bool own = row_idx == R;
                const int64_t row = I.cell_off + (int64_t)n[0] * row_idx;
                int32_t lo = 0, hi = 0;  // the lane's range in this row
                if (in) {
                    lo = own ? i + 1 : (int32_t)(base + a.start[row + xa[0]]);
                    hi = (int32_t)(base + a.start[row + xb[0] + 1]);
                    seen += hi > lo ? hi - lo : 0;
                }
                const int32_t u0 = own ? gi + 1 : (int32_t)(base + a.start[row + ga]);
                const int32_t u1 = (int32_t)(base + a.start[row + gb + 1]);
                for (int32_t c0 = u0; c0 < u1; c0 += kStageCap) {
                    const int32_t c1 = u1 - c0 < kStageCap ? u1 : c0 + kStageCap;
                    // Copy [c0, c1): each record's position and velocity.
                    // The previous chunk's reads have all returned: their
                    // values were used before its loop ended.
                    const float4* src = reinterpret_cast<const float4*>(a.rec) + 2 * (int64_t)c0;
                    for (int t = lane; t < c1 - c0; t += kWave) {
                        const float4 qa = src[2 * t], qb = src[2 * t + 1];
                        sp[t] = make_float4(qa.x, qa.y, qa.z, qb.x);
                        *reinterpret_cast<float2*>(sp + kStageCap + t) = make_float2(qb.y, qb.z);
                    }
                    // The wave's own writes, complete before any lane reads.
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    const int32_t j0 = lo > c0 ? lo : c0;
                    const int32_t j1 = hi < c1 ? hi : c1;
                    int32_t j = j0;
                    for (; j + 1 < j1; j += 2) {
                        const float4 pa = sp[j - c0], pb = sp[j + 1 - c0];
                        const float2 va = *reinterpret_cast<const float2*>(sp + kStageCap + (j - c0));
                        const float2 vb = *reinterpret_cast<const float2*>(sp + kStageCap + (j + 1 - c0));
                        screen2(j, pa, va, pb, vb);
                    }
                    if (j < j1) {
                        const float4 pj = sp[j - c0];
                        const float2 vj = *reinterpret_cast<const float2*>(sp + kStageCap + (j - c0));
                        screen(j, pj.x, pj.y, pj.z, pj.w, vj.x, vj.y, true);
                    }
                }
            }
        }
        if (valid && !joint) {
            for_neighbourhood<true>(a.start, I, base, n, G_.per, cx, cy, cz, i, [&](int32_t j0, int32_t j1) {
                seen += j1 > j0 ? j1 - j0 : 0;
                for (int32_t j = j0; j < j1; ++j) {
                    float xj, yj, zj, vxj, vyj, vzj;
                    Rec<float>::load6(a.rec, (uint32_t)j, xj, yj, zj, vxj, vyj, vzj);
                    screen(j, xj, yj, zj, vxj, vyj, vzj, true);
                }
            });
        }
        if (valid && mine != ~0ull) atomicMin(a.bkey + i, mine);
    }
    tests = (double)seen;
    cand = 2.0 * (double)nc;
}

// ---------------------------------------------------------------- 4a. fast particles of split c-bins
// With split c-bins the slow particles are binned on refined c-bins, at
// least as wide as the largest distance at which two slow particles can
// meet the criteria of Sec. 2.4 within the step (D + 2 v_c dt, v_c the speed
// bound), so every candidate pair of two slow particles lies in
// neighbouring refined c-bins, and every such pair that meets the criteria
// also lies in neighbouring configured c-bins.  The fast particles keep the
// configured c-bins and the configured 27-bin neighbourhood: their
// candidates are exactly those of the unsplit grid.

__device__ __forceinline__ int floor_div(int64_t a, int64_t b) {  // b > 0
    return (int)(a >= 0 ? a / b : -((-a + b - 1) / b));
}

// Fine (refined) c-bins along one axis that a fast particle at coordinate x,
// in configured c-bin cc, can meet a slow partner in: those that meet its
// configured neighbours' extent (cc - 1 .. cc + 1, wrapped on a periodic
// axis), cut to the fine c-bins within its reach (any pair meeting the
// criteria starts at most D + (|v_i| + v_c) dt apart on every axis), both
// widened by a rounding margin of the binnings (1e-3 + 1e-6 n_f fine
// c-bins, above the few-ulp error of an FP32 bin coordinate).  At most two
// ranges [fa, fb]; 0 when empty.  A record found there is kept only when
// its configured c-bin is a neighbour (checked exactly by the caller).  On
// an axis that is not refined the neighbours' extent is exact.
template <typename real>
__device__ __forceinline__ int fast_span(const Inst<real>& I, int ax, real x, double reach, int cc, bool periodic,
                                         int fa[2], int fb[2]) {
    const int nc = I.ncfg[ax], nf = I.n[ax];
    const double eps = 1e-3 + 1e-6 * (double)nf;
    const bool all = periodic && nc <= 3;  // every configured c-bin is a neighbour
    int lo = 0, hi = nf - 1;
    if (!all) {
        int c0 = cc - 1, c1 = cc + 1;
        if (!periodic) { c0 = c0 < 0 ? 0 : c0; c1 = c1 > nc - 1 ? nc - 1 : c1; }
        lo = c0;
        hi = c1;
        if (nf != nc) {
            const double r = (double)nf / (double)nc;
            lo = (int)floor((double)c0 * r - eps);
            hi = (int)floor((double)(c1 + 1) * r + eps);
        }
    }
    // The reach in fine c-bins (positions far outside the box keep the
    // neighbours' extent; bins of positions outside are clamped, as here).
    const double t = ((double)x - (double)I.lo[ax]) * (double)I.inv_w[ax];
    const double d = reach * (double)I.inv_w[ax];
    if (t > -0.5 * nf && t < 1.5 * nf) {
        int bl = (int)floor(t - d - eps), bh = (int)floor(t + d + eps);
        if (!periodic) {
            bl = bl < 0 ? 0 : (bl > nf - 1 ? nf - 1 : bl);
            bh = bh < 0 ? 0 : (bh > nf - 1 ? nf - 1 : bh);
        }
        if (all) { lo = bl; hi = bh; }
        else { lo = lo > bl ? lo : bl; hi = hi < bh ? hi : bh; }
    }
    if (hi < lo) return 0;
    if (!periodic) {
        fa[0] = lo < 0 ? 0 : lo;
        fb[0] = hi > nf - 1 ? nf - 1 : hi;
        return fb[0] >= fa[0] ? 1 : 0;
    }
    if (hi - lo + 1 >= nf) { fa[0] = 0; fb[0] = nf - 1; return 1; }
    const int k = floor_div(lo, nf);  // shift by whole periods so that 0 <= lo < nf
    lo -= k * nf;
    hi -= k * nf;
    if (hi > nf - 1) { fa[0] = lo; fb[0] = nf - 1; fa[1] = 0; fb[1] = hi - nf; return 2; }
    fa[0] = lo; fb[0] = hi;
    return 1;
}

// Largest number of fine c-bins fast_span gives on one axis for a reach of
// at most `reach` (the task list's stride per fast record).
template <typename real>
__device__ __forceinline__ int fast_span_len(const Inst<real>& I, int ax, double reach, bool periodic) {
    const int nc = I.ncfg[ax], nf = I.n[ax];
    const double eps = 1e-3 + 1e-6 * (double)nf;
    int len = (int)floor(2.0 * reach * (double)I.inv_w[ax] + 2.0 * eps) + 2;
    if (!(periodic && nc <= 3)) {
        const int nb = nf == nc ? 3 : (int)floor(3.0 * (double)nf / (double)nc + 2.0 * eps) + 2;
        len = len < nb ? len : nb;
    }
    return len < nf ? len : nf;
}

// Index t of the concatenation of at most two ranges [a[r], b[r]].
__device__ __forceinline__ int span_at(const int a[2], const int b[2], int len0, int t) {
    return t < len0 ? a[0] + t : a[1] + (t - len0);
}

// The configured neighbours of configured c-bin cc along one axis as
// (first, count - 1), wrapped on a periodic axis: bin c is a neighbour when
// (c - first) mod n <= span.  check: whether a slow record the fast
// particle at coordinate x can reach may lie outside them, so that its
// configured c-bin has to be checked.  The neighbours extend at least one
// configured c-bin beyond the particle's own; a record beyond the reach
// cannot meet the criteria, and one within it lies inside the neighbours
// unless the reach (widened by the rounding margin of the binnings) crosses
// a side that has a configured c-bin beyond it.  On an axis that is not
// refined the fine rows hold exactly the neighbours.
template <typename real>
__device__ __forceinline__ void coarse_nb(const Inst<real>& I, int ax, real x, double reach, int cc, bool periodic,
                                          int& first, int& span, bool& check) {
    const int nc = I.ncfg[ax];
    check = false;
    if (periodic && nc <= 3) { first = 0; span = nc - 1; return; }
    if (periodic) { first = cc == 0 ? nc - 1 : cc - 1; span = 2; }
    else {
        first = cc > 0 ? cc - 1 : 0;
        span = (cc < nc - 1 ? cc + 1 : nc - 1) - first;
    }
    if (I.n[ax] == nc) return;
    const double eps = 1e-3 + 1e-6 * (double)nc;  // in configured c-bins
    const double t = ((double)x - (double)I.lo[ax]) * (double)I.inv_wc[ax];
    const double d = reach * (double)I.inv_wc[ax];
    const bool below = periodic || cc >= 2, above = periodic || cc <= nc - 3;
    check = (below && t - d < (double)(cc - 1) + eps) || (above && t + d > (double)(cc + 2) - eps);
}

// Whether a slow record at (x, y, z) lies in a configured c-bin neighbouring
// the fast particle's, on the axes that need the check.
template <typename real>
__device__ __forceinline__ bool coarse_in(const Inst<real>& I, const bool chk[3], const int nc[3], const int first[3],
                                          const int span[3], real x, real y, real z) {
    const real p[3] = {x, y, z};
    bool in = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (!chk[ax]) continue;
        int u = axis_bin(p[ax], I.lo[ax], I.inv_wc[ax], nc[ax]) - first[ax];
        u += u < 0 ? nc[ax] : 0;
        in = in && u <= span[ax];
    }
    return in;
}

// Reach of a fast particle of speed^2 v2 towards slow partners, with the
// margin of the c-bin refinement for the rounding of the pair test.
template <typename real>
__device__ __forceinline__ double fast_reach(const Inst<real>& I, double v2) {
    return (sqrt((double)I.D2) + (sqrt(v2) + sqrt((double)I.vc2)) * (double)I.dt) * (1.0 + 1.0 / 64.0);
}

// Lexicographic minimum over the wave of (key, id) with a partner (j >= 0),
// the tie-break of the ordered scans.
template <typename real>
__device__ __forceinline__ void wave_best(int32_t& bj, real& bd2, uint32_t& bid) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const int32_t oj = __shfl_xor(bj, m);
        const real od = __shfl_xor(bd2, m);
        const uint32_t oi = __shfl_xor(bid, m);
        if (oj >= 0 && (bj < 0 || od < bd2 || (od == bd2 && oi < bid))) { bj = oj; bd2 = od; bid = oi; }
    }
}

// FP64: one fast record i of split c-bins, searched by a whole wave.  Every
// particle of its configured neighbourhood is a possible partner, as on the
// unsplit grid: the slow ones in the fine rows of fast_span (lanes take
// rows; a record is kept only when its configured c-bin is a neighbour), the
// fast ones on the configured c-bins (lanes take the nine rows).  The slow
// records' ordered scans take the fast particles of their configured
// neighbourhood (search_group).  The pair test, the ranking key and the
// tie-breaks are search_group's.
template <typename real, bool MIX>
__device__ void fast_record(const StepArgs<real>& a, const Inst<real>& I, int64_t base, int32_t i, int lane,
                            double& tests, double& cand, uint32_t& n_s0, uint32_t& n_c1) {
    const Geo<real> G_(I);
    const bool by_time = (I.flags & TPKMC_RANK_TIME) != 0;
    const int nf[3] = {I.n[0], I.n[1], I.n[2]};
    const int nc[3] = {I.ncfg[0], I.ncfg[1], I.ncfg[2]};
    real xi, yi, zi, vxi, vyi, vzi;
    uint32_t idi;
    RecU<real>::load(a.rec, i, xi, yi, zi, idi, vxi, vyi, vzi);
    const real pi[3] = {xi, yi, zi};
    const double reach = fast_reach(I, speed2((double)vxi, (double)vyi, (double)vzi));
    int cc[3], first[3], span[3];
    bool chk[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        cc[ax] = axis_bin(pi[ax], I.lo[ax], I.inv_wc[ax], nc[ax]);
        coarse_nb(I, ax, pi[ax], reach, cc[ax], G_.per[ax], first[ax], span[ax], chk[ax]);
    }
    int32_t bj = -1;
    real bd2 = real(0);
    uint32_t bid = 0;
    int32_t seen = 0, found = 0;
    auto test = [&](int32_t j, bool check) {
        real xj, yj, zj, vxj, vyj, vzj;
        uint32_t idj, flj;
        Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
        if (check && !coarse_in(I, chk, nc, first, span, xj, yj, zj)) return;
        ++seen;
        Screen<real> S;
        const bool p1 = PairTest<real, -1>::stage1(G_, xi, yi, zi, vxi, vyi, vzi, xj, yj, zj, vxj, vyj, vzj, S);
        if constexpr (MIX) {
            n_s0 += S.s0 < real(0) ? 1u : 0u;
            n_c1 += p1 ? 1u : 0u;
        }
        if (!p1 || !PairTest<real, -1>::stage2(G_, S)) return;
        const real d2 = PairTest<real, -1>::finish(G_, S);
        if (!(d2 >= real(0))) return;
        ++found;
        const real key = by_time ? PairTest<real, -1>::contact(G_, S) : d2;
        if (bj < 0 || key < bd2 || (key == bd2 && idj < bid)) { bj = j; bd2 = key; bid = idj; }
    };
    int xa[2], xb[2], ya[2], yb[2], za[2], zb[2];
    const int nxr = fast_span(I, 0, xi, reach, cc[0], G_.per[0], xa, xb);
    const int nyr = fast_span(I, 1, yi, reach, cc[1], G_.per[1], ya, yb);
    const int nzr = fast_span(I, 2, zi, reach, cc[2], G_.per[2], za, zb);
    const int ly0 = nyr ? yb[0] - ya[0] + 1 : 0, lz0 = nzr ? zb[0] - za[0] + 1 : 0;
    const int ny = ly0 + (nyr > 1 ? yb[1] - ya[1] + 1 : 0);
    const int nz = lz0 + (nzr > 1 ? zb[1] - za[1] + 1 : 0);
    for (int t = lane; t < ny * nz; t += kWave) {
        const int y = span_at(ya, yb, ly0, t % ny), z = span_at(za, zb, lz0, t / ny);
        const int64_t row = I.cell_off + (int64_t)nf[0] * row_of(I, y, z);
        for (int rx = 0; rx < nxr; ++rx) {
            const int32_t j0 = (int32_t)(base + a.start[row + xa[rx]]);
            const int32_t j1 = (int32_t)(base + a.start[row + xb[rx] + 1]);
            for (int32_t j = j0; j < j1; ++j) test(j, true);
        }
    }
    if (lane < 9)
        neighbourhood_row<false, true>(a.start, I, base, nc, G_.per, cc[0], cc[1], cc[2], i, lane,
                                       [&](int32_t j0, int32_t j1) {
            for (int32_t j = j0; j < j1; ++j) test(j, false);
        });
    double sn = (double)seen, fn = (double)found;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        sn += __shfl_xor(sn, m);
        fn += __shfl_xor(fn, m);
    }
    wave_best(bj, bd2, bid);
    if (lane == 0) a.best[i] = bj;
    tests += 0.5 * (sn - 1.0);  // the record met itself once
    cand += fn;
}

// FP32: the fast records' searches as a flat list of tasks, one per lane:
// (fast record, row) for the fine rows of fast_span (index t < ny * nz) and
// for the nine rows of configured c-bins of the fast particles (half
// neighbourhood), so lanes stay busy however few rows a record has or
// however many fast records there are.  A slow row longer than kLongRow
// records (dense bins) is walked by the whole wave, lanes striding over its
// records.  Every candidate lowers both keys with atomicMin, so the tasks of
// one record may run in any lanes and any order.
constexpr int kLongRow = 64;

template <bool MIX>
__device__ void fast_tasks(const StepArgs<float>& a, const Inst<float>& I, int64_t base, int64_t f0, int64_t ntask,
                           int per_rec, int rmax, int64_t q, int lane, double& seen, double& cand, uint32_t& n_s0,
                           uint32_t& n_c1) {
    const Geo<float> G_(I);
    const bool by_time = (I.flags & TPKMC_RANK_TIME) != 0;
    const int nf[3] = {I.n[0], I.n[1], I.n[2]};
    const int nc[3] = {I.ncfg[0], I.ncfg[1], I.ncfg[2]};
    const bool valid = q < ntask;
    int32_t i = 0;
    int t = 0;
    float xi = 0.f, yi = 0.f, zi = 0.f, vxi = 0.f, vyi = 0.f, vzi = 0.f;
    int cc[3] = {0, 0, 0}, first[3] = {0, 0, 0}, span[3] = {0, 0, 0};
    bool chk[3] = {false, false, false};
    int32_t ja[2] = {0, 0}, jb[2] = {0, 0};
    bool slow = false;
    if (valid) {
        i = (int32_t)(f0 + q / per_rec);
        t = (int)(q % per_rec);
        Rec<float>::load6(a.rec, (uint32_t)i, xi, yi, zi, vxi, vyi, vzi);
        const float pi[3] = {xi, yi, zi};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) cc[ax] = axis_bin(pi[ax], I.lo[ax], I.inv_wc[ax], nc[ax]);
        if (t < rmax) {
            const double reach = fast_reach(I, speed2((double)vxi, (double)vyi, (double)vzi));
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                coarse_nb(I, ax, pi[ax], reach, cc[ax], G_.per[ax], first[ax], span[ax], chk[ax]);
            int ya[2], yb[2], za[2], zb[2];
            const int nyr = fast_span(I, 1, yi, reach, cc[1], G_.per[1], ya, yb);
            const int nzr = fast_span(I, 2, zi, reach, cc[2], G_.per[2], za, zb);
            const int ly0 = nyr ? yb[0] - ya[0] + 1 : 0, lz0 = nzr ? zb[0] - za[0] + 1 : 0;
            const int ny = ly0 + (nyr > 1 ? yb[1] - ya[1] + 1 : 0);
            const int nz = lz0 + (nzr > 1 ? zb[1] - za[1] + 1 : 0);
            if (t < ny * nz) {
                int xa[2], xb[2];
                const int nxr = fast_span(I, 0, xi, reach, cc[0], G_.per[0], xa, xb);
                const int y = span_at(ya, yb, ly0, t % ny), z = span_at(za, zb, lz0, t / ny);
                const int64_t row = I.cell_off + (int64_t)nf[0] * row_of(I, y, z);
                for (int rx = 0; rx < nxr; ++rx) {
                    ja[rx] = (int32_t)(base + a.start[row + xa[rx]]);
                    jb[rx] = (int32_t)(base + a.start[row + xb[rx] + 1]);
                }
                slow = true;
            }
        }
    }
    // Tests slow or fast record j against fast record ii (the lane's own or,
    // for long rows, the owner lane's, whose values are passed in).
    auto test = [&](int32_t ii, float x0, float y0, float z0, float u0, float u1, float u2, int32_t j,
                    unsigned long long& mine) {
        float xj, yj, zj, vxj, vyj, vzj;
        Rec<float>::load6(a.rec, (uint32_t)j, xj, yj, zj, vxj, vyj, vzj);
        seen += 1.0;
        Screen<float> S;
        const bool p1 = PairTest<float, -1>::stage1(G_, x0, y0, z0, u0, u1, u2, xj, yj, zj, vxj, vyj, vzj, S);
        if constexpr (MIX) {
            n_s0 += S.s0 < 0.0f ? 1u : 0u;
            n_c1 += p1 ? 1u : 0u;
        }
        if (!p1 || !PairTest<float, -1>::stage2(G_, S)) return;
        const float d2 = PairTest<float, -1>::finish(G_, S);
        if (!(d2 >= 0.0f)) return;
        cand += 2.0;  // both orders, as search_group counts
        const float key = by_time ? PairTest<float, -1>::contact(G_, S) : d2;
        const unsigned long long hi = (unsigned long long)sortable(key) << 32;
        atomicMin(a.bkey + j, hi | (uint32_t)ii);
        const unsigned long long kk = hi | (uint32_t)j;
        mine = kk < mine ? kk : mine;
    };
    const int len = slow ? (jb[0] - ja[0]) + (jb[1] - ja[1]) : 0;
    // Long slow rows: the whole wave, one owner lane at a time.
    uint64_t longm = __ballot(len > kLongRow);
    while (longm) {
        const int o = __ffsll((long long)longm) - 1;
        longm &= longm - 1;
        const int32_t io = __builtin_amdgcn_readlane(i, o);
        const float xo = __shfl(xi, o), yo = __shfl(yi, o), zo = __shfl(zi, o);
        const float uo0 = __shfl(vxi, o), uo1 = __shfl(vyi, o), uo2 = __shfl(vzi, o);
        int fo[3], so[3];
        bool co[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            fo[ax] = __builtin_amdgcn_readlane(first[ax], o);
            so[ax] = __builtin_amdgcn_readlane(span[ax], o);
            co[ax] = __builtin_amdgcn_readlane((int)chk[ax], o) != 0;
        }
        unsigned long long mo = ~0ull;
#pragma unroll
        for (int rx = 0; rx < 2; ++rx) {
            const int32_t a0 = __builtin_amdgcn_readlane(ja[rx], o), b0 = __builtin_amdgcn_readlane(jb[rx], o);
            for (int32_t j = a0 + lane; j < b0; j += kWave) {
                float xj, yj, zj, vxj, vyj, vzj;
                Rec<float>::load6(a.rec, (uint32_t)j, xj, yj, zj, vxj, vyj, vzj);
                if (coarse_in(I, co, nc, fo, so, xj, yj, zj)) test(io, xo, yo, zo, uo0, uo1, uo2, j, mo);
            }
        }
        if (mo != ~0ull) atomicMin(a.bkey + io, mo);
    }
    unsigned long long mine = ~0ull;
    if (slow && len <= kLongRow) {
#pragma unroll
        for (int rx = 0; rx < 2; ++rx)
            for (int32_t j = ja[rx]; j < jb[rx]; ++j) {
                float xj, yj, zj, vxj, vyj, vzj;
                Rec<float>::load6(a.rec, (uint32_t)j, xj, yj, zj, vxj, vyj, vzj);
                if (coarse_in(I, chk, nc, first, span, xj, yj, zj)) test(i, xi, yi, zi, vxi, vyi, vzi, j, mine);
            }
    } else if (valid && t >= rmax) {
        neighbourhood_row<true, true>(a.start, I, base, nc, G_.per, cc[0], cc[1], cc[2], i, t - rmax,
                                      [&](int32_t j0, int32_t j1) {
            for (int32_t j = j0; j < j1; ++j) test(i, xi, yi, zi, vxi, vyi, vzi, j, mine);
        });
    }
    if (mine != ~0ull) atomicMin(a.bkey + i, mine);
}

// search_group for the instance's periodic axes: FP32 has builds for the
// masks of the usual boxes (none; z, as in the Noh implosions and the planar
// gases; y and z, as in the Sod tubes; all three), which leave the other axes
// out of the pair test; other masks, and FP64, read them at run time.
template <typename real, bool HALF, int G, bool UNIFORM, bool MIX>
__device__ __forceinline__ void search_for_axes(int pm, const StepArgs<real>& a, const Inst<real>& I, int64_t base,
                                                int32_t i0, int nrec, int32_t wave_first, int wave_ub,
                                                double& tests, double& cand, uint32_t& n_s0, uint32_t& n_c1) {
#define TPKMC_SEARCH(PMV) \
    search_group<real, HALF, PMV, G, UNIFORM, MIX>(a, I, base, i0, nrec, wave_first, wave_ub, tests, cand, n_s0, n_c1)
    if constexpr (std::is_same<real, float>::value) {
        switch (pm) {
            case 0: TPKMC_SEARCH(0); break;
            case 4: TPKMC_SEARCH(4); break;
            case 6: TPKMC_SEARCH(6); break;
            case 7: TPKMC_SEARCH(7); break;
            default: TPKMC_SEARCH(-1); break;
        }
    } else {
        if (pm == 0) TPKMC_SEARCH(0);
        else TPKMC_SEARCH(-1);
    }
#undef TPKMC_SEARCH
}

template <int G, bool MIX>
__device__ __forceinline__ void search_staged_for_axes(int pm, const StepArgs<float>& a, const Inst<float>& I,
                                                       int64_t base, int32_t wbase, int32_t stop, double& tests,
                                                       double& cand, uint32_t& n_s0, uint32_t& n_c1) {
#define TPKMC_STAGED(PMV) search_staged<PMV, G, MIX>(a, I, base, wbase, stop, tests, cand, n_s0, n_c1)
    switch (pm) {
        case 0: TPKMC_STAGED(0); break;
        case 4: TPKMC_STAGED(4); break;
        case 6: TPKMC_STAGED(6); break;
        case 7: TPKMC_STAGED(7); break;
        default: TPKMC_STAGED(-1); break;
    }
#undef TPKMC_STAGED
}

// One table entry (kBlock records) is covered by kBlock / G lanes, split
// into work-groups of blockDim.x lanes.  FP32 launches carry one LDS staging
// buffer per wave (kStageBytesPerWave of dynamic LDS).
// The FP32 two-records-per-lane shape (the usual autotuner choice) is held to
// at most 72 VGPRs, 7 waves per SIMD (with a lane mode walking both records
// at once it needed 78, and the seventh wave was worth 3-4% on the search);
// with the staged lane mode, one record per pass, it needs 68.
template <typename real, bool HALF, int G, bool MIX = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((HALF && G == 2) ? 7 : 1, 8)))
k_search(StepArgs<real> a) {
    __shared__ double lds[16];
    const int lanes = kBlock / G;
    const int sub = lanes / blockDim.x;
    const int lb = a.order > 0 ? xcd_chunk_remap(blockIdx.x, gridDim.x, a.order) : xcd_remap(blockIdx.x, gridDim.x);
    const int entry = lb / sub;
    const Blk bt = a.blk[entry];
    const Inst<real>& I = a.inst[bt.inst];
    if (I.flags & TPKMC_PAIR_RANDOM) return;  // partners from k_rp_* instead
    const int64_t i0 = (int64_t)bt.first + ((int64_t)(lb % sub) * blockDim.x + threadIdx.x) * G;
    const int64_t base = I.off - a.start[I.cell_off];
    const int64_t live_end = base + a.start[I.cell_off + I.C];
    const int64_t end = I.off + I.cnt;
    const int pm = (I.bc[0] == TPKMC_BC_PERIODIC ? 1 : 0) | (I.bc[1] == TPKMC_BC_PERIODIC ? 2 : 0) |
                   (I.bc[2] == TPKMC_BC_PERIODIC ? 4 : 0);
    double tests = 0.0, cand = 0.0;
    const int64_t live_stop = live_end < end ? live_end : end;
    const int nrec = i0 < live_stop ? (int)(live_stop - i0 < G ? live_stop - i0 : G) : 0;
    // Split c-bins: the slow records come first; the fast ones after them are
    // searched by k_search_fast.
    const int64_t slow_stop = (I.flags & kSplit) ? min(base + a.start[I.cell_off + I.Cf], live_stop) : live_stop;
    const int nslow = i0 < slow_stop ? (int)(slow_stop - i0 < nrec ? slow_stop - i0 : nrec) : 0;
    // Wave-uniform mode when the wave's live slow records lie in at most two
    // neighbouring bins of one row (dense bins): decided on the first and
    // last of them, so the branch is uniform.  Otherwise the lane mode:
    // staged through LDS in FP32 (search_staged), per lane in FP64.
    const uint64_t live = __ballot(nslow > 0);
    bool uni = false;
    int32_t wfirst = 0;
    int wub = 0;
    if (live) {
        const int fl = __ffsll((long long)live) - 1;
        const int ll = 63 - __clzll((long long)live);
        wfirst = __builtin_amdgcn_readlane((int32_t)i0, fl);
        const int32_t wlast = __builtin_amdgcn_readlane((int32_t)(i0 + nslow - 1), ll);
        real xf, yf, zf, vxf, vyf, vzf, xl, yl, zl, vxl, vyl, vzl;
        uint32_t idf, idl;
        RecU<real>::load(a.rec, wfirst, xf, yf, zf, idf, vxf, vyf, vzf);
        RecU<real>::load(a.rec, wlast, xl, yl, zl, idl, vxl, vyl, vzl);
        const int cxf = axis_bin(xf, I.lo[0], I.inv_w[0], I.n[0]);
        const int cxl = axis_bin(xl, I.lo[0], I.inv_w[0], I.n[0]);
        const bool per0 = I.bc[0] == TPKMC_BC_PERIODIC;
        int xa[2], xb[2];
        const int nrf = x_ranges(cxf, I.n[0], per0, xa, xb);
        const int nrl = x_ranges(cxl, I.n[0], per0, xa, xb);
        wub = xb[0];
        uni = nrf == 1 && nrl == 1 && cxl - cxf <= 1 &&
              axis_bin(yf, I.lo[1], I.inv_w[1], I.n[1]) == axis_bin(yl, I.lo[1], I.inv_w[1], I.n[1]) &&
              axis_bin(zf, I.lo[2], I.inv_w[2], I.n[2]) == axis_bin(zl, I.lo[2], I.inv_w[2], I.n[2]);
    }
    uint32_t n_s0 = 0, n_c1 = 0;
    if (uni) {
        if (nslow > 0)
            search_for_axes<real, HALF, G, true, MIX>(pm, a, I, base, (int32_t)i0, nslow, wfirst, wub, tests, cand,
                                                      n_s0, n_c1);
    } else if constexpr (HALF) {
        if (live) {  // wave-uniform: every lane of the wave takes part
            const int32_t wbase = (int32_t)(i0 - (int64_t)(threadIdx.x & 63) * G);
            search_staged_for_axes<G, MIX>(pm, a, I, base, wbase, (int32_t)slow_stop, tests, cand, n_s0, n_c1);
        }
    } else if (nslow > 0) {
        search_for_axes<real, HALF, G, false, MIX>(pm, a, I, base, (int32_t)i0, nslow, 0, 0, tests, cand, n_s0,
                                                   n_c1);
    }

    if constexpr (MIX) {
        // Counted twice per unordered pair, so every work-group's share is an
        // integer: ordered scans meet each pair from both sides (s0 is
        // symmetric in i and j bit for bit), half scans once (doubled here).
        // The host halves the totals.
        const double f = HALF ? 2.0 : 1.0;
        const double t0 = block_sum(2.0 * tests, lds), t1 = block_sum(f * (double)n_s0, lds),
                     t2 = block_sum(f * (double)n_c1, lds);
        if (threadIdx.x == 0) {
            atomicAdd(a.mix + 0, (unsigned long long)t0);
            atomicAdd(a.mix + 1, (unsigned long long)t1);
            atomicAdd(a.mix + 2, (unsigned long long)t2);
        }
        return;
    }
    if (!HALF) {
        for (int k = nrec; k < G; ++k)
            if (i0 + k < end) a.best[i0 + k] = -1;
    }
    const double t = block_sum(tests, lds);
    const double c = block_sum(cand, lds);
    if (threadIdx.x == 0) {
        double* gp = a.gpart + (int64_t)entry * kGPart;
        if (sub == 1) {
            gp[GP_TESTS2] = 2.0 * t;
            gp[GP_CAND] = c;
        } else {
            unsafeAtomicAdd(gp + GP_TESTS2, 2.0 * t);
            unsafeAtomicAdd(gp + GP_CAND, c);
        }
    }
}

// The fast records of split c-bins, in a launch of their own after k_search
// (FP32 keys combine with atomicMin in any order; in FP64 each fast record
// writes its own partner), so that the slow records' search keeps its
// register budget.  FP32 strides over the task list of fast_tasks; FP64 runs
// one fast record per wave (fast_record).  The search's work counters are
// summed per work-group and instance, and added to the instance's first
// block-table entry.
template <typename real, bool HALF, bool MIX = false>
__global__ void __launch_bounds__(256) k_search_fast(StepArgs<real> a, int n_inst) {
    __shared__ double lds[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    double mt = 0.0;
    uint32_t n_s0 = 0, n_c1 = 0;
    for (int k = 0; k < n_inst; ++k) {
        const Inst<real>& I = a.inst[k];
        if (!(I.flags & kSplit) || (I.flags & TPKMC_PAIR_RANDOM)) continue;
        const int64_t base = I.off - a.start[I.cell_off];
        const int64_t f0 = base + a.start[I.cell_off + I.Cf];
        const int64_t live_end = base + a.start[I.cell_off + I.C];
        const int64_t f1 = live_end < I.off + I.cnt ? live_end : I.off + I.cnt;
        double t = 0.0, c = 0.0;
        if constexpr (HALF) {
            // Rows per fast record: the fine rows within the largest reach
            // of this step's fastest particle, then the nine coarse rows.
            const double reach = fast_reach(I, I.vmax2_d);
            const bool per1 = I.bc[1] == TPKMC_BC_PERIODIC, per2 = I.bc[2] == TPKMC_BC_PERIODIC;
            const int rmax = fast_span_len(I, 1, reach, per1) * fast_span_len(I, 2, reach, per2);
            const int per_rec = rmax + 9;
            const int64_t ntask = (f1 - f0) * per_rec;
            for (int64_t q0 = tid - lane; q0 < ntask; q0 += nth)  // wave-uniform
                fast_tasks<MIX>(a, I, base, f0, ntask, per_rec, rmax, q0 + lane, lane, t, c, n_s0, n_c1);
        } else {
            const int64_t wave = tid / kWave, nwaves = nth / kWave;
            for (int64_t r = f0 + wave; r < f1; r += nwaves) {
                double tr = 0.0, cr = 0.0;
                const int32_t ri = __builtin_amdgcn_readfirstlane((int32_t)r);  // wave-uniform
                fast_record<real, MIX>(a, I, base, ri, lane, tr, cr, n_s0, n_c1);
                t += lane == 0 ? tr : 0.0;
                c += lane == 0 ? cr : 0.0;
            }
        }
        if constexpr (MIX) {
            mt += t;
        } else {
            // Uniform over the work-group (the instance loop is), so every
            // thread takes part in the sums.
            const double ts = block_sum(t, lds), cs = block_sum(c, lds);
            if (threadIdx.x == 0) {
                double* gp = a.gpart + (int64_t)I.blk0 * kGPart;
                if (ts > 0.0) unsafeAtomicAdd(gp + GP_TESTS2, 2.0 * ts);
                if (cs > 0.0) unsafeAtomicAdd(gp + GP_CAND, cs);
            }
        }
    }
    if constexpr (MIX) {
        // The counting convention of k_search's diagnostic build.
        const double f = HALF ? 2.0 : 1.0;
        const double t0 = block_sum(2.0 * mt, lds), t1 = block_sum(f * (double)n_s0, lds),
                     t2 = block_sum(f * (double)n_c1, lds);
        if (threadIdx.x == 0) {
            if (t0 > 0.0) atomicAdd(a.mix + 0, (unsigned long long)t0);
            if (t1 > 0.0) atomicAdd(a.mix + 1, (unsigned long long)t1);
            if (t2 > 0.0) atomicAdd(a.mix + 2, (unsigned long long)t2);
        }
    }
}

// ---------------------------------------------------------------- 4b. random partners
// Random partners inside each c-bin (TPKMC_PAIR_RANDOM, the usual DSMC rule
// of Sec. 2.3) in place of the search: every live record gets a Philox key,
// the records of a c-bin are ranked by (key, id), and ranks (0, 1), (2, 3),
// ... pair up.  Three passes (launch boundaries order them): the keys; the
// rank of every record among its c-bin's (a loop over the c-bin, O(n_c^2)
// per c-bin like the neighbourhood search) with the c-bin-local order in
// perm; the partners.  The rank goes through `best` (free until the last
// pass writes the FP64 partner there) and the keys through `rank` (free
// after the scatter).

__device__ __forceinline__ uint32_t random_key(const uint32_t k0, const uint32_t k1, uint32_t step,
                                               uint32_t instance, uint32_t id) {
    uint32_t c[4] = {step, id, id, (instance << 8) | 255u};
    philox4x32_10(c, k0, k1);
    return c[0];
}

template <typename real> __device__ __forceinline__ uint32_t record_id(const real* rec, int64_t i);
template <> __device__ __forceinline__ uint32_t record_id<float>(const float* rec, int64_t i) {
    return reinterpret_cast<const uint32_t*>(rec)[8 * i + 3];
}
template <> __device__ __forceinline__ uint32_t record_id<double>(const double* rec, int64_t i) {
    return (uint32_t)reinterpret_cast<const unsigned long long*>(rec)[8 * i + 3];
}

// Global c-bin of a record, from its position (the key kernel's arithmetic).
template <typename real>
__device__ __forceinline__ int64_t record_cbin(const Inst<real>& I, real x, real y, real z) {
    const int cx = axis_bin(x, I.lo[0], I.inv_w[0], I.n[0]);
    const int cy = axis_bin(y, I.lo[1], I.inv_w[1], I.n[1]);
    const int cz = axis_bin(z, I.lo[2], I.inv_w[2], I.n[2]);
    return I.cell_off + cx + (int64_t)I.n[0] * row_of(I, cy, cz);
}

template <typename real>
__global__ void __launch_bounds__(kBlock) k_rp_key(StepArgs<real> a) {
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    if (!(I.flags & TPKMC_PAIR_RANDOM)) return;
    const int64_t base = I.off - a.start[I.cell_off];
    const int64_t live_end = base + a.start[I.cell_off + I.C];
    const int64_t i = (int64_t)bt.first + threadIdx.x;
    if (i < live_end && i < I.off + I.cnt)
        reinterpret_cast<uint32_t*>(a.rank)[i] =
            random_key(I.seed_lo, I.seed_hi, I.step_lo, I.instance, record_id<real>(a.rec, i));
}

template <typename real>
__global__ void __launch_bounds__(kBlock) k_rp_rank(StepArgs<real> a) {
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    if (!(I.flags & TPKMC_PAIR_RANDOM)) return;
    const int64_t base = I.off - a.start[I.cell_off];
    const int64_t live_end = base + a.start[I.cell_off + I.C];
    const int64_t i = (int64_t)bt.first + threadIdx.x;
    if (!(i < live_end && i < I.off + I.cnt)) return;
    real x, y, z, vx, vy, vz;
    uint32_t id, fl;
    Rec<real>::load(a.rec, i, x, y, z, id, vx, vy, vz, fl);
    const int64_t k = record_cbin(I, x, y, z);
    const int64_t lo = base + a.start[k], hi = base + a.start[k + 1];
    const uint32_t* key = reinterpret_cast<const uint32_t*>(a.rank);
    const uint32_t mine = key[i];
    int32_t r = 0;
    for (int64_t j = lo; j < hi; ++j) {
        const uint32_t kj = key[j];
        r += (kj < mine || (kj == mine && record_id<real>(a.rec, j) < id)) ? 1 : 0;
    }
    a.perm[lo + r] = (int32_t)i;
    a.best[i] = r;
}

template <typename real>
__global__ void __launch_bounds__(kBlock) k_rp_partner(StepArgs<real> a) {
    __shared__ double lds[16];
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    if (!(I.flags & TPKMC_PAIR_RANDOM)) return;
    const int64_t base = I.off - a.start[I.cell_off];
    const int64_t live_end = base + a.start[I.cell_off + I.C];
    const int64_t i = (int64_t)bt.first + threadIdx.x;
    double formed = 0.0, paired = 0.0;
    if (i < I.off + I.cnt) {
        int32_t partner = -1;
        if (i < live_end) {
            real x, y, z, vx, vy, vz;
            uint32_t id, fl;
            Rec<real>::load(a.rec, i, x, y, z, id, vx, vy, vz, fl);
            const int64_t k = record_cbin(I, x, y, z);
            const int64_t lo = base + a.start[k], nc = base + a.start[k + 1] - lo;
            const int32_t r = a.best[i], q = r ^ 1;
            if (q < nc) {
                partner = a.perm[lo + q];
                paired = 1.0;
                formed = (r & 1) == 0 ? 1.0 : 0.0;
            }
        }
        if constexpr (std::is_same<real, double>::value) a.best[i] = partner;
        else a.bkey[i] = partner >= 0 ? (unsigned long long)(uint32_t)partner : ~0ull;
    }
    const double f = block_sum(formed, lds);
    const double c = block_sum(paired, lds);
    if (threadIdx.x == 0 && (f != 0.0 || c != 0.0)) {
        double* gp = a.gpart + (int64_t)blockIdx.x * kGPart;
        unsafeAtomicAdd(gp + GP_TESTS2, 2.0 * f);
        unsafeAtomicAdd(gp + GP_CAND, c);
    }
}

// Whether the random pair of record i (position x, y, z) and its partner
// collides: u < (((n_c - 1) sigma) g) dt / V_c in double, with the pair's own
// Philox draw; both records of the pair take the same decision.
template <typename real>
__device__ __forceinline__ bool random_pair_collides(const StepArgs<real>& a, const Inst<real>& I, real x, real y,
                                                     real z, uint32_t idi, real vxi, real vyi, real vzi,
                                                     uint32_t idj, real vxj, real vyj, real vzj) {
#pragma clang fp contract(off)
    const bool iA = idi < idj;
    const double ux = iA ? (double)vxi - (double)vxj : (double)vxj - (double)vxi;
    const double uy = iA ? (double)vyi - (double)vyj : (double)vyj - (double)vyi;
    const double uz = iA ? (double)vzi - (double)vzj : (double)vzj - (double)vzi;
    const double g = sqrt((ux * ux + uy * uy) + uz * uz);
    const int64_t k = record_cbin(I, x, y, z);
    const int64_t nc = (int64_t)a.start[k + 1] - a.start[k];
    const double prob = ((((double)(nc - 1) * I.sigma_d) * g) * I.dt_d) / I.cellvol_d;
    uint32_t c[4] = {I.step_lo, iA ? idi : idj, iA ? idj : idi, (I.instance << 8) | 255u};
    philox4x32_10(c, I.seed_lo, I.seed_hi);
    const double u = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
    return u < prob;
}

// ---------------------------------------------------------------- 5. move
// Partner record of record i after the search, or -1.
template <typename real> __device__ __forceinline__ int32_t partner_of(const StepArgs<real>& a, int64_t i);
template <> __device__ __forceinline__ int32_t partner_of<double>(const StepArgs<double>& a, int64_t i) {
    return a.best[i];
}
template <> __device__ __forceinline__ int32_t partner_of<float>(const StepArgs<float>& a, int64_t i) {
    const unsigned long long k = a.bkey[i];
    return k == ~0ull ? -1 : (int32_t)(uint32_t)k;
}

// o-bin (with the instance's offset) of a position.
template <typename real>
__device__ __forceinline__ int obin_of(const Inst<real>& I, real x, real y, real z) {
    const int bx = axis_bin(x, I.lo[0], I.inv_wo[0], I.no[0]);
    const int by = axis_bin(y, I.lo[1], I.inv_wo[1], I.no[1]);
    const int bz = axis_bin(z, I.lo[2], I.inv_wo[2], I.no[2]);
    return (int)(I.obin_off + bx + (int64_t)I.no[0] * (by + (int64_t)I.no[1] * bz));
}

// ------------------------------------------------------- exact o-bin sums
// The moment terms of one particle (kinds as in ObAcc), computed the same
// way in both passes: m (v - shift), m (v - shift)^2, the virial terms and
// the mass.
__device__ __forceinline__ void moment_terms(double m, double vx, double vy, double vz, const double* S,
                                             double virx, double viry, double virz, double t[kAccVals]) {
    const double ex = vx - S[0], ey = vy - S[1], ez = vz - S[2];
    t[0] = m * ex; t[1] = m * ey; t[2] = m * ez;
    t[3] = t[0] * ex; t[4] = t[1] * ey; t[5] = t[2] * ez;
    t[6] = virx; t[7] = viry; t[8] = virz;
    t[9] = m;
}

// Biased exponent E + kExpBias of the smallest power of two 2^E > |x| (0 for
// x = 0).
__device__ __forceinline__ int exp_above(double x) {
    return x != 0.0 ? ilogb(x) + 1 + kExpBias : 0;
}

// x rounded to the nearest multiple of 2^(E-50), in units of that quantum;
// scale = 2^(50-E) and |x| < 2^E, so |x scale| < 2^50.  Adding 1.5 2^52
// rounds x scale to an integer (nearest, ties to even; the product is exact)
// and leaves that integer plus 2^51 in the low mantissa bits.
__device__ __forceinline__ long long to_fixed(double x, double scale) {
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    return __double_as_longlong(fma(x, scale, kMagic)) - 0x4338000000000000ll;
}

// 2^(50-h-E) for a biased exponent E and headroom h, kept a normal double.
__device__ __forceinline__ double fixed_scale(int eb, int h) {
    const int e = eb > 0 ? eb - kExpBias : 0;
    return ldexp(1.0, 50 - h - max(e, -969));
}

template <int CTRL>
__device__ __forceinline__ long long dpp_move64(long long v) {
    const uint32_t l0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t l1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)((unsigned long long)v >> 32), CTRL,
                                                           0xF, 0xF, false);
    return (long long)(((unsigned long long)l1 << 32) | l0);
}

// Adds one work-group (or lane) sum of a value to the global sum of an
// o-bin (one int64; see ObAcc for the bound).
__device__ __forceinline__ void global_acc_add(ObAcc& G, int k, long long v) {
    if (v) atomicAdd((unsigned long long*)&G.sum[k], (unsigned long long)v);
}

// Work-group tables keyed by o-bin (open addressing), flushed to the global
// accumulators once per work-group: exponent maxima in the move, value sums
// in the moment pass.
constexpr int kSlots = 64;       // exponent table (the move's 256 records)
constexpr int kMomSlots = 128;   // value table (the moment pass's kMomEntries * 256 records)
constexpr int kTabWords = kAccVals;  // the values' integer sums
struct MomentTable {
    static constexpr int kN = kMomSlots;
    int key[kN];
    long long val[kN][kTabWords];
};
struct ExpTable {
    static constexpr int kN = kSlots;
    int key[kN];
    int e[kN][4];
    uint32_t n[kN][2];  // particles, colliders
};

template <typename Table>
__device__ __forceinline__ int table_slot(Table& T, int ob) {
    constexpr int N = Table::kN;
    const int h = (int)((ob * 0x9E3779B1u) >> 24);  // 8 bits
    for (int probe = 0; probe < N; ++probe) {
        const int s = (h + probe) & (N - 1);
        const int cur = T.key[s];
        if (cur == ob) return s;
        if (cur == -1) {
            const int prev = atomicCAS(&T.key[s], -1, ob);
            if (prev == -1 || prev == ob) return s;
        }
    }
    return -1;
}

// Runs of one o-bin across the lanes of a wave: whether this lane starts
// one, and lim = the lanes of its run inside its row of 16 lanes, from this
// lane on (for a segmented maximum by DPP row shifts of 1, 2, 4 and 8).
__device__ __forceinline__ int row_lim(int mob, int lane, bool& head) {
    const int prev_mob = __shfl_up(mob, 1);
    head = lane == 0 || prev_mob != mob;
    const uint64_t heads = __ballot(head);
    const uint64_t after = heads & ~lanes_le(lane);
    const int seg1 = after ? __ffsll((long long)after) - 1 : 64;
    const int rl = lane & 15;
    return min(seg1, lane - rl + 16) - lane;
}

__device__ __forceinline__ long long row_sum64(long long v, int lim) {
    long long u = dpp_move64<kRowShl1>(v);
    if (1 < lim) v += u;
    u = dpp_move64<kRowShl2>(v);
    if (2 < lim) v += u;
    u = dpp_move64<kRowShl4>(v);
    if (4 < lim) v += u;
    u = dpp_move64<kRowShl8>(v);
    if (8 < lim) v += u;
    return v;
}

__device__ __forceinline__ uint32_t row_sum32(uint32_t v, int lim) {
    uint32_t u = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowShl1, 0xF, 0xF, false);
    if (1 < lim) v += u;
    u = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowShl2, 0xF, 0xF, false);
    if (2 < lim) v += u;
    u = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowShl4, 0xF, 0xF, false);
    if (4 < lim) v += u;
    u = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowShl8, 0xF, 0xF, false);
    if (8 < lim) v += u;
    return v;
}

__device__ __forceinline__ int row_max32(int v, int lim) {
    int u = __builtin_amdgcn_mov_dpp(v, kRowShl1, 0xF, 0xF, false);
    if (1 < lim) v = max(v, u);
    u = __builtin_amdgcn_mov_dpp(v, kRowShl2, 0xF, 0xF, false);
    if (2 < lim) v = max(v, u);
    u = __builtin_amdgcn_mov_dpp(v, kRowShl4, 0xF, 0xF, false);
    if (4 < lim) v = max(v, u);
    u = __builtin_amdgcn_mov_dpp(v, kRowShl8, 0xF, 0xF, false);
    if (8 < lim) v = max(v, u);
    return v;
}

// Unambiguous pairs (each the other's closest candidate) scatter; every
// particle moves and meets the walls; global sums; with moments, the first
// pass of the exact o-bin sums (see ObAcc): the exponent maxima, and each
// particle's collider flag and virial terms for the moment pass.  Each lane
// takes kMoveRec consecutive records (a lane keeps its run's maxima in
// registers and touches the work-group's o-bin table only when the o-bin
// changes; the next record is loaded while the current one is processed).
// Since the moment sums moved to their own pass, one record per lane is the
// fastest: move and moment pass 0.66 ms on the 16M Sedov blast against 0.75
// and 0.97 ms with two and four records per lane, with the same order on
// the Noh implosion and the Sod tube.
constexpr int kMoveRec = 1;
constexpr int kMoveLanes = kBlock / kMoveRec;

// A lane's run maxima and counts of one o-bin into the work-group table, or
// straight into the global accumulators when the table is full.
template <typename real>
__device__ __forceinline__ void exp_flush(ExpTable& tab, const StepArgs<real>& a, int ob, const int* e, uint32_t cnt,
                                          uint32_t coll) {
    const int slot = table_slot(tab, ob);
    int* d = slot >= 0 ? tab.e[slot] : nullptr;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!e[k]) continue;
        if (d) atomicMax(d + k, e[k]);
        else atomicMax(&a.macc[ob].e[k], e[k]);
    }
    if (d) {
        if (cnt) atomicAdd(&tab.n[slot][0], cnt);
        if (coll) atomicAdd(&tab.n[slot][1], coll);
    } else if (cnt) {
        atomicAdd(&a.macc[ob].nc, (unsigned long long)cnt | ((unsigned long long)coll << 32));
    }
}

template <typename real>
__global__ void __launch_bounds__(kMoveLanes) k_move(StepArgs<real> a) {
    __shared__ ExpTable tab;
    __shared__ double red[kMoveLanes / 64][11];
    // Consecutive work-groups on one XCD: partners' records and keys, a few
    // c-bins away in record order, are then mostly in that XCD's L2.
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const Blk bt = a.blk[lb];
    const Inst<real>& I = a.inst[bt.inst];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t end = I.off + I.cnt;
    const bool reorder = (I.flags & TPKMC_ALLOW_REORDER) != 0;
    const bool has_mass = (I.flags & kHasMass) != 0;
    if (a.macc) {
        for (int t = tid; t < kSlots; t += kMoveLanes) {
            tab.key[t] = -1;
            for (int k = 0; k < 4; ++k) tab.e[t][k] = 0;
            tab.n[t][0] = tab.n[t][1] = 0;
        }
        __syncthreads();
    }
    double gpx = 0, gpy = 0, gpz = 0, gek = 0, gvm = 0, gvir = 0, gm = 0, galive = 0, gpairs = 0, gabs = 0, ghave = 0;
    int mob = -1;                              // o-bin of the run
    double sh[3] = {0.0, 0.0, 0.0};            // its velocity shift
    int me[4] = {0, 0, 0, 0};                  // its exponent maxima per kind
    uint32_t mcnt = 0, mcoll = 0;              // its particles and colliders
    // The next record and its partner key are loaded while the current one
    // is processed (two records in flight per lane).
    const int64_t i_first = (int64_t)bt.first + kMoveRec * tid;
    real nx_ = 0, ny_ = 0, nz_ = 0, nvx_ = 0, nvy_ = 0, nvz_ = 0;
    uint32_t nid_ = 0, nfl_ = 0;
    int32_t npj_ = -1;
    if (i_first < end) {
        Rec<real>::load(a.rec, i_first, nx_, ny_, nz_, nid_, nvx_, nvy_, nvz_, nfl_);
        npj_ = partner_of<real>(a, i_first);
    }
#pragma unroll 1
    for (int r = 0; r < kMoveRec; ++r) {
        const int64_t i = i_first + r;
        bool emit = false;
        uint32_t emit_a = 0, emit_b = 0;
        const real x = nx_, y = ny_, z = nz_, vx = nvx_, vy = nvy_, vz = nvz_;
        const uint32_t idi = nid_, fl = nfl_;
        const int32_t j_pre = npj_;
        if (r + 1 < kMoveRec && i + 1 < end) {
            Rec<real>::load(a.rec, i + 1, nx_, ny_, nz_, nid_, nvx_, nvy_, nvz_, nfl_);
            npj_ = partner_of<real>(a, i + 1);
        }
        if (i < end) {
            const int64_t dst = reorder ? i : (int64_t)a.src[i];
            const bool alive = (fl & 1u) != 0;
            if (!alive) {
                if (reorder) {
                    a.x[dst] = x; a.y[dst] = y; a.z[dst] = z;
                    a.vx[dst] = vx; a.vy[dst] = vy; a.vz[dst] = vz;
                    a.id[dst] = idi;
                    if (a.alive) a.alive[dst] = 0;
                    if (has_mass) a.mass[dst] = a.rmass[i];
                }
            } else {
                const real dt = I.dt;
                const real mi = has_mass ? a.rmass[i] : I.mass;
                const int32_t j = j_pre;
                bool mutual = j >= 0 && partner_of<real>(a, j) == (int32_t)i;
                ghave += j >= 0 ? 1.0 : 0.0;
                real nx = x, ny = y, nz = z, nvx = vx, nvy = vy, nvz = vz;
                double virx = 0, viry = 0, virz = 0;
                const bool random_pairs = (I.flags & TPKMC_PAIR_RANDOM) != 0;
                real xj = 0, yj = 0, zj = 0, vxj = 0, vyj = 0, vzj = 0;
                uint32_t idj = 0, flj = 0;
                if (mutual) {
                    Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
                    if (random_pairs)
                        mutual = random_pair_collides(a, I, x, y, z, idi, vx, vy, vz, idj, vxj, vyj, vzj);
                }
                if (mutual) {
                    const bool isA = idi < idj;
                    // Pair quantities with A = lower id, B = higher id.
                    const real xA = isA ? x : xj, yA = isA ? y : yj, zA = isA ? z : zj;
                    const real xB = isA ? xj : x, yB = isA ? yj : y, zB = isA ? zj : z;
                    const real vxA = isA ? vx : vxj, vyA = isA ? vy : vyj, vzA = isA ? vz : vzj;
                    const real vxB = isA ? vxj : vx, vyB = isA ? vyj : vy, vzB = isA ? vzj : vz;
                    real rx = xA - xB, ry = yA - yB, rz = zA - zB;
                    if (I.bc[0] == TPKMC_BC_PERIODIC) rx = min_image(rx, I.L[0], I.halfL[0]);
                    if (I.bc[1] == TPKMC_BC_PERIODIC) ry = min_image(ry, I.L[1], I.halfL[1]);
                    if (I.bc[2] == TPKMC_BC_PERIODIC) rz = min_image(rz, I.L[2], I.halfL[2]);
                    const real ux = vxA - vxB, uy = vyA - vyB, uz = vzA - vzB;
                    const real s0 = (rx * ux + ry * uy) + rz * uz;
                    const real vv = (ux * ux + uy * uy) + uz * uz;
                    // Random partners collide at the start of the step.
                    const real tp = random_pairs ? real(0) : -s0 / vv;
                    double nh[3];
                    pair_direction(I.seed_lo, I.seed_hi, I.step_lo, I.instance, isA ? idi : idj, isA ? idj : idi,
                                   (I.flags & TPKMC_PLANAR) != 0, nh);
                    // Centre-of-mass velocity and relative speed g kept, outgoing
                    // directions opposite along nhat.  Equal masses: the mean
                    // velocity, each moving g/2; masses mA, mB: the
                    // mass-weighted mean, A moving mB g / (mA + mB) and B
                    // mA g / (mA + mB).
                    const real g = sqrt(vv);
                    const real sg = isA ? real(1) : real(-1);
                    if (!has_mass) {
                        const real h = real(0.5) * g;
                        const real cmx = real(0.5) * (vxA + vxB), cmy = real(0.5) * (vyA + vyB),
                                   cmz = real(0.5) * (vzA + vzB);
                        const real hx = h * (real)nh[0], hy = h * (real)nh[1], hz = h * (real)nh[2];
                        nvx = isA ? cmx + hx : cmx - hx;
                        nvy = isA ? cmy + hy : cmy - hy;
                        nvz = isA ? cmz + hz : cmz - hz;
                    } else {
                        const real mj = a.rmass[j];
                        const real mA = isA ? mi : mj, mB = isA ? mj : mi;
                        const real M = mA + mB;
                        const real hA = (mB / M) * g, hB = (mA / M) * g;
                        const real cmx = (mA * vxA + mB * vxB) / M, cmy = (mA * vyA + mB * vyB) / M,
                                   cmz = (mA * vzA + mB * vzB) / M;
                        nvx = isA ? cmx + hA * (real)nh[0] : cmx - hB * (real)nh[0];
                        nvy = isA ? cmy + hA * (real)nh[1] : cmy - hB * (real)nh[1];
                        nvz = isA ? cmz + hA * (real)nh[2] : cmz - hB * (real)nh[2];
                    }
                    // Split move at the point of closest approach.
                    const real rest = dt - tp;
                    nx = (x + vx * tp) + nvx * rest;
                    ny = (y + vy * tp) + nvy * rest;
                    nz = (z + vz * tp) + nvz * rest;
                    // Virial: separation at closest approach (from the partner to
                    // this particle) times this particle's momentum change.
                    const real sx = sg * (rx + tp * ux), sy = sg * (ry + tp * uy), sz = sg * (rz + tp * uz);
                    virx = (double)(real(0.5) * sx * (mi * (nvx - vx)) / dt);
                    viry = (double)(real(0.5) * sy * (mi * (nvy - vy)) / dt);
                    virz = (double)(real(0.5) * sz * (mi * (nvz - vz)) / dt);
                    if (isA) {
                        gpairs += 1.0;
                        if (I.flags & TPKMC_EMIT_PAIRS) { emit = true; emit_a = idi; emit_b = idj; }
                    }
                } else {
                    nx = x + vx * dt;
                    ny = y + vy * dt;
                    nz = z + vz * dt;
                }
                // Walls, once per axis.
                bool gone = false;
                real* pos[3] = {&nx, &ny, &nz};
                real* vel[3] = {&nvx, &nvy, &nvz};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const real lo = I.lo[ax], hi = I.hi[ax], q = *pos[ax];
                    if (I.bc[ax] == TPKMC_BC_REFLECT) {
                        if (q < lo) { *pos[ax] = lo + (lo - q); *vel[ax] = -*vel[ax]; }
                        else if (q > hi) { *pos[ax] = hi - (q - hi); *vel[ax] = -*vel[ax]; }
                    } else if (I.bc[ax] == TPKMC_BC_PERIODIC) {
                        real r = q;
                        if (r < lo) r = r + I.L[ax];
                        if (r >= hi) r = r - I.L[ax];
                        *pos[ax] = r;
                    } else {
                        if (q < lo || q >= hi) gone = true;
                    }
                }
                a.x[dst] = nx; a.y[dst] = ny; a.z[dst] = nz;
                a.vx[dst] = nvx; a.vy[dst] = nvy; a.vz[dst] = nvz;
                if (reorder) a.id[dst] = idi;
                if (reorder && has_mass) a.mass[dst] = mi;
                if (a.alive && (reorder || gone)) a.alive[dst] = gone ? 0 : 1;
                if (gone) gabs += 1.0;
                const bool fin = finite3(nx, ny, nz) && finite3(nvx, nvy, nvz) &&
                                 (!has_mass || (mi > real(0) && mi < real(INFINITY)));
                if (!gone && fin) {
                    const double m = has_mass ? (double)mi : I.mass_d;
                    const double dvx = (double)nvx, dvy = (double)nvy, dvz = (double)nvz;
                    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
                    gpx += m * dvx; gpy += m * dvy; gpz += m * dvz;
                    gek += (0.5 * m) * v2;
                    gvm = v2 > gvm ? v2 : gvm;
                    gvir += (virx + viry) + virz;
                    gm += m;
                    galive += 1.0;
                    if (a.macc) {
                        const int ob = obin_of(I, nx, ny, nz);
                        if (ob != mob) {
                            if (mob >= 0) exp_flush(tab, a, mob, me, mcnt, mcoll);
                            const double* S = a.shift + (int64_t)ob * 3;
                            sh[0] = S[0]; sh[1] = S[1]; sh[2] = S[2];
                            mob = ob;
#pragma unroll
                            for (int k = 0; k < 4; ++k) me[k] = 0;
                            mcnt = mcoll = 0;
                        }
                        mcnt += 1;
                        mcoll += mutual ? 1u : 0u;
                        double t[kAccVals];
                        moment_terms(m, dvx, dvy, dvz, sh, virx, viry, virz, t);
                        me[0] = max(me[0], exp_above(fmax(fmax(fabs(t[0]), fabs(t[1])), fabs(t[2]))));
                        me[1] = max(me[1], exp_above(fmax(fmax(t[3], t[4]), t[5])));
                        if (mutual)
                            me[2] = max(me[2], exp_above(fmax(fmax(fabs(t[6]), fabs(t[7])), fabs(t[8]))));
                        if (has_mass) me[3] = max(me[3], exp_above(t[9]));
                        a.coll[dst] = mutual ? 1 : 0;
                        if (mutual) {
                            a.vir[3 * dst] = (real)virx;
                            a.vir[3 * dst + 1] = (real)viry;
                            a.vir[3 * dst + 2] = (real)virz;
                        }
                    }
                }
            }
        }
        // Pair list: one atomic per wave and record slot.
        if (a.pairs) {
            const uint64_t em = __ballot(emit);
            if (em) {
                const int leader = __ffsll((long long)em) - 1;
                unsigned long long pos0 = 0;
                if (lane == leader) pos0 = atomicAdd(a.pair_count, (unsigned long long)__popcll(em));
                pos0 = __shfl(pos0, leader);
                if (emit) {
                    const unsigned long long pos = pos0 + __popcll(em & ((1ull << lane) - 1ull));
                    if ((int64_t)pos < a.pair_cap) {
                        a.pairs[2 * pos] = emit_a;
                        a.pairs[2 * pos + 1] = emit_b;
                    }
                }
            }
        }
    }
    if (a.macc) {
        // Consecutive lanes hold consecutive records, so their last runs come
        // in runs of one o-bin across the wave: within each row of 16 lanes
        // the run's maxima go to its first lane, which alone goes through the
        // table; then the table goes to the global maxima.
        bool head;
        const int lim = row_lim(mob, lane, head);
#pragma unroll
        for (int k = 0; k < 4; ++k) me[k] = row_max32(me[k], lim);
        mcnt = row_sum32(mcnt, lim);
        mcoll = row_sum32(mcoll, lim);
        if ((head || (lane & 15) == 0) && mob >= 0) exp_flush(tab, a, mob, me, mcnt, mcoll);
        __syncthreads();
        for (int t = tid; t < kSlots * 5; t += kMoveLanes) {
            const int slot = t / 5, k = t % 5;
            const int ob = tab.key[slot];
            if (ob < 0) continue;
            if (k < 4) {
                if (tab.e[slot][k]) atomicMax(&a.macc[ob].e[k], tab.e[slot][k]);
            } else if (tab.n[slot][0]) {
                atomicAdd(&a.macc[ob].nc,
                          (unsigned long long)tab.n[slot][0] | ((unsigned long long)tab.n[slot][1] << 32));
            }
        }
    }
    double v[11] = {gpx, gpy, gpz, gek, gvm, gvir, gm, galive, gpairs, gabs, ghave};
#pragma unroll
    for (int k = 0; k < 11; ++k) v[k] = k == 4 ? wave_reduce<true>(v[k]) : wave_reduce<false>(v[k]);
    if (kMoveLanes > 64) {
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 11; ++k) red[tid >> 6][k] = v[k];
        __syncthreads();
        if (tid == 0)
            for (int w = 1; w < kMoveLanes / 64; ++w)
#pragma unroll
                for (int k = 0; k < 11; ++k) v[k] = k == 4 ? fmax(v[k], red[w][k]) : v[k] + red[w][k];
    }
    if (tid == 0) {
        double* gp = a.gpart + (int64_t)lb * kGPart;
        gp[GP_PX] = v[0]; gp[GP_PY] = v[1]; gp[GP_PZ] = v[2]; gp[GP_EKIN] = v[3]; gp[GP_VMAX2] = v[4];
        gp[GP_VIR] = v[5]; gp[GP_MASS] = v[6]; gp[GP_ALIVE] = v[7]; gp[GP_PAIRS] = v[8]; gp[GP_ABSORBED] = v[9];
        gp[GP_HAVEBEST] = v[10];
    }
}

// Second pass of the exact o-bin sums (see ObAcc), over the step's output
// state in record order, one record per lane in the move's blocks: each
// term is rounded to its o-bin's quantum; the integers of the lanes of one
// o-bin run are summed within each row of 16 lanes, then in the
// work-group's table, then into the global accumulators.  The sums are
// integers, so none of these orders is visible.  One record per lane, with
// the block and its instance uniform over the work-group (scalar loads),
// measured fastest on the sparse 16M Sedov blast; several consecutive
// records per lane lose more to their strided loads than they save.
template <typename real>
__device__ __forceinline__ void value_flush(MomentTable& tab, const StepArgs<real>& a, int ob, const long long* q) {
    const int slot = table_slot(tab, ob);
    if (slot >= 0) {
        unsigned long long* T = reinterpret_cast<unsigned long long*>(tab.val[slot]);
#pragma unroll
        for (int k = 0; k < kAccVals; ++k)
            if (q[k]) atomicAdd(T + k, (unsigned long long)q[k]);
    } else {
        ObAcc& G = a.macc[ob];
#pragma unroll
        for (int k = 0; k < kAccVals; ++k) global_acc_add(G, k, q[k]);
    }
}

// Block-table entries per work-group of the moment pass: its table sums the
// records of each o-bin over that many entries before the global atomics
// (measured with 1, 2, 4 and 8: 3.12, 3.05, 3.08 and 3.20 ms/step on the
// 16M Sedov blast, 1.18, 1.16, 1.16 and 1.17 on the Sod 4M tube).
constexpr int kMomEntries = 2;

template <typename real>
__global__ void __launch_bounds__(kBlock) k_moments(StepArgs<real> a) {
    __shared__ MomentTable tab;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    for (int t = tid; t < kMomSlots; t += kBlock) tab.key[t] = -1;
    for (int t = tid; t < kMomSlots * kTabWords; t += kBlock) (&tab.val[0][0])[t] = 0;
    __syncthreads();
    for (int ent = 0; ent < kMomEntries; ++ent) {
        const int entry = lb * kMomEntries + ent;
        if (entry >= a.nblk) break;  // uniform
        const Blk bt = a.blk[entry];
        const Inst<real>& I = a.inst[bt.inst];
        const int64_t end = I.off + I.cnt;
        const bool reorder = (I.flags & TPKMC_ALLOW_REORDER) != 0;
        const bool has_mass = (I.flags & kHasMass) != 0;
        const int64_t i = (int64_t)bt.first + tid;
        int ob = -1;
        long long q[kAccVals];
#pragma unroll
        for (int k = 0; k < kAccVals; ++k) q[k] = 0;
        bool coll = false;
        if (i < end) {
            // The same particles as the move's moment terms: alive after the
            // step (not absorbed), finite, with a valid mass.
            const int64_t p = reorder ? i : (int64_t)a.src[i];
            const bool alive = a.alive ? a.alive[p] != 0 : true;
            const real x = a.x[p], y = a.y[p], z = a.z[p], vx = a.vx[p], vy = a.vy[p], vz = a.vz[p];
            const real mi = has_mass ? a.mass[p] : I.mass;
            const bool fin = finite3(x, y, z) && finite3(vx, vy, vz) &&
                             (!has_mass || (mi > real(0) && mi < real(INFINITY)));
            if (alive && fin) {
                ob = obin_of(I, x, y, z);
                const bool c = a.coll[p] != 0;
                double vir[3] = {0.0, 0.0, 0.0};
                if (c) {
                    vir[0] = (double)a.vir[3 * p];
                    vir[1] = (double)a.vir[3 * p + 1];
                    vir[2] = (double)a.vir[3 * p + 2];
                }
                const double m = has_mass ? (double)mi : I.mass_d;
                const double* S = a.shift + (int64_t)ob * 3;
                double t[kAccVals];
                moment_terms(m, (double)vx, (double)vy, (double)vz, S, vir[0], vir[1], vir[2], t);
                // The quanta of the o-bin: its exponents and the headroom of its
                // particle count, both from the move.
                const ObAcc& G = a.macc[ob];
                const int h = acc_headroom(G.nc & 0xffffffffull);
                const double s0 = fixed_scale(G.e[0], h), s1 = fixed_scale(G.e[1], h);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    q[k] = to_fixed(t[k], s0);
                    q[3 + k] = to_fixed(t[3 + k], s1);
                }
                if (c) {
                    const double s2 = fixed_scale(G.e[2], h);
#pragma unroll
                    for (int k = 6; k < 9; ++k) q[k] = to_fixed(t[k], s2);
                }
                if (has_mass) q[9] = to_fixed(t[9], fixed_scale(G.e[3], h));
                coll = c;
            }
        }
        bool head;
        const int lim = row_lim(ob, lane, head);
        const bool anyc = __ballot(coll) != 0;
#pragma unroll
        for (int k = 0; k < kAccVals; ++k) {
            if ((k >= 6 && k <= 8 && !anyc) || (k == 9 && !has_mass)) continue;  // wave-uniform
            q[k] = row_sum64(q[k], lim);
        }
        if ((head || (lane & 15) == 0) && ob >= 0) value_flush(tab, a, ob, q);
    }
    __syncthreads();
    // The table to the global sums: one thread per (slot, value).
    for (int t = tid; t < kMomSlots * kTabWords; t += kBlock) {
        const int slot = t / kTabWords, wd = t % kTabWords;
        const int o = tab.key[slot];
        if (o >= 0) global_acc_add(a.macc[o], wd, tab.val[slot][wd]);
    }
}

// Per instance, from the work-group maxima of |v|^2 left by the key kernel:
// the step's largest speed (with split c-bins it bounds the fast particles'
// reach in the search); with ADAPTIVE_DT the time step of Sec. 3,
// dt = dx / v_max (dx of the configured c-bins), the caller's dt being the
// cap.  gridDim.x work-groups per instance fold the maxima into a running
// maximum (a single work-group would wait on its loads one after another);
// the last to arrive writes the instance's quantities for the later kernels.
template <typename real>
__global__ void __launch_bounds__(256) k_prep(Inst<real>* inst, const double* gpart) {
    __shared__ double lds[16];
    __shared__ bool last;
    Inst<real>& I = inst[blockIdx.y];
    if (!(I.flags & (TPKMC_ADAPTIVE_DT | kSplit))) return;  // whole work-group
    double v = 0.0;
    const double* g0 = gpart + (int64_t)I.blk0 * kGPart;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < I.nblk; b += gridDim.x * blockDim.x)
        v = fmax(v, g0[(int64_t)b * kGPart + GP_VMAX0]);
    v = block_max(v, lds);
    if (threadIdx.x == 0) {
        // Non-negative doubles order like their bit patterns.
        atomicMax(&I.run_v2, (unsigned long long)__double_as_longlong(v));
        __threadfence();
        last = atomicAdd(&I.prep_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    const double vmax2 = __longlong_as_double((long long)atomicExch(&I.run_v2, 0ull));
    atomicExch(&I.prep_done, 0u);
    I.vmax2_d = vmax2;
    if (I.flags & TPKMC_ADAPTIVE_DT) {
        double dt = I.dt_cap;
        if (I.dx_d > 0.0 && vmax2 > 0.0) {
            const double t = I.dx_d / sqrt(vmax2);
            if (t < dt) dt = t;
        }
        I.dt_d = dt;
        I.dt = (real)dt;
    }
}

// Tuning statistics of the speeds: per work-group, over the live particles
// with a finite state, the sum of |v|^2, their count, and the sum of |v|^2
// over those with |v|^2 above the instance's vc2 (0 when vc2 is 0), in the
// slots GP_PX, GP_PY and GP_PZ (free until the move writes them).
template <typename real>
__global__ void __launch_bounds__(kBlock) k_speed_stats(StepArgs<real> a) {
    __shared__ double lds[16];
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t p = (int64_t)bt.first + threadIdx.x;
    double v2 = 0.0, n = 0.0, hot = 0.0;
    if (p < I.off + I.cnt && (a.alive == nullptr || a.alive[p] != 0)) {
        const double vx = (double)a.vx[p], vy = (double)a.vy[p], vz = (double)a.vz[p];
        if (finite3((double)a.x[p], (double)a.y[p], (double)a.z[p]) && finite3(vx, vy, vz)) {
            v2 = speed2(vx, vy, vz);
            n = 1.0;
            hot = I.vc2 > real(0) && v2 > (double)I.vc2 ? v2 : 0.0;
        }
    }
    v2 = block_sum(v2, lds);
    n = block_sum(n, lds);
    hot = block_sum(hot, lds);
    if (threadIdx.x == 0) {
        a.gpart[(int64_t)blockIdx.x * kGPart + GP_PX] = v2;
        a.gpart[(int64_t)blockIdx.x * kGPart + GP_PY] = n;
        a.gpart[(int64_t)blockIdx.x * kGPart + GP_PZ] = hot;
    }
}

// ---------------------------------------------------------------- launchers
template <typename real>
void launch_key(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_key<real>, dim3(a.nblk), dim3(kWave), 0, s, a);
}
template <typename real>
void launch_scatter(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}
template <typename real>
void launch_prep(Inst<real>* inst, const double* gpart, int n_inst, int max_nblk, hipStream_t s) {
    const int gx = std::max(1, std::min(64, (max_nblk + 1023) / 1024));
    hipLaunchKernelGGL(k_prep<real>, dim3(gx, n_inst), dim3(256), 0, s, inst, gpart);
}
template <typename real>
void launch_speed_stats(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_speed_stats<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}
template <typename real>
void launch_search(const StepArgs<real>& a, int block, int group, hipStream_t s) {
    constexpr bool half = std::is_same<real, float>::value;
    const int lanes = kBlock / group;
    const int bs = block < lanes ? block : lanes;
    const unsigned grid = (unsigned)a.nblk * (unsigned)(lanes / bs);
    const size_t lds = half ? (size_t)(bs / kWave) * kStageBytesPerWave : 0;  // staging buffers
    if (group == 4) hipLaunchKernelGGL((k_search<real, half, 4>), dim3(grid), dim3(bs), lds, s, a);
    else if (group == 2) hipLaunchKernelGGL((k_search<real, half, 2>), dim3(grid), dim3(bs), lds, s, a);
    else hipLaunchKernelGGL((k_search<real, half, 1>), dim3(grid), dim3(bs), lds, s, a);
}
template <typename real>
void launch_search_mix(const StepArgs<real>& a, int block, int n_inst, bool split, hipStream_t s) {
    constexpr bool half = std::is_same<real, float>::value;
    const int lanes = kBlock / 2;
    const int bs = block < lanes ? block : lanes;
    const unsigned grid = (unsigned)a.nblk * (unsigned)(lanes / bs);
    const size_t lds = half ? (size_t)(bs / kWave) * kStageBytesPerWave : 0;
    hipLaunchKernelGGL((k_search<real, half, 2, true>), dim3(grid), dim3(bs), lds, s, a);
    if (split) {
        const unsigned fg = (unsigned)std::max(1, std::min(2048, a.nblk));
        hipLaunchKernelGGL((k_search_fast<real, half, true>), dim3(fg), dim3(256), 0, s, a, n_inst);
    }
}
template <typename real>
void launch_search_fast(const StepArgs<real>& a, int n_inst, hipStream_t s) {
    constexpr bool half = std::is_same<real, float>::value;
    const unsigned fg = (unsigned)std::max(1, std::min(2048, a.nblk));
    hipLaunchKernelGGL((k_search_fast<real, half>), dim3(fg), dim3(256), 0, s, a, n_inst);
}
template <typename real>
void launch_random_pairs(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_rp_key<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rp_rank<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rp_partner<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}
template <typename real>
void launch_move(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_move<real>, dim3(a.nblk), dim3(kMoveLanes), 0, s, a);
}
template <typename real>
void launch_moments(const StepArgs<real>& a, hipStream_t s) {
    const unsigned grid = (unsigned)((a.nblk + kMomEntries - 1) / kMomEntries);
    hipLaunchKernelGGL(k_moments<real>, dim3(grid), dim3(kBlock), 0, s, a);
}

}  // namespace tpkmc
