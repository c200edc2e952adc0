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

#include "tpkmc_internal.h"

namespace tpkmc {

// ---------------------------------------------------------------- records
// Record layout: x y z id | vx vy vz flags (8 reals).  flags bit 0 = alive.
template <typename real> struct Rec;

template <> struct Rec<float> {
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

// ---------------------------------------------------------------- helpers
// Bin along one axis: floor((x - lo) * n / L) clamped into [0, n - 1].
template <typename real>
__device__ __forceinline__ int axis_bin(real x, real lo, real inv_w, int n) {
    real t = (x - lo) * inv_w;
    if (!(t >= real(0))) return 0;
    if (t >= real(n)) return n - 1;
    return (int)t;
}

template <typename real>
__device__ __forceinline__ bool finite3(real a, real b, real c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ __forceinline__ uint64_t lanes_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Sum of an int over the work-group (blockDim.x <= 1024), result in all threads.
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

// Work-groups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD (own L2) receives a contiguous range of the table, where neighbouring
// work-groups share neighbour c-bins.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int nx = 8;
    const int xcd = bid % nx, local = bid / nx;
    const int per = nb / nx, rem = nb % nx;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
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

// Isotropic unit vector of the pair (idA < idB): Marsaglia's rejection method
// on two 53-bit uniforms per Philox draw; computed in double in both modes.
__device__ __forceinline__ void pair_direction(uint32_t k0, uint32_t k1, uint32_t step, uint32_t instance,
                                               uint32_t idA, uint32_t idB, double n[3]) {
    for (uint32_t attempt = 0; attempt < 256u; ++attempt) {
        uint32_t c[4] = {step, idA, idB, (instance << 8) | attempt};
        philox4x32_10(c, k0, k1);
        const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
        const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * (1.0 / 9007199254740992.0);
        const double x1 = 2.0 * u1 - 1.0;
        const double x2 = 2.0 * u2 - 1.0;
        const double s = x1 * x1 + x2 * x2;
        if (s < 1.0) {
            const double q = sqrt(1.0 - s);
            n[0] = (2.0 * x1) * q;
            n[1] = (2.0 * x2) * q;
            n[2] = 1.0 - 2.0 * s;
            return;
        }
    }
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
}

// ---------------------------------------------------------------- 1. key
// c-bin of every caller-order particle and its rank inside the c-bin.  Lanes
// of a wave holding the same c-bin in a run (the common case for sorted input)
// take one atomic for the whole run.
template <typename real>
__global__ void __launch_bounds__(kBlock) k_key(StepArgs<real> a) {
    __shared__ double lds[16];
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t p = (int64_t)bt.first + threadIdx.x;
    const bool in = p < I.off + I.cnt;
    int key = 0, fast = 0, nonfin = 0;
    if (in) {
        const bool alive = a.alive ? a.alive[p] != 0 : true;
        const real x = a.x[p], y = a.y[p], z = a.z[p];
        const real vx = a.vx[p], vy = a.vy[p], vz = a.vz[p];
        const bool fin = finite3(x, y, z) && finite3(vx, vy, vz);
        if (alive && fin) {
            const int cx = axis_bin(x, I.lo[0], I.inv_w[0], I.n[0]);
            const int cy = axis_bin(y, I.lo[1], I.inv_w[1], I.n[1]);
            const int cz = axis_bin(z, I.lo[2], I.inv_w[2], I.n[2]);
            key = (int)I.cell_off + cx + I.n[0] * (cy + I.n[1] * cz);
            fast = (fabs(vx) * I.dt > I.w[0]) || (fabs(vy) * I.dt > I.w[1]) || (fabs(vz) * I.dt > I.w[2]);
        } else {
            key = (int)(I.cell_off + I.C);
            nonfin = alive && !fin;
        }
    }
    const int lane = threadIdx.x & 63;
    const uint64_t active = __ballot(in);
    const int prev = __shfl_up(key, 1);
    const bool head = in && (lane == 0 || prev != key);
    const uint64_t heads = __ballot(head);
    const int seg0 = 63 - __clzll((long long)(heads & lanes_le(lane)));
    const uint64_t above = heads & ~lanes_le(lane);
    const int nact = __popcll(active);
    const int seg1 = above ? (__ffsll((long long)above) - 1) : nact;
    int base = 0;
    if (head) base = atomicAdd(&a.start[key], seg1 - seg0);
    base = __shfl(base, seg0 < 0 ? 0 : seg0);
    if (in) {
        a.key[p] = key;
        a.rank[p] = base + (lane - seg0);
    }
    const double nf = block_sum((double)fast, lds);
    const double nn = block_sum((double)nonfin, lds);
    if (threadIdx.x == 0) {
        double* gp = a.gpart + (int64_t)blockIdx.x * kGPart;
        gp[GP_FAST] = nf;
        gp[GP_NONFINITE] = nn;
        // The search kernel may accumulate into these with atomics.
        gp[GP_TESTS2] = 0.0;
        gp[GP_CAND] = 0.0;
        gp[GP_HAVEBEST] = 0.0;
    }
}

// ---------------------------------------------------------------- 3. scatter
// Caller-order particle -> its c-bin-ordered record.
template <typename real>
__global__ void __launch_bounds__(kBlock) k_scatter(StepArgs<real> a) {
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t p = (int64_t)bt.first + threadIdx.x;
    if (p >= I.off + I.cnt) return;
    const int64_t base = I.off - a.start[I.cell_off];
    const int k = a.key[p];
    const int64_t dst = base + a.start[k] + a.rank[p];
    const uint32_t fl = a.alive ? (a.alive[p] != 0) : 1u;
    Rec<real>::store(a.rec, dst, a.x[p], a.y[p], a.z[p], a.id[p], a.vx[p], a.vy[p], a.vz[p], fl);
    a.src[dst] = (int32_t)p;
}

// ---------------------------------------------------------------- 4. search
// Neighbourhood of c-bin (cx, cy, cz) as contiguous record ranges.
struct Ranges {
    int ny, nz, nxr;
    int ys[3], zs[3];
    int xlo[2], xhi[2];
};

__device__ __forceinline__ void axis_set(int c, int n, int bc, int out[3], int& cnt) {
    if (bc == TPKMC_BC_PERIODIC) {
        if (n <= 3) {
            cnt = n;
            for (int k = 0; k < n; ++k) out[k] = k;
        } else {
            cnt = 3;
            out[0] = c == 0 ? n - 1 : c - 1;
            out[1] = c;
            out[2] = c == n - 1 ? 0 : c + 1;
        }
    } else {
        cnt = 0;
        for (int d = -1; d <= 1; ++d) {
            const int v = c + d;
            if (v >= 0 && v < n) out[cnt++] = v;
        }
    }
}

__device__ __forceinline__ void x_ranges(int c, int n, int bc, Ranges& R) {
    if (bc == TPKMC_BC_PERIODIC && n > 3 && (c == 0 || c == n - 1)) {
        R.nxr = 2;
        if (c == 0) { R.xlo[0] = 0; R.xhi[0] = 1; R.xlo[1] = n - 1; R.xhi[1] = n - 1; }
        else { R.xlo[0] = 0; R.xhi[0] = 0; R.xlo[1] = n - 2; R.xhi[1] = n - 1; }
    } else if (bc == TPKMC_BC_PERIODIC && n <= 3) {
        R.nxr = 1; R.xlo[0] = 0; R.xhi[0] = n - 1;
    } else {
        R.nxr = 1;
        R.xlo[0] = c > 0 ? c - 1 : 0;
        R.xhi[0] = c < n - 1 ? c + 1 : n - 1;
    }
}

// The three criteria for the ordered pair (i, j), in the operation order of
// the reference: chi < 0 within the step, d_min^2 <= D^2.  Returns d_min^2 or
// a negative value when j is not a candidate.
template <typename real>
__device__ __forceinline__ real pair_d2(const Inst<real>& I, real xi, real yi, real zi, real vxi, real vyi,
                                        real vzi, real xj, real yj, real zj, real vxj, real vyj, real vzj) {
    real rx = xi - xj, ry = yi - yj, rz = zi - zj;
    if (I.bc[0] == TPKMC_BC_PERIODIC) { if (rx > I.halfL[0]) rx = rx - I.L[0]; else if (rx < -I.halfL[0]) rx = rx + I.L[0]; }
    if (I.bc[1] == TPKMC_BC_PERIODIC) { if (ry > I.halfL[1]) ry = ry - I.L[1]; else if (ry < -I.halfL[1]) ry = ry + I.L[1]; }
    if (I.bc[2] == TPKMC_BC_PERIODIC) { if (rz > I.halfL[2]) rz = rz - I.L[2]; else if (rz < -I.halfL[2]) rz = rz + I.L[2]; }
    const real ux = vxi - vxj, uy = vyi - vyj, uz = vzi - vzj;
    const real s0 = (rx * ux + ry * uy) + rz * uz;
    if (!(s0 < real(0))) return real(-1);
    const real vv = (ux * ux + uy * uy) + uz * uz;
    const real s1 = s0 + vv * I.dt;
    if (!(s1 > real(0))) return real(-1);
    const real tp = -s0 / vv;
    const real px = rx + tp * ux, py = ry + tp * uy, pz = rz + tp * uz;
    const real d2 = (px * px + py * py) + pz * pz;
    if (!(d2 <= I.D2)) return real(-1);
    return d2;
}

// Closest candidate of every live record (one lane per record, ordered
// pairs: each lane scans the whole neighbourhood, so no atomics and the
// choice does not depend on the order of records inside a c-bin).
template <typename real>
__global__ void __launch_bounds__(256) k_search(StepArgs<real> a) {
    __shared__ double lds[16];
    const int sub = kBlock / blockDim.x;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int entry = lb / sub;
    const Blk bt = a.blk[entry];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t i = (int64_t)bt.first + (int64_t)(lb % sub) * blockDim.x + threadIdx.x;
    const int64_t base = I.off - a.start[I.cell_off];
    const int64_t live_end = base + a.start[I.cell_off + I.C];
    double tests = 0.0, cand = 0.0, have = 0.0;
    if (i < live_end && i < I.off + I.cnt) {
        real xi, yi, zi, vxi, vyi, vzi;
        uint32_t idi, fl;
        Rec<real>::load(a.rec, i, xi, yi, zi, idi, vxi, vyi, vzi, fl);
        const int cx = axis_bin(xi, I.lo[0], I.inv_w[0], I.n[0]);
        const int cy = axis_bin(yi, I.lo[1], I.inv_w[1], I.n[1]);
        const int cz = axis_bin(zi, I.lo[2], I.inv_w[2], I.n[2]);
        Ranges R;
        axis_set(cy, I.n[1], I.bc[1], R.ys, R.ny);
        axis_set(cz, I.n[2], I.bc[2], R.zs, R.nz);
        x_ranges(cx, I.n[0], I.bc[0], R);
        int64_t bj = -1;
        real bd2 = real(0);
        uint32_t bid = 0;
        int64_t seen = 0;
        int ncand = 0;
        for (int iz = 0; iz < R.nz; ++iz) {
            for (int iy = 0; iy < R.ny; ++iy) {
                const int64_t row = I.cell_off + (int64_t)I.n[0] * (R.ys[iy] + (int64_t)I.n[1] * R.zs[iz]);
                for (int ix = 0; ix < R.nxr; ++ix) {
                    const int64_t j0 = base + a.start[row + R.xlo[ix]];
                    const int64_t j1 = base + a.start[row + R.xhi[ix] + 1];
                    seen += j1 - j0;
                    for (int64_t j = j0; j < j1; ++j) {
                        if (j == i) continue;
                        real xj, yj, zj, vxj, vyj, vzj;
                        uint32_t idj, flj;
                        Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
                        const real d2 = pair_d2(I, xi, yi, zi, vxi, vyi, vzi, xj, yj, zj, vxj, vyj, vzj);
                        if (d2 >= real(0)) {
                            ++ncand;
                            if (bj < 0 || d2 < bd2 || (d2 == bd2 && idj < bid)) {
                                bj = j; bd2 = d2; bid = idj;
                            }
                        }
                    }
                }
            }
        }
        a.best[i] = (int32_t)bj;
        tests = (double)(seen - 1);
        cand = (double)ncand;
        have = bj >= 0 ? 1.0 : 0.0;
    } else if (i < I.off + I.cnt) {
        a.best[i] = -1;
    }
    const double t = block_sum(tests, lds);
    const double c = block_sum(cand, lds);
    const double h = block_sum(have, lds);
    if (threadIdx.x == 0) {
        double* gp = a.gpart + (int64_t)entry * kGPart;
        if (sub == 1) {
            gp[GP_TESTS2] = t; gp[GP_CAND] = c; gp[GP_HAVEBEST] = h;
        } else {
            unsafeAtomicAdd(gp + GP_TESTS2, t);
            unsafeAtomicAdd(gp + GP_CAND, c);
            unsafeAtomicAdd(gp + GP_HAVEBEST, h);
        }
    }
}

// ---------------------------------------------------------------- 5. move
// Unambiguous pairs (each the other's closest candidate) scatter; every
// particle moves and meets the walls; o-bin moments and global sums.
template <typename real>
__global__ void __launch_bounds__(kBlock) k_move(StepArgs<real> a) {
    __shared__ double lds[16];
    const Blk bt = a.blk[blockIdx.x];
    const Inst<real>& I = a.inst[bt.inst];
    const int64_t i = (int64_t)bt.first + threadIdx.x;
    const bool in = i < I.off + I.cnt;
    const bool reorder = (I.flags & TPKMC_ALLOW_REORDER) != 0;
    double gpx = 0, gpy = 0, gpz = 0, gek = 0, gvm = 0, gvir = 0, gm = 0, galive = 0, gpairs = 0, gabs = 0;
    bool emit = false;
    uint32_t emit_a = 0, emit_b = 0;
    if (in) {
        real x, y, z, vx, vy, vz;
        uint32_t idi, fl;
        Rec<real>::load(a.rec, i, x, y, z, idi, vx, vy, vz, fl);
        const int64_t dst = reorder ? i : (int64_t)a.src[i];
        const bool alive = (fl & 1u) != 0;
        if (!alive) {
            if (reorder) {
                a.x[dst] = x; a.y[dst] = y; a.z[dst] = z;
                a.vx[dst] = vx; a.vy[dst] = vy; a.vz[dst] = vz;
                a.id[dst] = idi;
                if (a.alive) a.alive[dst] = 0;
            }
        } else {
            const real dt = I.dt;
            const int32_t j = a.best[i];
            const bool mutual = j >= 0 && a.best[j] == (int32_t)i;
            real nx = x, ny = y, nz = z, nvx = vx, nvy = vy, nvz = vz;
            double virx = 0, viry = 0, virz = 0;
            if (mutual) {
                real xj, yj, zj, vxj, vyj, vzj;
                uint32_t idj, flj;
                Rec<real>::load(a.rec, j, xj, yj, zj, idj, vxj, vyj, vzj, flj);
                const bool isA = idi < idj;
                // Pair quantities with A = lower id, B = higher id.
                const real xA = isA ? x : xj, yA = isA ? y : yj, zA = isA ? z : zj;
                const real xB = isA ? xj : x, yB = isA ? yj : y, zB = isA ? zj : z;
                const real vxA = isA ? vx : vxj, vyA = isA ? vy : vyj, vzA = isA ? vz : vzj;
                const real vxB = isA ? vxj : vx, vyB = isA ? vyj : vy, vzB = isA ? vzj : vz;
                real rx = xA - xB, ry = yA - yB, rz = zA - zB;
                if (I.bc[0] == TPKMC_BC_PERIODIC) { if (rx > I.halfL[0]) rx = rx - I.L[0]; else if (rx < -I.halfL[0]) rx = rx + I.L[0]; }
                if (I.bc[1] == TPKMC_BC_PERIODIC) { if (ry > I.halfL[1]) ry = ry - I.L[1]; else if (ry < -I.halfL[1]) ry = ry + I.L[1]; }
                if (I.bc[2] == TPKMC_BC_PERIODIC) { if (rz > I.halfL[2]) rz = rz - I.L[2]; else if (rz < -I.halfL[2]) rz = rz + I.L[2]; }
                const real ux = vxA - vxB, uy = vyA - vyB, uz = vzA - vzB;
                const real s0 = (rx * ux + ry * uy) + rz * uz;
                const real vv = (ux * ux + uy * uy) + uz * uz;
                const real tp = -s0 / vv;
                double nh[3];
                pair_direction(I.seed_lo, I.seed_hi, I.step_lo, I.instance, isA ? idi : idj, isA ? idj : idi, nh);
                // Equal masses: centre-of-mass velocity kept, relative speed g
                // kept, outgoing directions opposite along nhat.
                const real g = sqrt(vv);
                const real h = real(0.5) * g;
                const real sg = isA ? real(1) : real(-1);
                const real cmx = real(0.5) * (vxA + vxB), cmy = real(0.5) * (vyA + vyB), cmz = real(0.5) * (vzA + vzB);
                const real hx = h * (real)nh[0], hy = h * (real)nh[1], hz = h * (real)nh[2];
                nvx = isA ? cmx + hx : cmx - hx;
                nvy = isA ? cmy + hy : cmy - hy;
                nvz = isA ? cmz + hz : cmz - hz;
                // Split move at the point of closest approach.
                const real rest = dt - tp;
                nx = (x + vx * tp) + nvx * rest;
                ny = (y + vy * tp) + nvy * rest;
                nz = (z + vz * tp) + nvz * rest;
                // Virial: separation at closest approach (from the partner to
                // this particle) times this particle's momentum change.
                const real sx = sg * (rx + tp * ux), sy = sg * (ry + tp * uy), sz = sg * (rz + tp * uz);
                virx = (double)(real(0.5) * sx * (I.mass * (nvx - vx)) / dt);
                viry = (double)(real(0.5) * sy * (I.mass * (nvy - vy)) / dt);
                virz = (double)(real(0.5) * sz * (I.mass * (nvz - vz)) / dt);
                if (isA) {
                    gpairs = 1.0;
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
            if (a.alive && (reorder || gone)) a.alive[dst] = gone ? 0 : 1;
            if (gone) gabs = 1.0;
            const bool fin = finite3(nx, ny, nz) && finite3(nvx, nvy, nvz);
            if (!gone && fin) {
                const double m = I.mass_d;
                const double dvx = (double)nvx, dvy = (double)nvy, dvz = (double)nvz;
                const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
                gpx = m * dvx; gpy = m * dvy; gpz = m * dvz;
                gek = (0.5 * m) * v2;
                gvm = v2;
                gvir = (virx + viry) + virz;
                gm = m;
                galive = 1.0;
                if (a.moments) {
                    const int bx = axis_bin(nx, I.lo[0], I.inv_wo[0], I.no[0]);
                    const int by = axis_bin(ny, I.lo[1], I.inv_wo[1], I.no[1]);
                    const int bz = axis_bin(nz, I.lo[2], I.inv_wo[2], I.no[2]);
                    const int64_t ob = I.obin_off + bx + (int64_t)I.no[0] * (by + (int64_t)I.no[1] * bz);
                    double* M = a.moments + ob * TPKMC_MOMENT_STRIDE;
                    const double* S = a.shift + ob * 3;
                    const double ex = dvx - S[0], ey = dvy - S[1], ez = dvz - S[2];
                    unsafeAtomicAdd(M + 0, 1.0);
                    unsafeAtomicAdd(M + 1, m * ex);
                    unsafeAtomicAdd(M + 2, m * ey);
                    unsafeAtomicAdd(M + 3, m * ez);
                    unsafeAtomicAdd(M + 4, m * ex * ex);
                    unsafeAtomicAdd(M + 5, m * ey * ey);
                    unsafeAtomicAdd(M + 6, m * ez * ez);
                    if (mutual) {
                        unsafeAtomicAdd(M + 7, virx);
                        unsafeAtomicAdd(M + 8, viry);
                        unsafeAtomicAdd(M + 9, virz);
                        unsafeAtomicAdd(M + 10, 1.0);
                    }
                }
            }
        }
    }
    // Pair list: one atomic per wave.
    if (a.pairs) {
        const uint64_t em = __ballot(emit);
        if (em) {
            const int lane = threadIdx.x & 63;
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
    double* gp = a.gpart + (int64_t)blockIdx.x * kGPart;
    const double r0 = block_sum(gpx, lds);
    const double r1 = block_sum(gpy, lds);
    const double r2 = block_sum(gpz, lds);
    const double r3 = block_sum(gek, lds);
    const double r4 = block_max(gvm, lds);
    const double r5 = block_sum(gvir, lds);
    const double r6 = block_sum(gm, lds);
    const double r7 = block_sum(galive, lds);
    const double r8 = block_sum(gpairs, lds);
    const double r9 = block_sum(gabs, lds);
    if (threadIdx.x == 0) {
        gp[GP_PX] = r0; gp[GP_PY] = r1; gp[GP_PZ] = r2; gp[GP_EKIN] = r3; gp[GP_VMAX2] = r4;
        gp[GP_VIR] = r5; gp[GP_MASS] = r6; gp[GP_ALIVE] = r7; gp[GP_PAIRS] = r8; gp[GP_ABSORBED] = r9;
    }
}

// ---------------------------------------------------------------- launchers
template <typename real>
void launch_key(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_key<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}
template <typename real>
void launch_scatter(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}
template <typename real>
void launch_search(const StepArgs<real>& a, int block, hipStream_t s) {
    const int sub = kBlock / block;
    hipLaunchKernelGGL(k_search<real>, dim3(a.nblk * sub), dim3(block), 0, s, a);
}
template <typename real>
void launch_move(const StepArgs<real>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_move<real>, dim3(a.nblk), dim3(kBlock), 0, s, a);
}

}  // namespace tpkmc
