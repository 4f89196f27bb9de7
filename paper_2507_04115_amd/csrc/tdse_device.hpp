// tdse_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// complex fp64 arithmetic, wavefront shuffles and reductions, the cross-lane
// carry scans of the partitioned tridiagonal solve, and the Crank-Nicolson
// core that every kernel (forward, ground state, adjoint) runs per time step.
#pragma once
#include "tdse_internal.hpp"

namespace tdse {

// ------------------------------------------------------------ complex fp64
__device__ __forceinline__ cd mkc(double r, double i)
{
    cd z;
    z.re = r;
    z.im = i;
    return z;
}
__device__ __forceinline__ cd czero() { return mkc(0.0, 0.0); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return mkc(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cd cmul(cd a, cd b)
{
    return mkc(fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re));
}
// a * b + c
__device__ __forceinline__ cd cmad(cd a, cd b, cd c)
{
    return mkc(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}
__device__ __forceinline__ cd cscale(double s, cd a) { return mkc(s * a.re, s * a.im); }
__device__ __forceinline__ double cabs2(cd a) { return fma(a.re, a.re, a.im * a.im); }
__device__ __forceinline__ cd cconj(cd a) { return mkc(a.re, -a.im); }
__device__ __forceinline__ cd cinv(cd a)
{
    double s = 1.0 / fma(a.re, a.re, a.im * a.im);
    return mkc(a.re * s, -a.im * s);
}

__device__ __forceinline__ cd ld(const cd* p) { return *p; }

// Returns x unchanged but hides its value from the optimiser.  Table indices
// are passed through it once per time step so that the loop-invariant table
// loads stay inside the time loop (streamed from cache) instead of being
// hoisted into hundreds of registers and spilled.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ cd ld_psi(const double* p, int64_t j) { return mkc(p[2 * j], p[2 * j + 1]); }

// Loads a workgroup-uniform record and moves it into scalar registers.  Work
// items arrive through LDS, so the compiler cannot prove the record uniform
// on its own; without this every table pointer would occupy vector registers.
template <class T>
__device__ __forceinline__ T uniform_load(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "uniform_load needs a 4-byte multiple");
    T out;
    const int* src = reinterpret_cast<const int*>(p);
    int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ------------------------------------------------------------ wavefront ops
__device__ __forceinline__ cd shfl_up_c(cd a, int d)
{
    return mkc(__shfl_up(a.re, d), __shfl_up(a.im, d));
}
__device__ __forceinline__ cd shfl_down_c(cd a, int d)
{
    return mkc(__shfl_down(a.re, d), __shfl_down(a.im, d));
}
// Butterfly sum over the 64 lanes.  Every lane ends with a sum; lane 0's
// association order is fixed, and only lane 0's value is ever stored, so
// results are bitwise reproducible.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Workgroup sum in fixed order (waves 0..W-1).  `slots` holds kMaxWaves
// doubles of LDS; the caller alternates slot arrays between consecutive
// reductions so one barrier per reduction suffices.
__device__ __forceinline__ double block_sum(double v, double* slots, int lane, int wave, int W)
{
    v = wave_sum(v);
    if (lane == 0) slots[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < W; ++w) s += slots[w];
    return s;
}

// ------------------------------------------------------------ lane context
struct LaneCtx {
    int lane;   // lane in wavefront
    int wave;   // wavefront in workgroup
    int W;      // wavefronts per system
    int t;      // lane index within the system (0..T-1)
    int s;      // first grid point of the lane's chunk
    double vl, vr, ml, mr, dvl, dvr;
    cd ql, bl;
    int hasmask;
};

__device__ __forceinline__ LaneCtx make_lane_ctx(const SizeClass& sc, int tid)
{
    LaneCtx c;
    c.lane = tid & (kWave - 1);
    c.wave = tid / kWave;
    c.W = sc.T / kWave;
    c.t = tid;
    c.s = tid * sc.C;
    c.vl = sc.lt.vl[tid];
    c.vr = sc.lt.vr[tid];
    c.ml = sc.lt.ml[tid];
    c.mr = sc.lt.mr[tid];
    c.dvl = sc.lt.dvl[tid];
    c.dvr = sc.lt.dvr[tid];
    c.ql = sc.lt.ql[tid];
    c.bl = sc.lt.bl[tid];
    c.hasmask = sc.lt.hasmask[tid];
    return c;
}

// ------------------------------------------------------------ carry scans
// Forward carries of z_j = r_j + alpha_j z_{j-1}.  Input: the lane's chunk-end
// value computed with a zero carry-in.  Output: the true z at the point just
// before the lane's chunk (the lane's carry-in).  In-wave Kogge-Stone over
// `levels` levels with precomputed window products, then one cross-wave
// correction through LDS; windows longer than 2^levels lanes are dropped
// only when the host has verified that their products are below 2^-56.
__device__ __forceinline__ cd scan_fwd(cd z, const SizeClass& sc, const LaneCtx& lc, cd* lds)
{
    const int T = sc.T;
#pragma unroll
    for (int lev = 0; lev < kMaxLevels; ++lev) {
        if (lev < sc.levels) {
            const int d = 1 << lev;
            cd zs = shfl_up_c(z, d);
            if (lc.lane >= d) z = cmad(ld(sc.lt.pa + lev * T + lc.t), zs, z);
        }
    }
    cd prev = czero();
    if (lc.W > 1) {
        if (lc.lane == kWave - 1) lds[lc.wave] = z;
        __syncthreads();
        const int v0 = max(0, lc.wave - sc.xwaves);
        for (int w = v0; w < lc.wave; ++w) prev = cmad(ld(sc.lt.pw + w * kWave + kWave - 1), prev, lds[w]);
        if (lc.lane < (1 << sc.levels)) z = cmad(ld(sc.lt.pw + lc.t), prev, z);
    }
    cd up = shfl_up_c(z, 1);
    return lc.lane == 0 ? prev : up;
}

// Backward carries of y_j = w_j + beta_j y_{j+1}, mirrored: returns the true y
// at the point just after the lane's chunk.
__device__ __forceinline__ cd scan_bwd(cd y, const SizeClass& sc, const LaneCtx& lc, cd* lds)
{
    const int T = sc.T;
#pragma unroll
    for (int lev = 0; lev < kMaxLevels; ++lev) {
        if (lev < sc.levels) {
            const int d = 1 << lev;
            cd ys = shfl_down_c(y, d);
            if (lc.lane + d < kWave) y = cmad(ld(sc.lt.qb + lev * T + lc.t), ys, y);
        }
    }
    cd next = czero();
    if (lc.W > 1) {
        if (lc.lane == 0) lds[lc.wave] = y;
        __syncthreads();
        const int v1 = min(lc.W - 1, lc.wave + sc.xwaves);
        for (int w = v1; w > lc.wave; --w) next = cmad(ld(sc.lt.qw + w * kWave), next, lds[w]);
        if (lc.lane > kWave - 1 - (1 << sc.levels)) y = cmad(ld(sc.lt.qw + lc.t), next, y);
    }
    cd dn = shfl_down_c(y, 1);
    return lc.lane == kWave - 1 ? next : dn;
}

// ------------------------------------------------------------ CN core
// Coefficients of the right-hand side 12 R psi with R = M2 - h A,
// A = -D2/2 + M2 diag(V):
//   12 R psi_j = (psi_{j-1} + 10 psi_j + psi_{j+1})
//                - h' (w(V_{j-1}) psi_{j-1} + d(V_j) psi_j + w(V_{j+1}) psi_{j+1})
// with w(V) = kw_a V + kw_b = 12 |h| (V/12 - 1/(2 dx^2)),
//      d(V) = kd_a V + kd_b = 12 |h| (1/dx^2 + 10 V/12),
// and h' = i (real time, h = i dt/2) or 1 (imaginary time, h = dtau/2).
struct RhsCoef {
    double kw_a, kw_b, kd_a, kd_b;
};

__host__ __device__ inline RhsCoef make_rhs_coef(double habs, double dx)
{
    RhsCoef c;
    const double k = 12.0 * habs;
    c.kw_a = k / 12.0;
    c.kw_b = -k / (2.0 * dx * dx);
    c.kd_a = k * 10.0 / 12.0;
    c.kd_b = k / (dx * dx);
    return c;
}

// Applies psi <- L^{-1} R psi (before the field phase and absorber) to the
// lane's chunk v[0..C-1] whose neighbours are gl = psi_{s-1}, gr = psi_{s+C}.
// Returns the carries cf = z_{s-1} and cb = y_{s+C} (both exact), from which
// the caller rebuilds the ghost values of the next step without exchanging
// data between lanes:  y_{s+C} = cb,  y_{s-1} = q_{s-1} cf + beta_{s-1} y_s.
template <int C, bool REALTIME>
__device__ __forceinline__ void cn_apply(cd (&v)[C], cd gl, cd gr, const SizeClass& sc,
                                         const LaneCtx& lc, const RhsCoef rc, cd* lds_f,
                                         cd* lds_b, cd& cf, cd& cb)
{
    const int T = sc.T, t = opaque(lc.t);
    // 1. right-hand side, in place
    {
        cd prev = gl;
        double wprev = fma(lc.vl, rc.kw_a, rc.kw_b);
        double v0 = sc.pt.v[t];
        double wcur = fma(v0, rc.kw_a, rc.kw_b);
        double dcur = fma(v0, rc.kd_a, rc.kd_b);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const cd cur = v[k];
            const cd nxt = (k + 1 < C) ? v[k + 1] : gr;
            const double vn = (k + 1 < C) ? sc.pt.v[(k + 1) * T + t] : lc.vr;
            const double wn = fma(vn, rc.kw_a, rc.kw_b);
            const double dn = fma(vn, rc.kd_a, rc.kd_b);
            double re = fma(10.0, cur.re, prev.re + nxt.re);
            double im = fma(10.0, cur.im, prev.im + nxt.im);
            if (REALTIME) {
                re = fma(wprev, prev.im, re);
                re = fma(dcur, cur.im, re);
                re = fma(wn, nxt.im, re);
                im = fma(-wprev, prev.re, im);
                im = fma(-dcur, cur.re, im);
                im = fma(-wn, nxt.re, im);
            } else {
                re = fma(-wprev, prev.re, re);
                re = fma(-dcur, cur.re, re);
                re = fma(-wn, nxt.re, re);
                im = fma(-wprev, prev.im, im);
                im = fma(-dcur, cur.im, im);
                im = fma(-wn, nxt.im, im);
            }
            v[k] = mkc(re, im);
            prev = cur;
            wprev = wcur;
            wcur = wn;
            dcur = dn;
        }
    }
    // 2. forward recurrence with zero carry-in
#pragma unroll
    for (int k = 1; k < C; ++k) v[k] = cmad(ld(sc.pt.alpha + k * T + t), v[k - 1], v[k]);
    // 3. carry-in across lanes
    cf = scan_fwd(v[C - 1], sc, lc, lds_f);
    // 4. carry fix-up and pivot scaling
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const cd z = cmad(ld(sc.pt.at + k * T + t), cf, v[k]);
        v[k] = cmul(ld(sc.pt.q + k * T + t), z);
    }
    // 5. backward recurrence with zero carry-in
#pragma unroll
    for (int k = C - 2; k >= 0; --k) v[k] = cmad(ld(sc.pt.beta + k * T + t), v[k + 1], v[k]);
    // 6. carry-in from the right
    cb = scan_bwd(v[0], sc, lc, lds_b);
    // 7. carry fix-up
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = cmad(ld(sc.pt.bt + k * T + t), cb, v[k]);
}

// Field substep exp(-i dt E x_j) and absorber m_j applied to the chunk and to
// its two ghost points (x_{s-1} = xl).  The phase advances along the chunk by
// multiplication with exp(-i dt E dx); each lane starts from its own sincos.
template <int C>
__device__ __forceinline__ void phase_mask(cd (&v)[C], cd& gl, cd& gr, double e, double dt,
                                           double xl, double dx, const SizeClass& sc,
                                           const LaneCtx& lc)
{
    double s0, c0, s1, c1;
    sincos(-dt * e * xl, &s0, &c0);
    sincos(-dt * e * dx, &s1, &c1);
    cd ph = mkc(c0, s0);
    const cd w1 = mkc(c1, s1);
    gl = cscale(lc.ml, cmul(ph, gl));
    ph = cmul(ph, w1);
    if (lc.hasmask) {
        const int t = opaque(lc.t);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cscale(sc.pt.m[k * sc.T + t], cmul(ph, v[k]));
            ph = cmul(ph, w1);
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cmul(ph, v[k]);
            ph = cmul(ph, w1);
        }
    }
    gr = cscale(lc.mr, cmul(ph, gr));
}

// One full step psi^(i) -> psi^(i+1) (CN right-hand side, partitioned solve,
// ghost rebuild, field phase and absorber).
template <int C>
__device__ __forceinline__ void forward_step(cd (&v)[C], cd& gl, cd& gr, double e, double dt,
                                             double xl, const SizeClass& sc, const LaneCtx& lc,
                                             const RhsCoef rc, cd* lds_f, cd* lds_b)
{
    cd cf, cb;
    cn_apply<C, true>(v, gl, gr, sc, lc, rc, lds_f, lds_b, cf, cb);
    gl = cmad(lc.ql, cf, cmul(lc.bl, v[0]));
    gr = cb;
    phase_mask<C>(v, gl, gr, e, dt, xl, sc.dx, sc, lc);
}

}  // namespace tdse
