// tdse_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// complex fp64 arithmetic, wavefront shuffles and reductions, a reduced-range
// sincos, the cross-lane carry scans of the partitioned tridiagonal solve,
// and the Crank-Nicolson core that every kernel (forward, ground state,
// adjoint) runs once per time step.
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
__device__ __forceinline__ cd ld_psi(const double* p, int64_t j) { return mkc(p[2 * j], p[2 * j + 1]); }

// -(1 + h' w) q with h' = i (real time) or 1 (imaginary time): the
// elimination factors alpha, beta of the tridiagonal solve.
template <bool RT>
__device__ __forceinline__ cd elim(double w, cd q)
{
    if (RT) return mkc(fma(w, q.im, -q.re), fma(-w, q.re, -q.im));
    const double f = -(1.0 + w);
    return mkc(f * q.re, f * q.im);
}

// Load through the global address space.  Pointers that come out of
// structures are generic to the compiler, which would emit FLAT loads; those
// count against the LDS wait counter as well, so every LDS wait in the time
// loop would also wait for the L2.  (No volatile here: on gfx950 a volatile
// load is issued at system scope and bypasses the caches.)
__device__ __forceinline__ double ldg(const double* p)
{
    typedef const __attribute__((address_space(1))) double* gptr;
    return *(gptr)(p);
}
__device__ __forceinline__ int ldg(const int* p)
{
    typedef const __attribute__((address_space(1))) int* gptr;
    return *(gptr)(p);
}
__device__ __forceinline__ cd ldg(const cd* p)
{
    typedef double dvec2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) dvec2* gptr;
    const dvec2 v = *(gptr)(p);
    return mkc(v.x, v.y);
}

// Returns x unchanged but hides its value from the optimiser.  Table indices
// pass through it once per time step so that loop-invariant table loads stay
// inside the time loop instead of being hoisted into registers and spilled.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Hides a wave-uniform pointer from the optimiser (kept in SGPRs).
template <class T>
__device__ __forceinline__ T* launder_s(T* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Keeps the scheduler from hoisting the independent work of later grid
// points of an unrolled chunk loop above the current one: with four waves
// per SIMD latency is hidden across waves, and hoisting would only raise
// register pressure (and force spills).
#define TDSE_POINT_FENCE() __builtin_amdgcn_sched_barrier(0)
__device__ __forceinline__ void point_fence(cd a)
{
    asm volatile("" ::"v"(a.re), "v"(a.im));
    __builtin_amdgcn_sched_barrier(0);
}
__device__ __forceinline__ void point_fence(cd a, cd b)
{
    asm volatile("" ::"v"(a.re), "v"(a.im), "v"(b.re), "v"(b.im));
    __builtin_amdgcn_sched_barrier(0);
}
__device__ __forceinline__ void point_fence(double a, double b)
{
    asm volatile("" ::"v"(a), "v"(b));
    __builtin_amdgcn_sched_barrier(0);
}

// Loads a wave-uniform record into scalar registers.  Work items arrive
// through LDS, so the compiler cannot prove the record uniform on its own.
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
// Loads a record whose address is wave-uniform (held in SGPRs) through the
// constant address space, which the compiler turns into scalar loads.
template <class T>
__device__ __forceinline__ T scalar_load(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "scalar_load needs a 4-byte multiple");
    typedef const __attribute__((address_space(4))) int* cptr;
    const cptr src = (cptr)(p);
    T out;
    int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// A double constant materialised by two scalar moves where it is used.  FP64
// literals do not fit in a VALU instruction, so the compiler otherwise keeps
// every constant of the time loop in registers across the whole loop.
template <unsigned long long B>
__device__ __forceinline__ double kconst()
{
    int lo, hi;
    asm volatile("s_mov_b32 %0, %2\n\ts_mov_b32 %1, %3"
                 : "=s"(lo), "=s"(hi)
                 : "i"((int)(unsigned)(B & 0xffffffffull)), "i"((int)(unsigned)(B >> 32)));
    return __hiloint2double(hi, lo);
}
#define TDSE_K(x) ::tdse::kconst<__builtin_bit_cast(unsigned long long, (double)(x))>()

// ------------------------------------------------------------ sincos
// a * b + k with the constant k in scalar registers.  The compiler would
// otherwise prefer the two-address v_fmac form and copy k into a vector
// register pair before every step of a Horner chain.
__device__ __forceinline__ double fma_s(double a, double b, double k)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// sin and cos of x by Cody-Waite reduction to |r| <= pi/4 (x = k pi/2 + r,
// pi/2 split into a 32-bit head and two tails so k*head is exact for
// |k| < 2^20), then sin r = r + r^3 S(r^2) and cos r = 1 - r^2/2 + r^4 C(r^2)
// with S and C of degree 5: Chebyshev fits on r^2 in [0, (pi/4)^2] (the
// script csrc/sincos_coefficients.py derives them and checks the error:
// below 8e-17 for sin and 1.3e-16 for cos in double, i.e. rounding).
__device__ __forceinline__ void sincos_rr(double x, double* s, double* c)
{
    const double two_over_pi = TDSE_K(0.63661977236758134308);
    const double p1 = TDSE_K(1.5707963267341256);      // pi/2 rounded to 32 significant bits
    const double p2 = TDSE_K(6.077100506506192e-11);   // pi/2 - p1 rounded to double
    const double p3 = TDSE_K(3.5215598651832e-27);     // pi/2 - p1 - p2
    const double k = rint(x * two_over_pi);
    double r = fma(-k, p1, x);
    r = fma(-k, p2, r);
    r = fma(-k, p3, r);
    const double r2 = r * r;
    double ps = TDSE_K(1.5918129294866608e-10);
    ps = fma_s(ps, r2, TDSE_K(-2.5051131845003624e-08));
    ps = fma_s(ps, r2, TDSE_K(2.755731610255244e-06));
    ps = fma_s(ps, r2, TDSE_K(-0.00019841269836758574));
    ps = fma_s(ps, r2, TDSE_K(0.008333333333330948));
    ps = fma_s(ps, r2, TDSE_K(-0.16666666666666666));
    const double sr = fma(ps * r2, r, r);
    double pc = TDSE_K(-1.1382632425521717e-11);
    pc = fma_s(pc, r2, TDSE_K(2.08761462684032e-09));
    pc = fma_s(pc, r2, TDSE_K(-2.7557317271729793e-07));
    pc = fma_s(pc, r2, TDSE_K(2.480158729876569e-05));
    pc = fma_s(pc, r2, TDSE_K(-0.0013888888888887398));
    pc = fma_s(pc, r2, TDSE_K(0.041666666666666664));
    pc = fma(pc, r2, -0.5);
    const double cr = fma(pc, r2, 1.0);
    const int q = ((int)k) & 3;
    const double ss = (q & 1) ? cr : sr;
    const double cc = (q & 1) ? sr : cr;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}

// sin and cos of the per-point phase increment dt E dx, which is tiny
// (|x| < 0.05 always holds for sensible grids): Taylor series through x^9 and
// x^10 (truncation below 1e-19), through x^5 and x^6 for |x| <= 1e-3 (the
// usual case: dt E dx ~ 1e-4); larger arguments take the general path.
// The branches are uniform across the wavefront.
__device__ __forceinline__ void sincos_step(double x, double* s, double* c)
{
    if (fabs(x) > 0.05) {
        sincos_rr(x, s, c);
        return;
    }
    const double x2 = x * x;
    if (fabs(x) <= 1e-3) {
        // through x^5 and x^6 (truncation below 3e-22 relative)
        const double p5 = fma(x2, TDSE_K(8.3333333333333333333e-03), TDSE_K(-1.6666666666666666667e-01));  // 1/5!, -1/3!
        *s = fma(p5 * x2, x, x);
        double p6 = fma(x2, TDSE_K(-1.3888888888888888889e-03), TDSE_K(4.1666666666666666667e-02));        // -1/6!, 1/4!
        p6 = fma(p6, x2, -0.5);
        *c = fma(p6, x2, 1.0);
        return;
    }
    double ps = fma(x2, TDSE_K(2.7557319223985890653e-06), TDSE_K(-1.9841269841269841270e-04));   // 1/9!, -1/7!
    ps = fma_s(ps, x2, TDSE_K(8.3333333333333333333e-03));                                   // 1/5!
    ps = fma_s(ps, x2, TDSE_K(-1.6666666666666666667e-01));                                  // -1/3!
    *s = fma(ps * x2, x, x);
    double pc = fma(x2, TDSE_K(-2.7557319223985890653e-07), TDSE_K(2.4801587301587301587e-05));    // -1/10!, 1/8!
    pc = fma_s(pc, x2, TDSE_K(-1.3888888888888888889e-03));                                  // -1/6!
    pc = fma_s(pc, x2, TDSE_K(4.1666666666666666667e-02));                                   // 1/4!
    pc = fma(pc, x2, -0.5);                                                        // -1/2!
    *c = fma(pc, x2, 1.0);
}

// exp(-i dt e dx): the ratio of the field phase factors of neighbouring grid
// points in a step at field e.
__device__ __forceinline__ cd phase_ratio(double e, double dt, double dx)
{
    double s, c;
    sincos_step(-dt * e * dx, &s, &c);
    return mkc(c, s);
}

// ------------------------------------------------------------ wavefront ops
// DPP moves of the two halves of a double; lanes without a source (or in a
// masked row) read 0.  Controls: row_shr:n = 0x110+n, wave_shl:1 = 0x130,
// wave_shr:1 = 0x138, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double v)
{
    int lo, hi;
    if (ROWMASK == 0xf) {
        // every row written; bound_ctrl makes lanes without a source read 0
        lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
        hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    }
    return __hiloint2double(hi, lo);
}
// lane i receives lane i-1 (lane 0 receives 0)
__device__ __forceinline__ cd wave_shr1(cd a) { return mkc(dpp_d<0x138>(a.re), dpp_d<0x138>(a.im)); }
// lane i receives lane i+1 (lane 63 receives 0)
__device__ __forceinline__ cd wave_shl1(cd a) { return mkc(dpp_d<0x130>(a.re), dpp_d<0x130>(a.im)); }
// The same shifts, with the lane that has no source (lane 0, resp. 63)
// receiving `edge` instead of 0.
template <int CTRL>
__device__ __forceinline__ double dpp_keep(double v, double edge)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd wave_shr1_keep(cd a, cd edge)
{
    return mkc(dpp_keep<0x138>(a.re, edge.re), dpp_keep<0x138>(a.im, edge.im));
}
__device__ __forceinline__ cd wave_shl1_keep(cd a, cd edge)
{
    return mkc(dpp_keep<0x130>(a.re, edge.re), dpp_keep<0x130>(a.im, edge.im));
}

__device__ __forceinline__ cd shfl_up_c(cd a, int d)
{
    return mkc(__shfl_up(a.re, d), __shfl_up(a.im, d));
}
__device__ __forceinline__ cd shfl_down_c(cd a, int d)
{
    return mkc(__shfl_down(a.re, d), __shfl_down(a.im, d));
}
// Sum over the 64 lanes by DPP: inclusive scans within rows of 16
// (row_shr 1, 2, 4, 8), then the row totals are folded in with row
// broadcasts.  The total is valid in lane 63 only; the association order is
// fixed, so results are bitwise reproducible.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_d<0x111>(x);
    x += dpp_d<0x112>(x);
    x += dpp_d<0x114>(x);
    x += dpp_d<0x118>(x);
    x += dpp_d<0x142, 0xa>(x);
    x += dpp_d<0x143, 0xc>(x);
    return x;
}
constexpr int kSumLane = kWave - 1;  // lane holding wave_sum's result

// ------------------------------------------------------------ table views
// om and dV/dx of a size class seen through LDS (staged once per workgroup,
// shared by its systems) or directly in global memory.  The pivot factors q
// live in registers instead (LaneFactors).
template <bool OM_GLOBAL, bool DV_GLOBAL>
struct TabViewT {
    const double* om_;
    const double* dv_;
    __device__ __forceinline__ double om(int i) const { return OM_GLOBAL ? ldg(om_ + i) : om_[i]; }
    __device__ __forceinline__ double dv(int i) const { return DV_GLOBAL ? ldg(dv_ + i) : dv_[i]; }
};
using TabLds = TabViewT<false, false>;
using TabGlobal = TabViewT<true, true>;
using TabOmLds = TabViewT<false, true>;

// ------------------------------------------------------------ lane context
// Lane coordinates within the system's subgroup and the table indices of the
// two points next to the lane's chunk (clamped to the lane's own points at
// the ends of the grid, where the ghost values they multiply are zero).
struct LaneCtx {
    int lane;   // lane in wavefront
    int wave;   // wavefront within the system's subgroup
    int W;      // wavefronts per system
    int t;      // lane index within the system (0..T-1)
    int s;      // first grid point of the lane's chunk
    int b0;     // table index of the chunk's first point
    int C, T;   // points per lane, lanes per system
    // Table indices of point s-1 (the last point of lane t-1: 64(C-1) - 1
    // past b0 within a wavefront, b0 - 1 across a wavefront boundary) and of
    // point s+C (the first point of lane t+1), clamped at the two ends of the
    // grid.  Formed where they are used (from a fresh copy of t) rather than
    // kept live across the step.
    __device__ __forceinline__ int il() const
    {
        const int tt = opaque(t), ln = tt & (kWave - 1);
        return max(pbase(tt, C) - 1 + (ln ? 64 * (C - 1) : 0), 0);
    }
    __device__ __forceinline__ int ir() const
    {
        const int tt = opaque(t), ln = tt & (kWave - 1);
        return min(pbase(tt, C) + (ln == kWave - 1 ? 64 * C - 63 : 1), C * T - 1);
    }
};

// wave: the wavefront index t / 64, passed separately so that the compiler
// can keep it in a scalar register (it is uniform across the wavefront).
__device__ __forceinline__ LaneCtx make_lane_ctx(const SizeClass& sc, int t, int wave)
{
    LaneCtx c;
    const int C = sc.C;
    c.lane = t & (kWave - 1);
    c.wave = wave;
    c.W = sc.T / kWave;
    c.t = t;
    c.s = t * C;
    c.b0 = pbase(t, C);
    c.C = C;
    c.T = sc.T;
    return c;
}

// Pivot factors q are held in registers for a whole propagation when the
// chunk is short enough (C <= 8: 4C + 4 VGPRs); with 16 points per lane they
// would not fit beside the chunk itself and are read from global memory
// (L2-resident) where they are used.
template <int C>
struct QInRegs {
    static constexpr bool value = C <= 8;
};

// Per-lane factors: q at the C points of the chunk and at the point before
// it (when held in registers), and the absorber flags (bit 0: a mask value of
// the chunk differs from 1; bit 1: at s-1; bit 2: at s+C).  Where q is not
// in registers, AB selects where the elimination factors come from: the
// alpha and beta tables (no arithmetic, but three tables to keep in the L2
// instead of one) or q and om (two FMAs each).
template <int C, bool QREG = QInRegs<C>::value, bool AB = true>
struct LaneFactors {
    static constexpr bool kRegs = QREG;  // q held in registers
    static constexpr bool kTabAB = !QREG && AB;  // alpha, beta read from their tables
    static constexpr bool kOm = !kTabAB;         // om needed to form them
    static constexpr int NQ = QREG ? C : 1;
    cd q_[NQ];
    cd ql_;
    int mflags;
    // q at point k of the chunk and at s-1 (zero for the first lane)
    __device__ __forceinline__ cd q(int k, const SizeClass& sc, const LaneCtx& lc) const
    {
        if constexpr (QREG) return q_[k];
        else return ldg(sc.pt.q + lc.b0 + 64 * k);
    }
    __device__ __forceinline__ cd ql(const SizeClass& sc, const LaneCtx& lc) const
    {
        if constexpr (QREG) return ql_;
        else return lc.t > 0 ? ldg(sc.pt.q + lc.il()) : czero();
    }
    // Elimination factors at point k of the chunk: alpha_k from
    // om_{k-1} = om_p and q_{k-1} (the previous lane's last q for k = 0),
    // beta_k from om_{k+1} = om_n and q_k.
    template <bool RT>
    __device__ __forceinline__ cd alpha(int k, double om_p, const SizeClass& sc,
                                        const LaneCtx& lc) const
    {
        if constexpr (kTabAB) return ldg(sc.pt.alpha + lc.b0 + 64 * k);
        else return elim<RT>(om_p, k == 0 ? ql(sc, lc) : q(k - 1, sc, lc));
    }
    template <bool RT>
    __device__ __forceinline__ cd beta(int k, double om_n, const SizeClass& sc,
                                       const LaneCtx& lc) const
    {
        if constexpr (kTabAB) return ldg(sc.pt.beta + lc.b0 + 64 * k);
        else return elim<RT>(om_n, q(k, sc, lc));
    }
};

template <int C, bool QREG = QInRegs<C>::value, bool AB = true>
__device__ __forceinline__ LaneFactors<C, QREG, AB> load_factors(const SizeClass& sc,
                                                                 const LaneCtx& lc)
{
    LaneFactors<C, QREG, AB> f;
    if constexpr (QREG) {
#pragma unroll
        for (int k = 0; k < C; ++k) f.q_[k] = ldg(sc.pt.q + lc.b0 + 64 * k);
        f.ql_ = lc.t > 0 ? ldg(sc.pt.q + lc.il()) : czero();
    } else {
        f.q_[0] = czero();
        f.ql_ = czero();
    }
    f.mflags = ldg(sc.lt.hasmask + lc.t);
    return f;
}

// Unsigned byte offset of lane t in a per-lane array of 16-byte records;
// loads through it use a scalar base register plus one vector offset.
__device__ __forceinline__ cd ld_lane(const cd* base, unsigned off_bytes)
{
    return ldg(reinterpret_cast<const cd*>(reinterpret_cast<const char*>(base) + off_bytes));
}

// State record of the adjoint's checkpoints: chunk values and the two
// ghosts, [C+2][T] complex.  The record base is wave-uniform (scalar
// registers); each access adds the lane's byte offset 16 t, so the loads
// and stores take one VGPR offset.
__device__ __forceinline__ void st_lane(double* base, unsigned off_bytes, cd x)
{
    typedef double dvec2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) dvec2* gptr;
    dvec2 w;
    w.x = x.re;
    w.y = x.im;
    *(gptr)(reinterpret_cast<char*>(base) + off_bytes) = w;
}

template <int C>
__device__ __forceinline__ void store_state(double* base, int T, unsigned off, const cd (&v)[C],
                                            cd gl, cd gr)
{
#pragma unroll
    for (int k = 0; k < C; ++k) st_lane(base + 2 * (size_t)k * T, off, v[k]);
    st_lane(base + 2 * (size_t)C * T, off, gl);
    st_lane(base + 2 * (size_t)(C + 1) * T, off, gr);
}

// ------------------------------------------------------------ carry scans
// Forward carries of z_j = r_j + alpha_j z_{j-1}.  Input: the lane's chunk-end
// value computed with a zero carry-in.  Output: the true z at the point just
// before the lane's chunk (the lane's carry-in).  In-wave Kogge-Stone over
// `levels` levels with precomputed window products, then one cross-wave
// correction through LDS; windows longer than 2^levels lanes are dropped
// only when the host has verified that their products are below 2^-56.
// a0, a1, aw: the lane's window products of levels 0 and 1 and of the
// cross-wave correction, loaded by the caller ahead of time.
__device__ __forceinline__ cd scan_fwd(cd z, cd a0, cd a1, cd aw, const SizeClass& sc,
                                       const LaneCtx& lc, cd* lds)
{
    const unsigned off = 16u * (unsigned)lc.t;
    // levels 0 and 1 shift by whole-wave DPP moves (lanes below the shift
    // receive 0, which leaves them unchanged); deeper levels use bpermute
    if (sc.levels > 0) z = cmad(a0, wave_shr1(z), z);
    if (sc.levels > 1) z = cmad(a1, wave_shr1(wave_shr1(z)), z);
    for (int lev = 2; lev < sc.levels; ++lev) {
        const int d = 1 << lev;
        cd zs = shfl_up_c(z, d);
        const cd p = ld_lane(sc.lt.pa + lev * sc.T, off);
        if (lc.lane >= d) z = cmad(p, zs, z);
    }
    cd prev = czero();
    // The barrier is taken even by single-wavefront systems: subgroups of
    // different sizes share a workgroup and must take the same barriers.
    if (lc.W > 1 && lc.lane == kWave - 1) lds[lc.wave] = z;
    __syncthreads();
    if (lc.W > 1) {
        const int v0 = max(0, lc.wave - sc.xwaves);  // wave-uniform
        if (v0 < lc.wave) {
            prev = lds[v0];
            for (int w = v0 + 1; w < lc.wave; ++w)
                prev = cmad(ldg(sc.lt.pw + w * kWave + kWave - 1), prev, lds[w]);
        }
        z = cmad(aw, prev, z);  // aw = 0 in lanes past the scan's reach
    }
    return wave_shr1_keep(z, prev);
}

// Backward carries of y_j = w_j + beta_j y_{j+1}, mirrored: returns the true y
// at the point just after the lane's chunk.
__device__ __forceinline__ cd scan_bwd(cd y, cd b0, cd b1, cd bw, const SizeClass& sc,
                                       const LaneCtx& lc, cd* lds)
{
    const unsigned off = 16u * (unsigned)lc.t;
    if (sc.levels > 0) y = cmad(b0, wave_shl1(y), y);
    if (sc.levels > 1) y = cmad(b1, wave_shl1(wave_shl1(y)), y);
    for (int lev = 2; lev < sc.levels; ++lev) {
        const int d = 1 << lev;
        cd ys = shfl_down_c(y, d);
        const cd p = ld_lane(sc.lt.qb + lev * sc.T, off);
        if (lc.lane + d < kWave) y = cmad(p, ys, y);
    }
    cd next = czero();
    if (lc.W > 1 && lc.lane == 0) lds[lc.wave] = y;
    __syncthreads();
    if (lc.W > 1) {
        const int v1 = min(lc.W - 1, lc.wave + sc.xwaves);  // wave-uniform
        if (v1 > lc.wave) {
            next = lds[v1];
            for (int w = v1 - 1; w > lc.wave; --w) next = cmad(ldg(sc.lt.qw + w * kWave), next, lds[w]);
        }
        y = cmad(bw, next, y);  // bw = 0 in lanes past the scan's reach
    }
    return wave_shl1_keep(y, next);
}

// ------------------------------------------------------------ CN core
// Right-hand side 12 R psi with R = M2 - h A, A = -D2/2 + M2 diag(V), h = h' |h|
// (h' = i in real time, 1 in imaginary time).  With S the stencil
// S(x)_j = x_{j-1} + 10 x_j + x_{j+1}, om as in PointTables and
// dofs = 72 |h| / dx^2 (the diagonal of 12 |h| (-D2/2)):
//   12 R psi = S(psi) - h' (S(om psi) + dofs psi)
//            = (g_{j-1} + g_{j+1}) + 10 gh_j,
//   g_j  = (1 - h' om_j) psi_j,   gh_j = (1 - h' (om_j + dofs/10)) psi_j.
// In real time gh_j = g_j - i (dofs/10) psi_j is formed from g_j (two FMAs):
// om_j and dofs/10 are both about 6 |h| / dx^2 and their sum is several times
// smaller, so this loses about 2.5 bits of the step's rounding, far below the
// method's error.  In imaginary time 1 - (om_j + dofs/10) can vanish and gh
// is formed from psi directly.
struct RhsCoef {
    double dofs10;  // dofs / 10 (precomputed per size class)
};

// (1 - h' w) x
template <bool RT>
__device__ __forceinline__ cd gfac(double w, cd x)
{
    if (RT) return mkc(fma(w, x.im, x.re), fma(-w, x.re, x.im));
    return mkc(fma(-w, x.re, x.re), fma(-w, x.im, x.im));
}

// Applies psi <- L^{-1} R psi (before the field phase and absorber) to the
// lane's chunk v[0..C-1] whose neighbours are gl = psi_{s-1}, gr = psi_{s+C},
// and replaces gl, gr by the new neighbour values.  Four sweeps over the
// chunk: right-hand side fused with the forward recurrence from a zero carry
// (chunk-end value only); forward recurrence from the exact carry with the
// pivot scaling; backward recurrence from a zero carry (chunk-start value
// only); backward recurrence from the exact carry.  The new neighbours follow
// from the exact carries cf = z_{s-1} and cb = y_{s+C} without exchanging
// data between lanes:  y_{s+C} = cb,  y_{s-1} = q_{s-1} cf + beta_{s-1} y_s.
template <int C, bool RT, class TV, class LF>
__device__ __forceinline__ void cn_apply(cd (&v)[C], cd& gl, cd& gr, const LF& f,
                                         const TV& tb, const SizeClass& sc, const LaneCtx& lc,
                                         const RhsCoef rc, cd* lds_f, cd* lds_b)
{
    const int b0 = lc.b0;
    const unsigned off = 16u * (unsigned)lc.t;
    const double oml = tb.om(lc.il());
    const double omr = tb.om(lc.ir());
    // points ahead of its use at which a factor read from memory (L2) is
    // issued: one in sweeps A and B, whose per-point work covers it and where
    // a second point's factors would be spilled; three in sweeps C and D,
    // which do one complex FMA per point (N = 9216-16384: +2-3 %)
    constexpr int kAhead = 1;
    constexpr int kAheadBwd = 3;
    // window products of the forward scan, loaded three quarters of the way
    // through sweep A (at its last point where q is read from memory)
    cd a0 = czero(), a1 = czero(), aw = czero();
    // A. right-hand side in place, chunk-end value of z with zero carry-in
    cd ze = czero();
    {
        double om_p = oml;
        double om_c = tb.om(b0);
        double om_n = C > 1 ? tb.om(b0 + 64) : omr;
        cd g_p = gfac<RT>(oml, gl);
        cd g_c = gfac<RT>(om_c, v[0]);
        // elimination factors read from their table (L2): issued kAhead
        // points ahead of their use
        cd al[C];
        if constexpr (LF::kTabAB) {
#pragma unroll
            for (int j = 1; j < kAhead && j < C; ++j) al[j] = f.template alpha<RT>(j, 0.0, sc, lc);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if (k == (LF::kRegs ? 3 * C / 4 : C - 1)) {
                if (sc.levels > 0) a0 = ld_lane(sc.lt.pa, off);
                if (sc.levels > 1) a1 = ld_lane(sc.lt.pa + sc.T, off);
                if (lc.lane < (1 << sc.levels)) aw = ld_lane(sc.lt.pw, off);
            }
            // om of the point after next, issued one point ahead of its use
            const double om_nn = (k + 2 < C) ? tb.om(b0 + 64 * (k + 2)) : omr;
            if constexpr (LF::kTabAB) {
                if (k + kAhead < C) al[k + kAhead] = f.template alpha<RT>(k + kAhead, 0.0, sc, lc);
            }
            TDSE_POINT_FENCE();
            const cd g_n = gfac<RT>(om_n, (k + 1 < C) ? v[k + 1] : gr);
            // real time: gh = g - i (dofs/10) psi from g (two FMAs); the
            // cancellation of om and dofs/10 costs about 2.5 bits per step
            // there. Imaginary time forms it from psi, since 1 - (om +
            // dofs/10) can vanish.
            const cd gh = RT ? mkc(fma(rc.dofs10, v[k].im, g_c.re), fma(-rc.dofs10, v[k].re, g_c.im))
                             : gfac<RT>(om_c + rc.dofs10, v[k]);
            const cd r = mkc(fma(10.0, gh.re, g_p.re + g_n.re), fma(10.0, gh.im, g_p.im + g_n.im));
            v[k] = r;
            if constexpr (LF::kTabAB) ze = (k == 0) ? r : cmad(al[k], ze, r);
            else ze = (k == 0) ? r : cmad(f.template alpha<RT>(k, om_p, sc, lc), ze, r);
            g_p = g_c;
            g_c = g_n;
            om_p = om_c;
            om_c = om_n;
            om_n = om_nn;
            point_fence(r, ze);
        }
    }
    const cd cf = scan_fwd(ze, a0, a1, aw, sc, lc, lds_f);
    // window products of the backward scan: loaded ahead of sweep B when the
    // registers allow, else just before the scan
    cd b0c = czero(), b1c = czero(), bw = czero();
    auto load_bwd_windows = [&]() {
        if (sc.levels > 0) b0c = ld_lane(sc.lt.qb, off);
        if (sc.levels > 1) b1c = ld_lane(sc.lt.qb + sc.T, off);
        if (lc.lane > kWave - 1 - (1 << sc.levels)) bw = ld_lane(sc.lt.qw, off);
    };
    if constexpr (LF::kRegs) load_bwd_windows();
    double om_last;  // om_{C-1}, read by sweep B for sweep C
    // B. forward recurrence from the exact carry, w = q z.  When q is read
    // from memory, each sweep hides the chunk base from the optimiser so
    // that it reloads its factors rather than keeping earlier sweeps' values
    // live (they would be spilled).
    {
        LaneCtx lcb = lc;
        if constexpr (!LF::kRegs) lcb.b0 = opaque(lc.b0);
        cd z = cf;
        double om_p = oml;
        // factors read from memory (alpha from its table, q): issued kAhead
        // points ahead of their use
        cd al[C], qm[C];
#pragma unroll
        for (int j = 0; j < kAhead && j < C; ++j) {
            if constexpr (LF::kTabAB) al[j] = f.template alpha<RT>(j, 0.0, sc, lcb);
            if constexpr (!LF::kRegs) qm[j] = f.q(j, sc, lcb);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
            // om_k for the next point (at the last point, om_{C-1} for sweep
            // C), issued ahead of this point's work so that its LDS latency
            // overlaps it
            const double om_k = tb.om(lcb.b0 + 64 * k);
            if (k + kAhead < C) {
                if constexpr (LF::kTabAB) al[k + kAhead] = f.template alpha<RT>(k + kAhead, 0.0, sc, lcb);
                if constexpr (!LF::kRegs) qm[k + kAhead] = f.q(k + kAhead, sc, lcb);
            }
            TDSE_POINT_FENCE();
            if constexpr (LF::kTabAB) z = cmad(al[k], z, v[k]);
            else z = cmad(f.template alpha<RT>(k, om_p, sc, lcb), z, v[k]);
            if constexpr (LF::kRegs) v[k] = cmul(f.q(k, sc, lcb), z);
            else v[k] = cmul(qm[k], z);
            om_p = om_k;
            point_fence(v[k]);
        }
        om_last = om_p;
    }
    // C. chunk-start value of y with zero carry-in
    cd yb = v[C - 1];
    {
        LaneCtx lcc = lc;
        if constexpr (!LF::kRegs) lcc.b0 = opaque(lc.b0);
        const int bc = lcc.b0;
        double om_n = LF::kOm ? om_last : 0.0;
        // the table's beta issued kAheadBwd points ahead of its use
        cd be[C];
        if constexpr (LF::kTabAB) {
#pragma unroll
            for (int j = C - 2; j > C - 2 - kAheadBwd && j >= 0; --j)
                be[j] = f.template beta<RT>(j, 0.0, sc, lcc);
        }
#pragma unroll
        for (int k = C - 2; k >= 0; --k) {
            // om_k for the next point, issued one point ahead
            const double om_k = (LF::kOm && k > 0) ? tb.om(bc + 64 * k) : 0.0;
            if constexpr (LF::kTabAB) {
                if (k - kAheadBwd >= 0) be[k - kAheadBwd] = f.template beta<RT>(k - kAheadBwd, 0.0, sc, lcc);
            }
            TDSE_POINT_FENCE();
            if constexpr (LF::kTabAB) yb = cmad(be[k], yb, v[k]);
            else yb = cmad(f.template beta<RT>(k, om_n, sc, lcc), yb, v[k]);
            om_n = om_k;
            point_fence(yb);
        }
    }
    if constexpr (!LF::kRegs) load_bwd_windows();
    const cd cb = scan_bwd(yb, b0c, b1c, bw, sc, lc, lds_b);
    // D. backward recurrence from the exact carry
    double om_0;
    {
        LaneCtx lcd = lc;
        if constexpr (!LF::kRegs) lcd.b0 = opaque(lc.b0);
        cd y = cb;
        double om_n = omr;
        cd be[C];
        if constexpr (LF::kTabAB) {
#pragma unroll
            for (int j = C - 1; j > C - 1 - kAheadBwd && j >= 0; --j)
                be[j] = f.template beta<RT>(j, 0.0, sc, lcd);
        }
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            // om_k for the next point (om_0 for the ghost), issued ahead; the
            // table's beta kAheadBwd points ahead
            const double om_k = tb.om(lcd.b0 + 64 * k);
            if constexpr (LF::kTabAB) {
                if (k - kAheadBwd >= 0) be[k - kAheadBwd] = f.template beta<RT>(k - kAheadBwd, 0.0, sc, lcd);
            }
            TDSE_POINT_FENCE();
            if constexpr (LF::kTabAB) y = cmad(be[k], y, v[k]);
            else y = cmad(f.template beta<RT>(k, om_n, sc, lcd), y, v[k]);
            v[k] = y;
            om_n = om_k;
            point_fence(y);
        }
        om_0 = om_n;
    }
    const cd ql = f.ql(sc, lc);
    gl = cmad(ql, cf, cmul(elim<RT>(om_0, ql), v[0]));
    gr = cb;
}

// Field substep exp(-i dt E x_j) and absorber m_j on the chunk and its two
// ghost points (x_{s-1} = xl).  The phase advances along the chunk by
// multiplication with w1 = exp(-i dt E dx) (phase_ratio); each lane starts
// from its own sincos.
// BRANCHLESS: the absorber factor is applied to every point (1 away from
// the edges); used where a branch would make the two paths' results meet in
// different registers and cost spills of the chunk.
template <int C, bool BRANCHLESS>
__device__ __forceinline__ void phase_mask(cd (&v)[C], cd& gl, cd& gr, double e, double dt,
                                           double xl, const cd w1, int mflags,
                                           const SizeClass& sc, const LaneCtx& lc)
{
    double s0, c0;
    sincos_rr(-dt * e * xl, &s0, &c0);
    cd ph = mkc(c0, s0);
    gl = cmul(ph, gl);
    if (mflags & 2) gl = cscale(ldg(sc.pt.m + lc.il()), gl);
    ph = cmul(ph, w1);
    if constexpr (BRANCHLESS && C <= 12) {
        // the next point's absorber value (L2) issued one point ahead (at 16
        // points per lane the extra live value costs more spills than the
        // latency it hides: 14 % slower at N = 16384)
        double m_c = ldg(sc.pt.m + lc.b0);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const double m_n = k + 1 < C ? ldg(sc.pt.m + lc.b0 + 64 * (k + 1)) : 0.0;
            TDSE_POINT_FENCE();
            v[k] = cscale(m_c, cmul(ph, v[k]));
            ph = cmul(ph, w1);
            m_c = m_n;
            point_fence(v[k], ph);
        }
    } else if constexpr (BRANCHLESS) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cscale(ldg(sc.pt.m + lc.b0 + 64 * k), cmul(ph, v[k]));
            ph = cmul(ph, w1);
            point_fence(v[k], ph);
        }
    } else if (mflags & 1) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cscale(ldg(sc.pt.m + lc.b0 + 64 * k), cmul(ph, v[k]));
            ph = cmul(ph, w1);
            point_fence(v[k], ph);
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cmul(ph, v[k]);
            ph = cmul(ph, w1);
            point_fence(v[k], ph);
        }
    }
    gr = cmul(ph, gr);
    if (mflags & 4) gr = cscale(ldg(sc.pt.m + lc.ir()), gr);
}

// Where forward_step takes the step's phase ratio from, after the solve (so
// after its barriers): computed in place, or read from the subgroup's LDS
// block that fill_ratios wrote ahead.
struct RatioNow {
    double e, dt, dx;
    __device__ __forceinline__ cd operator()() const { return phase_ratio(e, dt, dx); }
};
struct RatioLds {
    const cd* p;
    __device__ __forceinline__ cd operator()() const { return *p; }
};

// One full step psi^(i) -> psi^(i+1) (CN right-hand side, partitioned solve,
// ghost rebuild, field phase and absorber).
template <int C, class TV, class LF, class RF>
__device__ __forceinline__ void forward_step(cd (&v)[C], cd& gl, cd& gr, const LF& f,
                                             double e, const RF ratio, double dt, double xl,
                                             const TV& tb, const SizeClass& sc,
                                             const LaneCtx& lc, const RhsCoef rc, cd* lds_f,
                                             cd* lds_b)
{
    cn_apply<C, true, TV>(v, gl, gr, f, tb, sc, lc, rc, lds_f, lds_b);
    phase_mask<C, !LF::kRegs>(v, gl, gr, e, dt, xl, ratio(), f.mflags, sc, lc);
}

// Copies the om and dV/dx tables of a size class into LDS: 16 bytes per
// point, shared by every system the workgroup propagates.
__device__ __forceinline__ TabLds stage_tables(const SizeClass& sc, double* lds)
{
    const int np = sc.C * sc.T;
    double* om = lds;
    double* dv = lds + np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        om[i] = sc.pt.om[i];
        dv[i] = sc.pt.dv[i];
    }
    __syncthreads();
    TabLds tv;
    tv.om_ = om;
    tv.dv_ = dv;
    return tv;
}

__device__ __forceinline__ TabGlobal global_tables(const SizeClass& sc)
{
    TabGlobal tv;
    tv.om_ = sc.pt.om;
    tv.dv_ = sc.pt.dv;
    return tv;
}

template <int TAB>
struct TableSource;
template <>
struct TableSource<kTabLds> {
    using type = TabLds;
    static __device__ __forceinline__ TabLds make(const SizeClass& sc, double* lds) { return stage_tables(sc, lds); }
    static __device__ __forceinline__ TabLds view(const SizeClass& sc, double* lds)
    {
        TabLds tv;
        tv.om_ = lds;
        tv.dv_ = lds + sc.C * sc.T;
        return tv;
    }
};
template <>
struct TableSource<kTabOmLds> {
    using type = TabOmLds;
    static __device__ __forceinline__ TabOmLds view(const SizeClass& sc, double* lds)
    {
        TabOmLds tv;
        tv.om_ = lds;
        tv.dv_ = sc.pt.dv;
        return tv;
    }
};
template <>
struct TableSource<kTabGlobal> {
    using type = TabGlobal;
    static __device__ __forceinline__ TabGlobal make(const SizeClass& sc, double*) { return global_tables(sc); }
    static __device__ __forceinline__ TabGlobal view(const SizeClass& sc, double*) { return global_tables(sc); }
};

// Everything one time step needs to know about its size class.  The time
// loops rebuild it at the top of every step from a class address that the
// optimiser cannot see through: otherwise the addresses, lane predicates and
// coordinates derived from the class are hoisted out of the loop and kept
// live across it, far beyond the register budget of four waves per SIMD.
// Rebuilding costs a few scalar loads and integer operations per step.
template <int TAB>
struct StepView {
    SizeClass sc;
    LaneCtx lc;
    typename TableSource<TAB>::type tb;
    RhsCoef rc;
    double xs;  // x of the lane's first point
    double xl;  // x of the point before it
};

// wsys: wave-uniform index of the calling wavefront within its system; the
// lane index is rebuilt from the hardware lane id, so no per-lane index stays
// live across the time loop.
template <int TAB>
__device__ __forceinline__ StepView<TAB> step_view(const SizeClass* cls, int wsys, double* smem)
{
    StepView<TAB> v;
    v.sc = scalar_load(launder_s(cls));
    v.lc = make_lane_ctx(v.sc, wsys * kWave + opaque((int)__lane_id()), wsys);
    v.tb = TableSource<TAB>::view(v.sc, smem);
    v.rc.dofs10 = v.sc.dofs10;
    const double c = 0.5 * (double)(v.sc.n - 1);
    v.xs = ((double)v.lc.s - c) * v.sc.dx;
    v.xl = ((double)(v.lc.s - 1) - c) * v.sc.dx;
    return v;
}

// ------------------------------------------------------------ time-loop helpers
// Per-subgroup LDS block: forward and backward carry slots, two reduction
// slot arrays, the phase ratios of the next kFlush steps, the observables
// ring, a few flags.
struct SubSmem {
    cd* lds_f;
    cd* lds_b;
    double* red0;
    double* red1;
    cd* ratio;
    double* ring;
    int* misc;
};

__device__ __forceinline__ SubSmem carve_sub(char* base, int W)
{
    SubSmem s;
    s.lds_f = reinterpret_cast<cd*>(base);
    s.lds_b = s.lds_f + kMaxWaves;
    s.red0 = reinterpret_cast<double*>(s.lds_b + kMaxWaves);
    s.red1 = s.red0 + kMaxWaves;
    s.ratio = reinterpret_cast<cd*>(s.red1 + kMaxWaves);
    s.ring = reinterpret_cast<double*>(s.ratio + kFlush);
    s.misc = reinterpret_cast<int*>(s.ring + kRing * W * 3);
    return s;
}

// Per-lane partial sums of the observables of the current state, reduced over
// the wavefront; the lane holding the totals stores (sum V'|psi|^2,
// sum x|psi|^2, sum |psi|^2).
template <int C, class TV>
__device__ __forceinline__ void observe(const cd (&v)[C], const TV& tb, int T,
                                        const LaneCtx& lc, double xs, double dx, double* slot)
{
    double sn = 0.0, sk = 0.0, sv = 0.0;
    double dv = tb.dv(lc.b0);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        // dV/dx of the next point, issued one point ahead of its use
        const double dv_n = k + 1 < C ? tb.dv(lc.b0 + 64 * (k + 1)) : 0.0;
        TDSE_POINT_FENCE();
        const double p = cabs2(v[k]);
        sn = k == 0 ? p : sn + p;
        if (k > 0) sk = fma((double)k, p, sk);
        sv = k == 0 ? dv * p : fma(dv, p, sv);
        dv = dv_n;
        point_fence(sv, sn);
    }
    double sx = fma(xs, sn, dx * sk);
    // three independent DPP reductions: a one-pass reduce-scatter of the
    // three sums over permlane swaps issues fewer instructions but measured
    // 3-10 % slower (one serial chain instead of three interleaved ones)
    sn = wave_sum(sn);
    sx = wave_sum(sx);
    sv = wave_sum(sv);
    if (lc.lane == kSumLane) {
        slot[lc.wave * 3 + 0] = sv;
        slot[lc.wave * 3 + 1] = sx;
        slot[lc.wave * 3 + 2] = sn;
    }
}

// The same sums plus the two population observables of the current state
// (ring values 3..5 of the wavefront): the overlap sum_j conj(phi_j) psi_j
// with the reference state phi (natural point order, interleaved complex,
// n points; padding points read phi_{n-1} against psi = 0) and
// sum_{|x_j| <= radius} |psi_j|^2 with x_j = (j - (n-1)/2) dx.
template <int C, class TV>
__device__ __forceinline__ void observe_pop(const cd (&v)[C], const TV& tb, int T,
                                            const LaneCtx& lc, double xs, double dx, int n,
                                            const double* phi, double radius, double* slot)
{
    double sn = 0.0, sk = 0.0, sv = 0.0, orr = 0.0, oi = 0.0, sr = 0.0;
    const cd* ph = reinterpret_cast<const cd*>(phi);
    const double c = 0.5 * (double)(n - 1);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double p = cabs2(v[k]);
        sn += p;
        sk = fma((double)k, p, sk);
        sv = fma(tb.dv(lc.b0 + 64 * k), p, sv);
        const int j = lc.s + k;
        const cd f = ldg(ph + min(j, n - 1));
        orr = fma(f.re, v[k].re, fma(f.im, v[k].im, orr));
        oi = fma(f.re, v[k].im, fma(-f.im, v[k].re, oi));
        const double xj = ((double)j - c) * dx;
        sr += (fabs(xj) <= radius) ? p : 0.0;
    }
    double sx = fma(xs, sn, dx * sk);
    sn = wave_sum(sn);
    sx = wave_sum(sx);
    sv = wave_sum(sv);
    orr = wave_sum(orr);
    oi = wave_sum(oi);
    sr = wave_sum(sr);
    if (lc.lane == kSumLane) {
        double* o = slot + lc.wave * 6;
        o[0] = sv;
        o[1] = sx;
        o[2] = sn;
        o[3] = orr;
        o[4] = oi;
        o[5] = sr;
    }
}

// Sums the per-wave partials of samples [a0, a1] in wave order and writes
//   accel = dx (sum V'|psi|^2 + E sum |psi|^2), xexp = dx sum x|psi|^2,
//   norm = dx sum |psi|^2.
// With POP the ring holds six values per wavefront and sample in a ring of
// kRing / 2 samples (the same LDS bytes), and the populations are written:
//   gs_row  = |dx sum conj(phi) psi|^2,   vol_row = dx sum_{|x| <= r} |psi|^2.
// n2_row, when set, receives the norm as well (the checkpoint store's row).
template <bool POP = false>
__device__ __forceinline__ void flush(int a0, int a1, int t, int T, const double* ring, int W,
                                      double dx, const double* erow, double* acc_row,
                                      double* x_row, double* n_row, double n0, int* flag,
                                      double* gs_row = nullptr, double* vol_row = nullptr,
                                      double* n2_row = nullptr)
{
    constexpr int NV = POP ? 6 : 3;
    constexpr int RING = POP ? kRing / 2 : kRing;
    for (int smp = a0 + t; smp <= a1; smp += T) {
        const double* r = ring + (smp % RING) * W * NV;
        double sv = 0.0, sx = 0.0, sn = 0.0;
        for (int w = 0; w < W; ++w) {
            sv += r[w * NV + 0];
            sx += r[w * NV + 1];
            sn += r[w * NV + 2];
        }
        if constexpr (POP) {
            double orr = 0.0, oi = 0.0, sr = 0.0;
            for (int w = 0; w < W; ++w) {
                orr += r[w * NV + 3];
                oi += r[w * NV + 4];
                sr += r[w * NV + 5];
            }
            orr *= dx;
            oi *= dx;
            if (gs_row) gs_row[smp] = fma(orr, orr, oi * oi);
            if (vol_row) vol_row[smp] = dx * sr;
        }
        const double nn = dx * sn;
        const double acc = dx * fma(erow[smp], sn, sv);
        acc_row[smp] = acc;
        if (x_row) x_row[smp] = dx * sx;
        if (n_row) n_row[smp] = nn;
        if (n2_row) n2_row[smp] = nn;
        int f = 0;
        if (!isfinite(acc) || !isfinite(nn) || !isfinite(sx)) f |= 1;
        if (nn > n0 * (1.0 + 1e-8)) f |= 2;
        if (f) atomicOr(flag, f);
    }
}

}  // namespace tdse
