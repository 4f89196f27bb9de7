// tdse_adjoint.hip -- discrete adjoint of the batched forward propagation.
//
// Forward map (section "1D-TSDE Implementation (CTDSE)" substeps, then the
// absorber): psi^{i+1} = D_i U psi^i with U = L^{-1} R and
// D_i = diag(m_j exp(-i dt E_i x_j)); outputs
// a_i = dx sum_j |psi^i_j|^2 (V'_j + E_i)  (section "Microscopic Response in
// XUV regime (TDSE)", Eq. dipole acceleration).
//
// For a loss l(a) with abar_i = dl/da_i the costate lambda^i = dl/dpsi^i
// (dl = Re <lambda, dpsi>) obeys
//   lambda^nt = 2 abar_nt dx (V' + E_nt) psi^nt,
//   lambda^i  = U^H D_i^H lambda^{i+1} + 2 abar_i dx (V' + E_i) psi^i,
// and dl/dE_i = abar_i n_i + dt sum_j x_j Im(conj(lambda^{i+1}_j) psi^{i+1}_j).
// U is the Cayley transform of the real symmetric Numerov Hamiltonian
// H = M2^{-1}(-D2/2) + V, so U is complex symmetric and U^H = conj(U).
// Working with kappa = conj(lambda) the backward step is therefore the same
// Crank-Nicolson core as the forward step, applied after the phase:
//   kappa^i = U (D_i kappa^{i+1}) + 2 abar_i dx (V' + E_i) conj(psi^i),
//   dl/dE_i = abar_i n_i + dt sum_j x_j Im(kappa^{i+1}_j psi^{i+1}_j).
// psi^i is recomputed segment by segment from checkpoints stored every K
// steps during an initial forward pass; segment states live in a per-slot
// HBM buffer in the lane-interleaved layout (coalesced 16 B per lane), chunk
// values only (the ghosts are read from the neighbouring lanes' entries).
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

namespace {

template <int C>
__device__ __forceinline__ void load_state(const double* base, int T, unsigned off, cd (&v)[C],
                                           cd& gl, cd& gr)
{
    const cd* b = reinterpret_cast<const cd*>(base);
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = ld_lane(b + (size_t)k * T, off);
    gl = ld_lane(b + (size_t)C * T, off);
    gr = ld_lane(b + (size_t)(C + 1) * T, off);
}

// Segment record: the chunk values only, [C][T] complex.  The ghosts are the
// neighbouring lanes' end values, read back from the same record (the same
// cache lines as the lane's own loads); outside the grid they are zero, as
// in the forward step.  The offsets are clamped so that every load stays in
// the record.
template <int C>
__device__ __forceinline__ void store_chunk(double* base, int T, unsigned off, const cd (&v)[C])
{
#pragma unroll
    for (int k = 0; k < C; ++k) st_lane(base + 2 * (size_t)k * T, off, v[k]);
}

template <int C>
__device__ __forceinline__ void chunk_ghosts(const cd* b, int T, int t, unsigned off, cd& gl, cd& gr)
{
    const cd l = ld_lane(b + (size_t)(C - 1) * T, t > 0 ? off - 16u : off);
    const cd r = ld_lane(b, t + 1 < T ? off + 16u : off);
    gl = t > 0 ? l : czero();
    gr = t + 1 < T ? r : czero();
}

template <int C>
__device__ __forceinline__ void load_chunk(const double* base, int T, int t, unsigned off,
                                           cd (&v)[C], cd& gl, cd& gr)
{
    const cd* b = reinterpret_cast<const cd*>(base);
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = ld_lane(b + (size_t)k * T, off);
    chunk_ghosts<C>(b, T, t, off, gl, gr);
}

// Outputs of the forward pass for samples [a0, a1]: the acceleration, <x> and
// norm rows the caller asked for, and the norm row the reverse sweep uses.
// Flags as in the forward kernel: bit 0 non-finite output, bit 1 the norm
// grew by more than 1e-8 relative to sample 0 (n0 < 0: not known yet).
__device__ __forceinline__ void flush_fwd(int a0, int a1, int t, int T, const double* ring, int W,
                                          double dx, const double* erow, double* acc_row,
                                          double* x_row, double* nu_row, double* n_row, double n0,
                                          int* flag)
{
    for (int smp = a0 + t; smp <= a1; smp += T) {
        const double* r = ring + (smp % kRing) * W * 3;
        double sv = 0.0, sx = 0.0, sn = 0.0;
        for (int w = 0; w < W; ++w) {
            sv += r[w * 3 + 0];
            sx += r[w * 3 + 1];
            sn += r[w * 3 + 2];
        }
        const double nn = dx * sn;
        const double acc = dx * fma(erow[smp], sn, sv);
        if (acc_row) acc_row[smp] = acc;
        if (x_row) x_row[smp] = dx * sx;
        if (nu_row) nu_row[smp] = nn;
        n_row[smp] = nn;
        int f = 0;
        if (!isfinite(acc) || !isfinite(nn) || !isfinite(sx)) f |= 1;
        if (n0 >= 0.0 && nn > n0 * (1.0 + 1e-8)) f |= 2;
        if (f) atomicOr(flag, f);
    }
}

// dx sum |psi|^2 of sample 0 from its ring slot (intact until sample kRing).
__device__ __forceinline__ double ring_norm0(const double* ring, int W, double dx)
{
    double sn = 0.0;
    for (int w = 0; w < W; ++w) sn += ring[w * 3 + 2];
    return dx * sn;
}

// grad_i = abar_i n_i + dt * sum_w partial_w(i) for i in [a0, a1]
__device__ __forceinline__ void flush_grad(int a0, int a1, int t, int T, const double* ring,
                                           int W, double dt, const double* abar,
                                           const double* n_row, double* g_row, int* flag)
{
    for (int smp = a0 + t; smp <= a1; smp += T) {
        const double* r = ring + (smp % kRing) * W;
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += r[w];
        const double g = fma(abar[smp], n_row[smp], dt * s);
        g_row[smp] = g;
        if (!isfinite(g)) atomicOr(flag, 1);
    }
}

// sum_j x_j Im(kappa_j psi_j) over the lane's chunk, reduced over the wave.
template <int C>
__device__ __forceinline__ void grad_partial(const cd (&kap)[C], const cd (&psi)[C], double xs,
                                             double dx, const LaneCtx& lc, double* slot)
{
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double im = fma(kap[k].re, psi[k].im, kap[k].im * psi[k].re);
        s0 += im;
        s1 = fma((double)k, im, s1);
    }
    double g = wave_sum(fma(xs, s0, dx * s1));
    if (lc.lane == kSumLane) slot[lc.wave] = g;
}

// kappa += c_j conj(psi_j) with c_j = ci (V'_j + e), on the chunk and ghosts.
template <int C, class TV>
__device__ __forceinline__ void add_source(cd (&kap)[C], cd& kgl, cd& kgr, const cd (&psi)[C],
                                           cd gl, cd gr, double ci, double e, const TV& tb,
                                           int T, const LaneCtx& lc)
{
#pragma unroll
    for (int k = 0; k < C; ++k)
        kap[k] = cadd(kap[k], cscale(ci * (tb.dv(lc.b0 + 64 * k) + e), cconj(psi[k])));
    // the clamped neighbour indices of the end lanes meet zero ghost values
    kgl = cadd(kgl, cscale(ci * (tb.dv(lc.il()) + e), cconj(gl)));
    kgr = cadd(kgr, cscale(ci * (tb.dv(lc.ir()) + e), cconj(gr)));
}

// add_source and grad_partial in one pass that reads psi^i from its segment
// record one point at a time, for chunks too long to hold psi and the
// costate in registers together.  Same operations in the same order, so the
// results are those of load_chunk followed by the two calls above.
template <int C, class TV>
__device__ __forceinline__ void source_grad_streamed(cd (&kap)[C], cd& kgl, cd& kgr,
                                                     const double* rec, int T, int t, unsigned off,
                                                     double ci, double e, const TV& tb,
                                                     const LaneCtx& lc, bool want_grad, double xs,
                                                     double dx, double* slot)
{
    const cd* b = reinterpret_cast<const cd*>(rec);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const cd p = ld_lane(b + (size_t)k * T, off);
        kap[k] = cadd(kap[k], cscale(ci * (tb.dv(lc.b0 + 64 * k) + e), cconj(p)));
        const double im = fma(kap[k].re, p.im, kap[k].im * p.re);
        s0 += im;
        s1 = fma((double)k, im, s1);
    }
    cd gl, gr;
    chunk_ghosts<C>(b, T, t, off, gl, gr);
    kgl = cadd(kgl, cscale(ci * (tb.dv(lc.il()) + e), cconj(gl)));
    kgr = cadd(kgr, cscale(ci * (tb.dv(lc.ir()) + e), cconj(gr)));
    if (want_grad) {
        const double g = wave_sum(fma(xs, s0, dx * s1));
        if (lc.lane == kSumLane) slot[lc.wave] = g;
    }
}

// ------------------------------------------------------------ two chains
// The reverse-only sweep advances two independent Crank-Nicolson chains at
// once: the costate of one segment and the recomputation of the segment
// before it.  They share the lane layout, the tables and the carry window
// products, and each carry scan takes one barrier for both, so the two
// chains' instructions interleave in one stream (twice the independent work
// per wavefront at 2 waves per SIMD).  scan_fwd2, scan_bwd2 and cn_apply2
// are scan_fwd, scan_bwd and cn_apply applied to both chains, operation for
// operation, so each chain's results are bitwise those of the single form.
__device__ __forceinline__ void scan_fwd2(cd& z1, cd& z2, cd a0, cd a1, cd aw, const SizeClass& sc,
                                          const LaneCtx& lc, cd* lds1, cd* lds2, cd& out1,
                                          cd& out2)
{
    const unsigned off = 16u * (unsigned)lc.t;
    if (sc.levels > 0) {
        z1 = cmad(a0, wave_shr1(z1), z1);
        z2 = cmad(a0, wave_shr1(z2), z2);
    }
    if (sc.levels > 1) {
        z1 = cmad(a1, wave_shr1(wave_shr1(z1)), z1);
        z2 = cmad(a1, wave_shr1(wave_shr1(z2)), z2);
    }
    for (int lev = 2; lev < sc.levels; ++lev) {
        const int d = 1 << lev;
        const cd zs1 = shfl_up_c(z1, d), zs2 = shfl_up_c(z2, d);
        const cd p = ld_lane(sc.lt.pa + lev * sc.T, off);
        if (lc.lane >= d) {
            z1 = cmad(p, zs1, z1);
            z2 = cmad(p, zs2, z2);
        }
    }
    cd prev1 = czero(), prev2 = czero();
    if (lc.W > 1 && lc.lane == kWave - 1) {
        lds1[lc.wave] = z1;
        lds2[lc.wave] = z2;
    }
    __syncthreads();
    if (lc.W > 1) {
        const int v0 = max(0, lc.wave - sc.xwaves);
        if (v0 < lc.wave) {
            prev1 = lds1[v0];
            prev2 = lds2[v0];
            for (int w = v0 + 1; w < lc.wave; ++w) {
                const cd pw = ldg(sc.lt.pw + w * kWave + kWave - 1);
                prev1 = cmad(pw, prev1, lds1[w]);
                prev2 = cmad(pw, prev2, lds2[w]);
            }
        }
        z1 = cmad(aw, prev1, z1);
        z2 = cmad(aw, prev2, z2);
    }
    out1 = wave_shr1_keep(z1, prev1);
    out2 = wave_shr1_keep(z2, prev2);
}

__device__ __forceinline__ void scan_bwd2(cd& y1, cd& y2, cd b0, cd b1, cd bw, const SizeClass& sc,
                                          const LaneCtx& lc, cd* lds1, cd* lds2, cd& out1,
                                          cd& out2)
{
    const unsigned off = 16u * (unsigned)lc.t;
    if (sc.levels > 0) {
        y1 = cmad(b0, wave_shl1(y1), y1);
        y2 = cmad(b0, wave_shl1(y2), y2);
    }
    if (sc.levels > 1) {
        y1 = cmad(b1, wave_shl1(wave_shl1(y1)), y1);
        y2 = cmad(b1, wave_shl1(wave_shl1(y2)), y2);
    }
    for (int lev = 2; lev < sc.levels; ++lev) {
        const int d = 1 << lev;
        const cd ys1 = shfl_down_c(y1, d), ys2 = shfl_down_c(y2, d);
        const cd p = ld_lane(sc.lt.qb + lev * sc.T, off);
        if (lc.lane + d < kWave) {
            y1 = cmad(p, ys1, y1);
            y2 = cmad(p, ys2, y2);
        }
    }
    cd next1 = czero(), next2 = czero();
    if (lc.W > 1 && lc.lane == 0) {
        lds1[lc.wave] = y1;
        lds2[lc.wave] = y2;
    }
    __syncthreads();
    if (lc.W > 1) {
        const int v1 = min(lc.W - 1, lc.wave + sc.xwaves);
        if (v1 > lc.wave) {
            next1 = lds1[v1];
            next2 = lds2[v1];
            for (int w = v1 - 1; w > lc.wave; --w) {
                const cd qw = ldg(sc.lt.qw + w * kWave);
                next1 = cmad(qw, next1, lds1[w]);
                next2 = cmad(qw, next2, lds2[w]);
            }
        }
        y1 = cmad(bw, next1, y1);
        y2 = cmad(bw, next2, y2);
    }
    out1 = wave_shl1_keep(y1, next1);
    out2 = wave_shl1_keep(y2, next2);
}

// cn_apply (real time, q in registers) on two chunk states.
template <int C, class TV, class LF>
__device__ __forceinline__ void cn_apply2(cd (&v1)[C], cd& gl1, cd& gr1, cd (&v2)[C], cd& gl2,
                                          cd& gr2, const LF& f, const TV& tb, const SizeClass& sc,
                                          const LaneCtx& lc, const RhsCoef rc, cd* lf1, cd* lb1,
                                          cd* lf2, cd* lb2)
{
    static_assert(LF::kRegs, "two chains need the pivot factors in registers");
    constexpr bool RT = true;
    const int b0 = lc.b0;
    const unsigned off = 16u * (unsigned)lc.t;
    const double oml = tb.om(lc.il());
    const double omr = tb.om(lc.ir());
    cd a0 = czero(), a1 = czero(), aw = czero();
    // A. right-hand sides in place, chunk-end values with zero carry-in
    cd ze1 = czero(), ze2 = czero();
    {
        double om_p = oml;
        double om_c = tb.om(b0);
        double om_n = C > 1 ? tb.om(b0 + 64) : omr;
        cd gp1 = gfac<RT>(oml, gl1), gp2 = gfac<RT>(oml, gl2);
        cd gc1 = gfac<RT>(om_c, v1[0]), gc2 = gfac<RT>(om_c, v2[0]);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if (k == C / 2) {
                if (sc.levels > 0) a0 = ld_lane(sc.lt.pa, off);
                if (sc.levels > 1) a1 = ld_lane(sc.lt.pa + sc.T, off);
                if (lc.lane < (1 << sc.levels)) aw = ld_lane(sc.lt.pw, off);
            }
            // om of the point after next, issued one point ahead of its use
            const double om_nn = (k + 2 < C) ? tb.om(b0 + 64 * (k + 2)) : omr;
            TDSE_POINT_FENCE();
            const cd al = f.template alpha<RT>(k, om_p, sc, lc);
            const cd gn1 = gfac<RT>(om_n, (k + 1 < C) ? v1[k + 1] : gr1);
            const cd gn2 = gfac<RT>(om_n, (k + 1 < C) ? v2[k + 1] : gr2);
            // gh = g - i (dofs/10) psi from g, as cn_apply forms it in real time
            const cd gh1 = mkc(fma(rc.dofs10, v1[k].im, gc1.re), fma(-rc.dofs10, v1[k].re, gc1.im));
            const cd gh2 = mkc(fma(rc.dofs10, v2[k].im, gc2.re), fma(-rc.dofs10, v2[k].re, gc2.im));
            const cd r1 = mkc(fma(10.0, gh1.re, gp1.re + gn1.re), fma(10.0, gh1.im, gp1.im + gn1.im));
            const cd r2 = mkc(fma(10.0, gh2.re, gp2.re + gn2.re), fma(10.0, gh2.im, gp2.im + gn2.im));
            v1[k] = r1;
            v2[k] = r2;
            ze1 = (k == 0) ? r1 : cmad(al, ze1, r1);
            ze2 = (k == 0) ? r2 : cmad(al, ze2, r2);
            gp1 = gc1;
            gc1 = gn1;
            gp2 = gc2;
            gc2 = gn2;
            om_p = om_c;
            om_c = om_n;
            om_n = om_nn;
            point_fence(ze1, ze2);
        }
    }
    cd cf1, cf2;
    scan_fwd2(ze1, ze2, a0, a1, aw, sc, lc, lf1, lf2, cf1, cf2);
    cd b0c = czero(), b1c = czero(), bw = czero();
    if (sc.levels > 0) b0c = ld_lane(sc.lt.qb, off);
    if (sc.levels > 1) b1c = ld_lane(sc.lt.qb + sc.T, off);
    if (lc.lane > kWave - 1 - (1 << sc.levels)) bw = ld_lane(sc.lt.qw, off);
    // B. forward recurrences from the exact carries, w = q z; each point
    // issues the next one's om load first (at the last point sweep C's)
    double om_last;
    {
        cd z1 = cf1, z2 = cf2;
        double om_p = oml;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const double om_k = tb.om(b0 + 64 * k);
            TDSE_POINT_FENCE();
            const cd al = f.template alpha<RT>(k, om_p, sc, lc);
            const cd qk = f.q(k, sc, lc);
            z1 = cmad(al, z1, v1[k]);
            z2 = cmad(al, z2, v2[k]);
            v1[k] = cmul(qk, z1);
            v2[k] = cmul(qk, z2);
            om_p = om_k;
            point_fence(v1[k], v2[k]);
        }
        om_last = om_p;
    }
    // C. chunk-start values with zero carry-in (om one point ahead)
    cd yb1 = v1[C - 1], yb2 = v2[C - 1];
    {
        double om_n = om_last;
#pragma unroll
        for (int k = C - 2; k >= 0; --k) {
            const double om_k = k > 0 ? tb.om(b0 + 64 * k) : 0.0;
            TDSE_POINT_FENCE();
            const cd be = f.template beta<RT>(k, om_n, sc, lc);
            yb1 = cmad(be, yb1, v1[k]);
            yb2 = cmad(be, yb2, v2[k]);
            om_n = om_k;
            point_fence(yb1, yb2);
        }
    }
    cd cb1, cb2;
    scan_bwd2(yb1, yb2, b0c, b1c, bw, sc, lc, lb1, lb2, cb1, cb2);
    // D. backward recurrences from the exact carries
    double om_0;
    {
        cd y1 = cb1, y2 = cb2;
        double om_n = omr;
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            const double om_k = tb.om(b0 + 64 * k);  // the next point's (om_0 last)
            TDSE_POINT_FENCE();
            const cd be = f.template beta<RT>(k, om_n, sc, lc);
            y1 = cmad(be, y1, v1[k]);
            y2 = cmad(be, y2, v2[k]);
            v1[k] = y1;
            v2[k] = y2;
            om_n = om_k;
            point_fence(y1, y2);
        }
        om_0 = om_n;
    }
    const cd ql = f.ql(sc, lc);
    const cd e0 = elim<RT>(om_0, ql);
    gl1 = cmad(ql, cf1, cmul(e0, v1[0]));
    gl2 = cmad(ql, cf2, cmul(e0, v2[0]));
    gr1 = cb1;
    gr2 = cb2;
}

}  // namespace

// REV: the reverse sweep alone (tdse_adjoint_batch_stored: the checkpoints
// were stored by the forward kernel).  Without the forward pass in the same
// kernel, the costate is parked in the slot while a segment is recomputed
// and psi^i is read point by point at every chunk length, which leaves room
// for the pivot factors in registers up to 8 points per lane.
// NARROW: workgroups of at most 512 threads (2 waves per SIMD, 256
// registers per lane) instead of 1024 (4 waves, 128).  The adjoint holds the
// costate, the pivot factors and the recomputed state together; at 128
// registers the 8-point layout spilled about 80 of them per lane.
template <int C, bool LDSTAB, bool AB = false, bool REV = false, bool NARROW = false>
__global__ void __launch_bounds__(NARROW ? 512 : 1024) adjoint_kernel(FwdArgs a)
{
    // the costate doubles the chunk state: at 128 registers the pivot factors
    // stay in registers only for 4 points per lane, and from 16 points (or in
    // the reverse-only sweep) the costate is parked in the slot while a
    // segment is recomputed and psi^i is read point by point.  The narrow
    // instances (256 registers) keep q in registers up to 8 points and load
    // psi^i ahead of the costate step, so its latency overlaps the step.
    constexpr bool kAdjQRegs = (REV || NARROW) ? C <= 8 : C <= 4;
    constexpr bool kStream = (REV && !NARROW) || C >= 16;
    // the narrow reverse-only sweep runs the costate and the recomputation
    // as two chains in one instruction stream (two segment buffers)
    constexpr bool kDual = REV && NARROW && C <= 8;
    extern __shared__ double smem_raw[];
    const SizeClass sc = uniform_load(a.classes + a.cls);
    const int T = sc.T, W = T / kWave, np = C * T;
    const int S = blockDim.x / T;
    const int tid = threadIdx.x, sub = uniform(tid / T), t = tid - sub * T;
    const int wsys = uniform(t / kWave);  // wavefront within the system
    const unsigned loff = 16u * (unsigned)t;  // lane offset in state records
    const size_t sb = a.sub_bytes;
    char* per = reinterpret_cast<char*>(smem_raw) + (LDSTAB ? kLdsTableBytes * np : 0);
    const SubSmem sm = carve_sub(per + sub * sb, W);
    int* wg_item = reinterpret_cast<int*>(per + S * sb);
    TableSource<LDSTAB>::make(sc, smem_raw);  // stages the tables once per workgroup
    const double dx = sc.dx;
    const int n = sc.n, s = t * C;
    const SizeClass* const clsp = a.classes + a.cls;
    const int nt = a.nt, K = a.k_ckpt;
    const int nseg = nt / K + 1;
    const size_t np2 = 2 * (size_t)(C + 2) * T;  // doubles per state record
    const size_t nps = 2 * (size_t)C * T;        // doubles per segment record
    double* const slot = a.work + ((size_t)blockIdx.x * S + sub) * (size_t)a.slot_doubles;
    double* ring = sm.ring;
    int* flag = sm.misc + 1;

    for (;;) {
        if (tid == 0) {
            wg_item[0] = atomicAdd(a.queue, S);
            wg_item[1] = 0;
        }
        if (t == 0) {
            sm.misc[1] = 0;
            sm.misc[2] = 0;
        }
        __syncthreads();
        const int base = uniform(wg_item[0]);
        if (base >= a.count) break;
        const int item = base + sub;
        const bool active = item < a.count;  // uniform within the subgroup
        const int p = active ? uniform(a.order[item]) : 0;
        const SysDesc d = uniform_load(a.sys + p);
        const size_t row = (size_t)p * (size_t)(nt + 1);
        const double* erow = a.E + row;
        const double* abar = a.abar ? a.abar + row : nullptr;
        double* g_row = a.grad ? a.grad + row : nullptr;
        double* acc_row = (active && a.accel) ? a.accel + row : nullptr;
        double* x_row = (active && a.xexp) ? a.xexp + row : nullptr;
        double* nu_row = (active && a.norm) ? a.norm + row : nullptr;
        const double* src = REV ? nullptr : (a.psi0 ? a.psi0 + 2 * d.psi_off : a.gs + 2 * a.gs_off[a.cls]);
        // checkpoints and norm row: the system's own (stored) or the slot's
        double* ckpt = a.store ? a.store + uniform_load(a.store_off + p) : slot;
        double* n_row = ckpt + np2 * nseg;
        double* seg = a.store ? slot : n_row + ((nt + 2) & ~1);
        double* kbuf = seg + nps * (K + 1);  // parked costate (one state record)

        // rows with an all-zero abar have a zero gradient and need no reverse sweep
        if (active && a.mode != kAdjForwardOnly)
            for (int i = t; i <= nt; i += T)
                if (abar[i] != 0.0) {
                    sm.misc[2] = 1;
                    wg_item[1] = 1;
                }
        __syncthreads();
        const bool need_grad = uniform(sm.misc[2]) != 0;
        const bool wg_need = uniform(wg_item[1]) != 0;  // uniform over the workgroup

        // ---------------- forward pass: outputs, norms, checkpoints
        cd v[C];
        cd gl = czero(), gr = czero();
        if constexpr (!REV) {
#pragma unroll
            for (int k = 0; k < C; ++k) v[k] = (active && s + k < n) ? ld_psi(src, s + k) : czero();
            gl = (active && s > 0 && s - 1 < n) ? ld_psi(src, s - 1) : czero();
            gr = (active && s + C < n) ? ld_psi(src, s + C) : czero();
        }
        LaneFactors<C, kAdjQRegs, AB> f;
        {
            const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
            f = load_factors<C, kAdjQRegs, AB>(sv.sc, sv.lc);
        }
        if constexpr (!REV) {
        int flushed = 0;
        // forward pass length (uniform): none when the checkpoints are stored
        const int nfwd = a.mode == kAdjReverseOnly ? -1
                         : (a.mode == kAdjForwardOnly || wg_need || a.accel) ? nt : -1;
        double n0 = -1.0;
        for (int i = 0; i <= nfwd; ++i) {
            const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
            if (i % K == 0) store_state<C>(ckpt + np2 * (i / K), T, loff, v, gl, gr);
            observe<C>(v, sv.tb, T, sv.lc, sv.xs, dx, ring + (i % kRing) * W * 3);
            if (i == nt) break;
            forward_step<C>(v, gl, gr, f, erow[i], RatioNow{erow[i], a.dt, sv.sc.dx}, a.dt, sv.xl,
                            sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
            if ((i + 1) % kFlush == 0) {
                __syncthreads();
                if (flushed == 0) n0 = ring_norm0(ring, W, dx);
                if (active)
                    flush_fwd(i + 1 - kFlush, i, t, T, ring, W, dx, erow, acc_row, x_row, nu_row,
                              n_row, n0, flag);
                flushed = i + 1;
            }
        }
        __syncthreads();
        if (nfwd >= 0) {
            if (flushed == 0) n0 = ring_norm0(ring, W, dx);
            if (active)
                flush_fwd(flushed, nt, t, T, ring, W, dx, erow, acc_row, x_row, nu_row, n_row, n0,
                          flag);
            if (active && a.psi_final) {
                double* dst = a.psi_final + 2 * d.psi_off;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    if (s + k < n) {
                        dst[2 * (s + k)] = v[k].re;
                        dst[2 * (s + k) + 1] = v[k].im;
                    }
                }
            }
        }
        __syncthreads();
        }  // forward pass

        // ---------------- reverse sweep (every subgroup runs it, so barriers
        // stay uniform; subgroups without a gradient write nothing)
        if (active && need_grad && t == 0) g_row[nt] = abar[nt] * n_row[nt];
        cd kap[C];
#pragma unroll
        for (int k = 0; k < C; ++k) kap[k] = czero();
        cd kgl = czero(), kgr = czero();
        if constexpr (kDual) {
        // ---- two chains: while the costate runs backwards through segment
        // sidx (read from one segment buffer), the segment before it is
        // recomputed into the other.  In the reverse-only sweep the ring
        // holds one value per wavefront and sample (the gradient partials),
        // so its upper part carries the second chain's carry slots.
        cd* const lf2 = reinterpret_cast<cd*>(ring + kRing * W);
        cd* const lb2 = lf2 + W;
        double* const seg2 = kbuf + np2;
        auto buf = [&](int sx) { return (sx & 1) ? seg2 : seg; };
        if (wg_need) {
            // the last segment is recomputed alone
            const int sl = nseg - 1;
            const int s0l = sl * K, s1l = min(s0l + K, nt);
            load_state<C>(ckpt + np2 * sl, T, loff, v, gl, gr);
            store_chunk<C>(buf(sl), T, loff, v);
            for (int i = s0l; i < s1l; ++i) {
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                forward_step<C>(v, gl, gr, f, erow[i], RatioNow{erow[i], a.dt, sv.sc.dx}, a.dt,
                                sv.xl, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
                store_chunk<C>(buf(sl) + nps * (i - s0l + 1), T, loff, v);
            }
            {
                // kappa^nt = 2 abar_nt dx (V' + E_nt) conj(psi^nt), psi^nt = v
                // with the ghosts of its stored record
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                __syncthreads();
                chunk_ghosts<C>(reinterpret_cast<const cd*>(buf(sl) + nps * (s1l - s0l)), T, t, loff,
                                gl, gr);
                add_source<C>(kap, kgl, kgr, v, gl, gr, 2.0 * abar[nt] * dx, erow[nt], sv.tb, T,
                              sv.lc);
                if (nt > 0) grad_partial<C>(kap, v, sv.xs, dx, sv.lc, ring + ((nt - 1) % kRing) * W);
                if (nt > 0 && (nt - 1) % kFlush == 0) {
                    __syncthreads();
                    if (active && need_grad)
                        flush_grad(nt - 1, nt - 1, t, T, ring, W, a.dt, abar, n_row, g_row, flag);
                }
            }
            // one costate step i: kappa <- U (D_i kappa) + source(psi^i), and
            // the partial of grad_{i-1}; psi^i read from its record first
            auto costate_tail = [&](int i, int s0, const double* bc) {
                const double e = erow[i];
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                cd pv[C], pgl, pgr;
                load_chunk<C>(bc + nps * (i - s0), T, t, loff, pv, pgl, pgr);
                phase_mask<C, !kAdjQRegs>(kap, kgl, kgr, e, a.dt, sv.xl, phase_ratio(e, a.dt, dx),
                                          f.mflags, sv.sc, sv.lc);
                cn_apply<C, true>(kap, kgl, kgr, f, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
                add_source<C>(kap, kgl, kgr, pv, pgl, pgr, 2.0 * abar[i] * dx, e, sv.tb, T, sv.lc);
                if (i > 0) grad_partial<C>(kap, pv, sv.xs, dx, sv.lc, ring + ((i - 1) % kRing) * W);
            };
            auto grad_flush = [&](int i) {
                if (i > 0 && (i - 1) % kFlush == 0) {
                    __syncthreads();
                    if (active && need_grad)
                        flush_grad(i - 1, min(i - 1 + kFlush - 1, nt - 1), t, T, ring, W, a.dt,
                                   abar, n_row, g_row, flag);
                }
            };
            for (int sidx = sl; sidx >= 0; --sidx) {
                const int s0 = sidx * K, s1 = min(s0 + K, nt);
                const int ncost = s1 - s0;           // costate steps of segment sidx
                const int nrec = sidx > 0 ? K : 0;   // recompute steps of segment sidx - 1
                const int r0 = s0 - K;
                const double* const bc = buf(sidx);
                double* const br = buf(sidx + 1);    // the other buffer
                if (nrec > 0) {
                    load_state<C>(ckpt + np2 * (sidx - 1), T, loff, v, gl, gr);
                    store_chunk<C>(br, T, loff, v);
                }
                const int both = min(ncost, nrec);
                for (int it = 0; it < both; ++it) {
                    const int i = s1 - 1 - it, ir = r0 + it;
                    const double e = erow[i];
                    const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                    cd pv[C], pgl, pgr;
                    load_chunk<C>(bc + nps * (i - s0), T, t, loff, pv, pgl, pgr);
                    phase_mask<C, !kAdjQRegs>(kap, kgl, kgr, e, a.dt, sv.xl,
                                              phase_ratio(e, a.dt, dx), f.mflags, sv.sc, sv.lc);
                    cn_apply2<C>(kap, kgl, kgr, v, gl, gr, f, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f,
                                 sm.lds_b, lf2, lb2);
                    phase_mask<C, !kAdjQRegs>(v, gl, gr, erow[ir], a.dt, sv.xl,
                                              phase_ratio(erow[ir], a.dt, dx), f.mflags, sv.sc,
                                              sv.lc);
                    store_chunk<C>(br + nps * (it + 1), T, loff, v);
                    add_source<C>(kap, kgl, kgr, pv, pgl, pgr, 2.0 * abar[i] * dx, e, sv.tb, T,
                                  sv.lc);
                    if (i > 0)
                        grad_partial<C>(kap, pv, sv.xs, dx, sv.lc, ring + ((i - 1) % kRing) * W);
                    grad_flush(i);
                }
                // the costate alone (segment 0 has no segment before it)
                for (int it = both; it < ncost; ++it) {
                    costate_tail(s1 - 1 - it, s0, bc);
                    grad_flush(s1 - 1 - it);
                }
                // the recomputation alone (after a last segment shorter than K)
                for (int it = both; it < nrec; ++it) {
                    const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                    forward_step<C>(v, gl, gr, f, erow[r0 + it],
                                    RatioNow{erow[r0 + it], a.dt, sv.sc.dx}, a.dt, sv.xl, sv.tb,
                                    sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
                    store_chunk<C>(br + nps * (it + 1), T, loff, v);
                }
            }
        }
        } else {
        bool started = false;
        for (int sidx = wg_need ? nseg - 1 : -1; sidx >= 0; --sidx) {
            const int s0 = sidx * K;
            const int s1 = min(s0 + K, nt);
            // recompute psi^{s0..s1} into the segment buffer
            if constexpr (kStream) {
                // the streamed reads of the previous segment's states (after
                // the last costate step's barriers) are done in every wave
                // before its first state is overwritten
                __syncthreads();
                store_state<C>(kbuf, T, loff, kap, kgl, kgr);
            }
            load_state<C>(ckpt + np2 * sidx, T, loff, v, gl, gr);
            store_chunk<C>(seg, T, loff, v);
            for (int i = s0; i < s1; ++i) {
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                forward_step<C>(v, gl, gr, f, erow[i], RatioNow{erow[i], a.dt, sv.sc.dx}, a.dt,
                                sv.xl, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
                store_chunk<C>(seg + nps * (i - s0 + 1), T, loff, v);
            }
            if constexpr (kStream) load_state<C>(kbuf, T, loff, kap, kgl, kgr);
            if (!started) {
                // kappa^nt = 2 abar_nt dx (V' + E_nt) conj(psi^nt); psi^nt = v
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                if constexpr (kStream) {
                    // psi^nt was just stored; its ghosts are other waves' entries
                    __syncthreads();
                    source_grad_streamed<C>(kap, kgl, kgr, seg + nps * (s1 - s0), T, t, loff,
                                            2.0 * abar[nt] * dx, erow[nt], sv.tb, sv.lc, nt > 0,
                                            sv.xs, dx, ring + ((nt > 0 ? nt - 1 : 0) % kRing) * W);
                } else {
                    // the ghosts of psi^nt as every later step reads them: the
                    // neighbouring lanes' entries of the stored state (the
                    // streamed form and the reverse-only kernel do the same)
                    __syncthreads();
                    chunk_ghosts<C>(reinterpret_cast<const cd*>(seg + nps * (s1 - s0)), T, t, loff,
                                    gl, gr);
                    add_source<C>(kap, kgl, kgr, v, gl, gr, 2.0 * abar[nt] * dx, erow[nt], sv.tb,
                                  T, sv.lc);
                    if (nt > 0)
                        grad_partial<C>(kap, v, sv.xs, dx, sv.lc, ring + ((nt - 1) % kRing) * W);
                }
                started = true;
                if (nt > 0 && (nt - 1) % kFlush == 0) {
                    __syncthreads();
                    if (active && need_grad)
                        flush_grad(nt - 1, nt - 1, t, T, ring, W, a.dt, abar, n_row, g_row, flag);
                }
            }
            for (int i = s1 - 1; i >= s0; --i) {
                // kappa <- U (D_i kappa)
                const double e = erow[i];
                const StepView<LDSTAB> sv = step_view<LDSTAB>(clsp, wsys, smem_raw);
                // psi^i is loaded first: its latency overlaps the costate step
                if constexpr (!kStream) load_chunk<C>(seg + nps * (i - s0), T, t, loff, v, gl, gr);
                phase_mask<C, !kAdjQRegs>(kap, kgl, kgr, e, a.dt, sv.xl, phase_ratio(e, a.dt, dx),
                                          f.mflags, sv.sc, sv.lc);
                cn_apply<C, true>(kap, kgl, kgr, f, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
                // + 2 abar_i dx (V' + E_i) conj(psi^i), and the partial of
                // grad_{i-1} from kappa^i and psi^i
                if constexpr (kStream) {
                    source_grad_streamed<C>(kap, kgl, kgr, seg + nps * (i - s0), T, t, loff,
                                            2.0 * abar[i] * dx, e, sv.tb, sv.lc, i > 0, sv.xs, dx,
                                            ring + ((i > 0 ? i - 1 : 0) % kRing) * W);
                } else {
                    add_source<C>(kap, kgl, kgr, v, gl, gr, 2.0 * abar[i] * dx, e, sv.tb, T, sv.lc);
                    if (i > 0) grad_partial<C>(kap, v, sv.xs, dx, sv.lc, ring + ((i - 1) % kRing) * W);
                }
                if (i > 0) {
                    if ((i - 1) % kFlush == 0) {
                        __syncthreads();
                        if (active && need_grad)
                            flush_grad(i - 1, min(i - 1 + kFlush - 1, nt - 1), t, T, ring, W, a.dt,
                                       abar, n_row, g_row, flag);
                    }
                }
            }
        }
        }  // single chain
        if (active && !need_grad && a.mode != kAdjForwardOnly)
            for (int i = t; i <= nt; i += T) g_row[i] = 0.0;
        __syncthreads();
        if (active && t == 0 && a.status) a.status[p] = sm.misc[1];
    }
}

// Copies checkpoint `index` (the state at step index * K) of every system out
// of the per-system store into a ragged wavefunction buffer in natural point
// order: point j = t C + k of the lane-chunked record [k][t].
__global__ void __launch_bounds__(256) stored_state_kernel(const SizeClass* classes,
                                                           const SysDesc* sys, const double* store,
                                                           const int64_t* store_off, int index,
                                                           double* psi_out)
{
    const int b = blockIdx.y;
    const SysDesc d = sys[b];
    const SizeClass& sc = classes[d.cls];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sc.n) return;
    const size_t np2 = 2 * (size_t)(sc.C + 2) * sc.T;
    const double* rec = store + store_off[b] + np2 * (size_t)index;
    const size_t at = 2 * ((size_t)(j % sc.C) * sc.T + (size_t)(j / sc.C));
    psi_out[2 * (d.psi_off + j)] = rec[at];
    psi_out[2 * (d.psi_off + j) + 1] = rec[at + 1];
}

hipError_t launch_stored_state(const SizeClass* classes, const SysDesc* sys, int batch, int n_max,
                               const double* store, const int64_t* store_off, int index,
                               double* psi_out, hipStream_t st)
{
    hipLaunchKernelGGL(stored_state_kernel, dim3((n_max + 255) / 256, batch), dim3(256), 0, st,
                       classes, sys, store, store_off, index, psi_out);
    return hipGetLastError();
}

size_t adjoint_smem_bytes(int C, int T, int S, bool lds_tables)
{
    return (lds_tables ? (size_t)kLdsTableBytes * C * T : 0) + S * sub_smem_bytes(T / kWave) +
           16;
}

template <int C, bool L, bool REV, bool NARROW>
static int occ_adj(int threads, size_t sh)
{
    int nb = 0;
    void (*k)(FwdArgs) = adjoint_kernel<C, L, false, REV, NARROW>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)) != hipSuccess ||
        threads > fa.maxThreadsPerBlock)
        return 0;  // beyond the kernel's launch bounds
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, sh) != hipSuccess) return 0;
    return nb;
}

template <bool REV, bool NARROW>
static int adjoint_occupancy_t(int C, int th, size_t sh, bool lds_tables)
{
    switch (C * 2 + (lds_tables ? 1 : 0)) {
        case 8: return occ_adj<4, false, REV, NARROW>(th, sh);
        case 9: return occ_adj<4, true, REV, NARROW>(th, sh);
        case 16: return occ_adj<8, false, REV, NARROW>(th, sh);
        case 17: return occ_adj<8, true, REV, NARROW>(th, sh);
        case 32: return occ_adj<16, false, REV, NARROW>(th, sh);
        case 33: return occ_adj<16, true, REV, NARROW>(th, sh);
        default: return 0;
    }
}

bool adjoint_narrow(int threads) { return threads <= 512; }

int adjoint_occupancy(int C, int T, int S, bool lds_tables, bool stored)
{
    const size_t sh = adjoint_smem_bytes(C, T, S, lds_tables);
    if (sh > (size_t)kMaxLds) return 0;
    const int th = S * T;
    // a plan with stored checkpoints launches both instances with one
    // packing: the reverse-only one bounds it
    if (adjoint_narrow(th)) {
        if (stored && adjoint_occupancy_t<true, true>(C, th, sh, lds_tables) < 1) return 0;
        return adjoint_occupancy_t<false, true>(C, th, sh, lds_tables);
    }
    if (stored && adjoint_occupancy_t<true, false>(C, th, sh, lds_tables) < 1) return 0;
    return adjoint_occupancy_t<false, false>(C, th, sh, lds_tables);
}

template <bool REV, bool NARROW>
static hipError_t launch_adjoint_t(int C, bool lds_tables, const FwdArgs& a, int T, int S, int grid,
                                   hipStream_t st)
{
    const size_t sh = adjoint_smem_bytes(C, T, S, lds_tables);
    const dim3 b(T * S);
    // 16 points per lane: elimination factors from their tables (a.ab) or
    // formed from q and om.  At 8 points the tables measured 26 % slower on
    // the 256 on-axis systems of the full focal volume (N = 8192), so that
    // layout always forms them.
    switch (C * 4 + (lds_tables ? 2 : 0) + (a.ab && C > 8 ? 1 : 0)) {
        case 16: hipLaunchKernelGGL((adjoint_kernel<4, false, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 18: hipLaunchKernelGGL((adjoint_kernel<4, true, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 32: hipLaunchKernelGGL((adjoint_kernel<8, false, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 34: hipLaunchKernelGGL((adjoint_kernel<8, true, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 64: hipLaunchKernelGGL((adjoint_kernel<16, false, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 65: hipLaunchKernelGGL((adjoint_kernel<16, false, true, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 66: hipLaunchKernelGGL((adjoint_kernel<16, true, false, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        case 67: hipLaunchKernelGGL((adjoint_kernel<16, true, true, REV, NARROW>), dim3(grid), b, sh, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(int C, bool lds_tables, const FwdArgs& a, int T, int S, int grid,
                          hipStream_t st)
{
    const bool nar = adjoint_narrow(S * T);
    if (a.mode == kAdjReverseOnly)
        return nar ? launch_adjoint_t<true, true>(C, lds_tables, a, T, S, grid, st)
                   : launch_adjoint_t<true, false>(C, lds_tables, a, T, S, grid, st);
    return nar ? launch_adjoint_t<false, true>(C, lds_tables, a, T, S, grid, st)
               : launch_adjoint_t<false, false>(C, lds_tables, a, T, S, grid, st);
}

// Reorders the systems of one launch so that rows with a non-zero abar come
// first and all-zero rows last (one workgroup per row); a workgroup of the
// adjoint kernel whose systems all have zero rows then skips the reverse
// sweep.  The order within each part depends on scheduling, the per-row
// results do not.
__global__ void __launch_bounds__(256) compact_rows_kernel(const double* abar, int nt,
                                                           const int32_t* order_in, int count,
                                                           int32_t* order_out, int32_t* counters)
{
    __shared__ int nz;
    if (threadIdx.x == 0) nz = 0;
    __syncthreads();
    const int p = order_in[blockIdx.x];
    const double* row = abar + (size_t)p * (size_t)(nt + 1);
    for (int i = threadIdx.x; i <= nt; i += blockDim.x)
        if (row[i] != 0.0) nz = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (nz) order_out[atomicAdd(counters, 1)] = p;
        else order_out[count - 1 - atomicAdd(counters + 1, 1)] = p;
    }
}

hipError_t launch_compact_rows(const double* abar, int nt, const int32_t* order_in, int count,
                               int32_t* order_out, int32_t* counters, hipStream_t st)
{
    hipLaunchKernelGGL(compact_rows_kernel, dim3(count), dim3(256), 0, st, abar, nt, order_in,
                       count, order_out, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------- yield
// A_k = dt sum_i w_i a_i exp(-i 2 pi k i / M), M = nt + 1, w_i = sin^2(pi i / nt),
// for the band bins k = k_lo .. k_lo + nk - 1.  One workgroup per (bin, row);
// each thread sums a contiguous run of samples, advancing both the DFT phase
// and the window by complex rotation from an exact start (k i mod M).
__global__ void __launch_bounds__(256) band_dft_kernel(YieldArgs a)
{
    __shared__ double red[2][256];
    const int kk = blockIdx.x, b = blockIdx.y;
    const int64_t M = (int64_t)a.nt + 1;
    const int64_t k = a.k_lo + kk;
    const int run = (int)((M + blockDim.x - 1) / blockDim.x);
    const int64_t i0 = (int64_t)threadIdx.x * run;
    const int64_t i1 = min(i0 + run, M);
    const double* arow = a.accel + (size_t)b * M;
    double sre = 0.0, sim = 0.0;
    if (i0 < i1) {
        double sp, cp, sr, cr, sw, cw, swr, cwr;
        sincos(-2.0 * M_PI * (double)((k * i0) % M) / (double)M, &sp, &cp);
        sincos(-2.0 * M_PI * (double)k / (double)M, &sr, &cr);
        sincos(M_PI * (double)i0 / (double)a.nt, &sw, &cw);
        sincos(M_PI / (double)a.nt, &swr, &cwr);
        cd ph = mkc(cp, sp), rot = mkc(cr, sr), wz = mkc(cw, sw), wrot = mkc(cwr, swr);
        for (int64_t i = i0; i < i1; ++i) {
            const double wa = wz.im * wz.im * arow[i];
            sre = fma(wa, ph.re, sre);
            sim = fma(wa, ph.im, sim);
            ph = cmul(ph, rot);
            wz = cmul(wz, wrot);
        }
    }
    red[0][threadIdx.x] = sre;
    red[1][threadIdx.x] = sim;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.amp[2 * ((size_t)b * a.nk + kk)] = a.dt * red[0][0];
        a.amp[2 * ((size_t)b * a.nk + kk) + 1] = a.dt * red[1][0];
    }
}

// yield_b = domega sum_k |A_k|^2 and
// abar_i = 2 domega dt w_i sum_k Re(conj(A_k) exp(-i 2 pi k i / M)), scaled by
// the row weight.  One thread per sample; the phase advances over k.
__global__ void __launch_bounds__(256) band_grad_kernel(YieldArgs a)
{
    const int b = blockIdx.y;
    const int64_t M = (int64_t)a.nt + 1;
    const double dw = 2.0 * M_PI / ((double)M * a.dt);
    const double wgt = a.row_weight ? a.row_weight[b] : 1.0;
    const double* amp = a.amp + 2 * (size_t)b * a.nk;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double y = 0.0;
        for (int kk = 0; kk < a.nk; ++kk) y += amp[2 * kk] * amp[2 * kk] + amp[2 * kk + 1] * amp[2 * kk + 1];
        a.yield[b] = wgt * dw * y;
    }
    if (!a.abar) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double s = 0.0;
    if (a.nk > 0 && wgt != 0.0) {
        double sp, cp, sr, cr;
        sincos(-2.0 * M_PI * (double)(((int64_t)a.k_lo * i) % M) / (double)M, &sp, &cp);
        sincos(-2.0 * M_PI * (double)i / (double)M, &sr, &cr);
        cd ph = mkc(cp, sp);
        const cd rot = mkc(cr, sr);
        for (int kk = 0; kk < a.nk; ++kk) {
            // Re(conj(A) ph) = A.re ph.re + A.im ph.im
            s = fma(amp[2 * kk], ph.re, fma(amp[2 * kk + 1], ph.im, s));
            ph = cmul(ph, rot);
        }
    }
    const double sw = sin(M_PI * (double)i / (double)a.nt);
    a.abar[(size_t)b * M + i] = wgt * 2.0 * dw * a.dt * sw * sw * s;
}

hipError_t launch_band_dft(const YieldArgs& a, hipStream_t st)
{
    if (a.nk < 1) return hipSuccess;
    hipLaunchKernelGGL(band_dft_kernel, dim3(a.nk, a.batch), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_yield(const YieldArgs& a, hipStream_t st)
{
    if (a.nk > 0) {
        hipLaunchKernelGGL(band_dft_kernel, dim3(a.nk, a.batch), dim3(256), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t M = (int64_t)a.nt + 1;
    hipLaunchKernelGGL(band_grad_kernel, dim3((unsigned)((M + 255) / 256), a.batch), dim3(256), 0,
                       st, a);
    return hipGetLastError();
}

}  // namespace tdse
