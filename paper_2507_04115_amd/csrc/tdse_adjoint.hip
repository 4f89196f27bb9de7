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
// HBM buffer in the lane-interleaved layout (coalesced 16 B per lane).
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

namespace {

__host__ __device__ inline size_t adj_smem_bytes(int W)
{
    return sizeof(cd) * 2 * kMaxWaves + sizeof(double) * 2 * kMaxWaves +
           sizeof(double) * kRing * W * 3 + 8 * sizeof(int);
}

// State record: chunk values and the two ghosts, [C+2][T] complex.
template <int C>
__device__ __forceinline__ void store_state(double* base, int T, int t, const cd (&v)[C], cd gl,
                                            cd gr)
{
    double2* b = reinterpret_cast<double2*>(base);
#pragma unroll
    for (int k = 0; k < C; ++k) b[k * T + t] = make_double2(v[k].re, v[k].im);
    b[C * T + t] = make_double2(gl.re, gl.im);
    b[(C + 1) * T + t] = make_double2(gr.re, gr.im);
}

template <int C>
__device__ __forceinline__ void load_state(const double* base, int T, int t, cd (&v)[C], cd& gl,
                                           cd& gr)
{
    const double2* b = reinterpret_cast<const double2*>(base);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double2 x = b[k * T + t];
        v[k] = mkc(x.x, x.y);
    }
    double2 x = b[C * T + t];
    gl = mkc(x.x, x.y);
    x = b[(C + 1) * T + t];
    gr = mkc(x.x, x.y);
}

template <int C>
__device__ __forceinline__ void observe_a(const cd (&v)[C], const SizeClass& sc, const LaneCtx& lc,
                                          double xs, double* slot)
{
    double sn = 0.0, sk = 0.0, sv = 0.0;
    const int t = opaque(lc.t);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double p = cabs2(v[k]);
        sn += p;
        sk = fma((double)k, p, sk);
        sv = fma(sc.pt.dv[k * sc.T + t], p, sv);
    }
    double sx = fma(xs, sn, sc.dx * sk);
    sn = wave_sum(sn);
    sx = wave_sum(sx);
    sv = wave_sum(sv);
    if (lc.lane == 0) {
        slot[lc.wave * 3 + 0] = sv;
        slot[lc.wave * 3 + 1] = sx;
        slot[lc.wave * 3 + 2] = sn;
    }
}

__device__ __forceinline__ void flush_fwd(int a0, int a1, const double* ring, int W, double dx,
                                          const double* erow, double* acc_row, double* n_row,
                                          int* flag)
{
    for (int smp = a0 + (int)threadIdx.x; smp <= a1; smp += blockDim.x) {
        const double* r = ring + (smp % kRing) * W * 3;
        double sv = 0.0, sn = 0.0;
        for (int w = 0; w < W; ++w) {
            sv += r[w * 3 + 0];
            sn += r[w * 3 + 2];
        }
        const double acc = dx * fma(erow[smp], sn, sv);
        if (acc_row) acc_row[smp] = acc;
        n_row[smp] = dx * sn;
        if (!isfinite(acc) || !isfinite(sn)) atomicOr(flag, 1);
    }
}

// grad_i = abar_i n_i + dt * sum_w partial_w(i) for i in [a0, a1]
__device__ __forceinline__ void flush_grad(int a0, int a1, const double* ring, int W, double dt,
                                           const double* abar, const double* n_row, double* g_row,
                                           int* flag)
{
    for (int smp = a0 + (int)threadIdx.x; smp <= a1; smp += blockDim.x) {
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
    if (lc.lane == 0) slot[lc.wave] = g;
}

}  // namespace

template <int C>
__global__ void __launch_bounds__(256) adjoint_kernel(FwdArgs a)
{
    extern __shared__ double smem_raw[];
    const int tid = threadIdx.x;
    const int W = blockDim.x / kWave;
    cd* lds_f = reinterpret_cast<cd*>(smem_raw);
    cd* lds_b = lds_f + kMaxWaves;
    double* ring = reinterpret_cast<double*>(lds_b + kMaxWaves) + 2 * kMaxWaves;
    int* misc = reinterpret_cast<int*>(ring + kRing * W * 3);

    const int nt = a.nt, K = a.k_ckpt;
    const int nseg = nt / K + 1;
    double* slot_base = a.ckpt + (size_t)blockIdx.x * (size_t)a.slot_stride_ckpt;

    for (;;) {
        if (tid == 0) {
            misc[0] = atomicAdd(a.queue, 1);
            misc[1] = 0;
            misc[2] = 0;
        }
        __syncthreads();
        const int item = uniform(misc[0]);
        if (item >= a.count) break;
        const int p = uniform(a.order[item]);
        const SysDesc d = uniform_load(a.sys + p);
        const SizeClass sc = uniform_load(a.classes + d.cls);
        const int T = sc.T;
        const size_t np2 = 2 * (size_t)(C + 2) * T;  // doubles per state record
        double* ckpt = slot_base;
        double* seg = ckpt + np2 * nseg;
        double* n_row = seg + np2 * (K + 1);
        const size_t row = (size_t)p * (size_t)(nt + 1);
        const double* erow = a.E + row;
        const double* abar = a.abar + row;
        double* g_row = a.grad + row;
        double* acc_row = a.accel ? a.accel + row : nullptr;

        // rows with an all-zero abar have a zero gradient
        for (int i = tid; i <= nt; i += blockDim.x)
            if (abar[i] != 0.0) misc[2] = 1;
        __syncthreads();
        if (misc[2] == 0 && acc_row == nullptr) {
            for (int i = tid; i <= nt; i += blockDim.x) g_row[i] = 0.0;
            if (tid == 0 && a.status) a.status[p] = 0;
            __syncthreads();
            continue;
        }
        const bool need_grad = misc[2] != 0;

        const LaneCtx lc = make_lane_ctx(sc, tid);
        const RhsCoef rc = make_rhs_coef(0.5 * a.dt, sc.dx);
        const double dx = sc.dx;
        const int n = sc.n, s = lc.s;
        const double xs = ((double)s - 0.5 * (double)(n - 1)) * dx;
        const double xl = ((double)(s - 1) - 0.5 * (double)(n - 1)) * dx;
        const double* src = a.psi0 ? a.psi0 + 2 * d.psi_off : a.gs + 2 * a.gs_off[d.cls];

        // ---------------- forward pass: outputs, norms, checkpoints
        cd v[C];
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = (s + k < n) ? ld_psi(src, s + k) : czero();
        cd gl = (s > 0 && s - 1 < n) ? ld_psi(src, s - 1) : czero();
        cd gr = (s + C < n) ? ld_psi(src, s + C) : czero();
        int flushed = 0;
        for (int i = 0; i <= nt; ++i) {
            if (i % K == 0) store_state<C>(ckpt + np2 * (i / K), T, tid, v, gl, gr);
            observe_a<C>(v, sc, lc, xs, ring + (i % kRing) * W * 3);
            if (i == nt) break;
            forward_step<C>(v, gl, gr, erow[i], a.dt, xl, sc, lc, rc, lds_f, lds_b);
            if ((i + 1) % kFlush == 0) {
                __syncthreads();
                flush_fwd(i + 1 - kFlush, i, ring, W, dx, erow, acc_row, n_row, misc + 1);
                flushed = i + 1;
            }
        }
        __syncthreads();
        flush_fwd(flushed, nt, ring, W, dx, erow, acc_row, n_row, misc + 1);
        __syncthreads();

        if (!need_grad) {
            for (int i = tid; i <= nt; i += blockDim.x) g_row[i] = 0.0;
        } else {
            // ---------------- backward pass
            if (tid == 0) g_row[nt] = abar[nt] * n_row[nt];
            cd kap[C], kgl = czero(), kgr = czero();
            bool started = false;
            for (int sidx = nseg - 1; sidx >= 0; --sidx) {
                const int s0 = sidx * K;
                const int s1 = min(s0 + K, nt);
                // recompute psi^{s0..s1} into the segment buffer
                load_state<C>(ckpt + np2 * sidx, T, tid, v, gl, gr);
                store_state<C>(seg, T, tid, v, gl, gr);
                for (int i = s0; i < s1; ++i) {
                    forward_step<C>(v, gl, gr, erow[i], a.dt, xl, sc, lc, rc, lds_f, lds_b);
                    store_state<C>(seg + np2 * (i - s0 + 1), T, tid, v, gl, gr);
                }
                if (!started) {
                    // kappa^nt = 2 abar_nt dx (V' + E_nt) conj(psi^nt); psi^nt = v
                    const double cn = 2.0 * abar[nt] * dx;
                    const double en = erow[nt];
#pragma unroll
                    for (int k = 0; k < C; ++k)
                        kap[k] = cscale(cn * (sc.pt.dv[k * T + tid] + en), cconj(v[k]));
                    kgl = cscale(cn * (lc.dvl + en), cconj(gl));
                    kgr = cscale(cn * (lc.dvr + en), cconj(gr));
                    if (nt > 0) grad_partial<C>(kap, v, xs, dx, lc, ring + ((nt - 1) % kRing) * W);
                    started = true;
                    if (nt > 0 && (nt - 1) % kFlush == 0) {
                        __syncthreads();
                        flush_grad(nt - 1, nt - 1, ring, W, a.dt, abar, n_row, g_row, misc + 1);
                    }
                }
                for (int i = s1 - 1; i >= s0; --i) {
                    // kappa <- U (D_i kappa)
                    const double e = erow[i];
                    phase_mask<C>(kap, kgl, kgr, e, a.dt, xl, dx, sc, lc);
                    cd cf, cb;
                    cn_apply<C, true>(kap, kgl, kgr, sc, lc, rc, lds_f, lds_b, cf, cb);
                    kgl = cmad(lc.ql, cf, cmul(lc.bl, kap[0]));
                    kgr = cb;
                    // + 2 abar_i dx (V' + E_i) conj(psi^i)
                    load_state<C>(seg + np2 * (i - s0), T, tid, v, gl, gr);
                    const double ci = 2.0 * abar[i] * dx;
                    const int to = opaque(tid);
#pragma unroll
                    for (int k = 0; k < C; ++k)
                        kap[k] = cadd(kap[k], cscale(ci * (sc.pt.dv[k * T + to] + e), cconj(v[k])));
                    kgl = cadd(kgl, cscale(ci * (lc.dvl + e), cconj(gl)));
                    kgr = cadd(kgr, cscale(ci * (lc.dvr + e), cconj(gr)));
                    if (i > 0) {
                        // partial of grad_{i-1} from kappa^i and psi^i
                        grad_partial<C>(kap, v, xs, dx, lc, ring + ((i - 1) % kRing) * W);
                        if ((i - 1) % kFlush == 0) {
                            __syncthreads();
                            flush_grad(i - 1, min(i - 1 + kFlush - 1, nt - 1), ring, W, a.dt, abar,
                                       n_row, g_row, misc + 1);
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0 && a.status) a.status[p] = misc[1];
    }
}

template <int C>
static int occ_adj(int T)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, adjoint_kernel<C>, T,
                                                     adj_smem_bytes(T / kWave)) != hipSuccess)
        return 0;
    return nb;
}

int adjoint_occupancy(int C, int T)
{
    switch (C) {
        case 4: return occ_adj<4>(T);
        case 8: return occ_adj<8>(T);
        case 16: return occ_adj<16>(T);
        default: return 0;
    }
}

hipError_t launch_adjoint(int C, const FwdArgs& a, int T, int grid, hipStream_t st)
{
    const size_t sh = adj_smem_bytes(T / kWave);
    switch (C) {
        case 4: hipLaunchKernelGGL(adjoint_kernel<4>, dim3(grid), dim3(T), sh, st, a); break;
        case 8: hipLaunchKernelGGL(adjoint_kernel<8>, dim3(grid), dim3(T), sh, st, a); break;
        case 16: hipLaunchKernelGGL(adjoint_kernel<16>, dim3(grid), dim3(T), sh, st, a); break;
        default: return hipErrorInvalidValue;
    }
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
