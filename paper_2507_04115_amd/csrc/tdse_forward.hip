// tdse_forward.hip -- persistent batched forward propagation and the
// imaginary-time ground state on gfx950.
//
// Layout: one workgroup of T = 64 W lanes owns one system at a time; lane t
// keeps grid points [t C, t C + C) of psi in VGPRs for the whole time loop,
// plus one ghost value on each side.  Per step (section "1D-TSDE
// Implementation (CTDSE)", three substeps):
//   1. r = 12 R psi in place                      (first substep)
//   2. L y = r by a partitioned Thomas solve      (second substep):
//      lane-local recurrences with zero carry, carries across lanes by a
//      Kogge-Stone scan over the wavefront (DPP/LDS-free shuffles) and one
//      LDS exchange between wavefronts, then lane-local fix-ups
//   3. psi_j = m_j exp(-i dt E_i x_j) y_j         (third substep + absorber)
//   4. per-lane partial sums of |psi|^2, x|psi|^2, V'|psi|^2, wavefront sums,
//      a ring of per-wave partials in LDS flushed every 32 samples as
//      coalesced rows of accel/xexp/norm.
// Only E_i (8 B per system-step) is read from HBM inside the loop; only the
// three observables (24 B per system-step) are written.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

namespace {

struct Smem {
    cd* lds_f;
    cd* lds_b;
    double* red0;
    double* red1;
    double* ring;
    int* misc;
};

__device__ __forceinline__ Smem carve(double* base, int W)
{
    Smem s;
    s.lds_f = reinterpret_cast<cd*>(base);
    s.lds_b = s.lds_f + kMaxWaves;
    s.red0 = reinterpret_cast<double*>(s.lds_b + kMaxWaves);
    s.red1 = s.red0 + kMaxWaves;
    s.ring = s.red1 + kMaxWaves;
    s.misc = reinterpret_cast<int*>(s.ring + kRing * W * 3);
    return s;
}

__host__ __device__ inline size_t smem_bytes(int W)
{
    return sizeof(cd) * 2 * kMaxWaves + sizeof(double) * 2 * kMaxWaves +
           sizeof(double) * kRing * W * 3 + 4 * sizeof(int);
}

// Per-lane partial sums of the observables of the current state, reduced over
// the wavefront; lane 0 stores (sum V'|psi|^2, sum x|psi|^2, sum |psi|^2).
template <int C>
__device__ __forceinline__ void observe(const cd (&v)[C], const SizeClass& sc, const LaneCtx& lc,
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

// Sums the per-wave partials of samples [a0, a1] in wave order and writes
//   accel = dx (sum V'|psi|^2 + E sum |psi|^2), xexp = dx sum x|psi|^2,
//   norm = dx sum |psi|^2.
__device__ __forceinline__ void flush(int a0, int a1, const double* ring, int W, double dx,
                                      const double* erow, double* acc_row, double* x_row,
                                      double* n_row, double n0, int* flag)
{
    for (int smp = a0 + (int)threadIdx.x; smp <= a1; smp += blockDim.x) {
        const double* r = ring + (smp % kRing) * W * 3;
        double sv = 0.0, sx = 0.0, sn = 0.0;
        for (int w = 0; w < W; ++w) {
            sv += r[w * 3 + 0];
            sx += r[w * 3 + 1];
            sn += r[w * 3 + 2];
        }
        const double nn = dx * sn;
        const double acc = dx * fma(erow[smp], sn, sv);
        acc_row[smp] = acc;
        if (x_row) x_row[smp] = dx * sx;
        if (n_row) n_row[smp] = nn;
        int f = 0;
        if (!isfinite(acc) || !isfinite(nn) || !isfinite(sx)) f |= 1;
        if (nn > n0 * (1.0 + 1e-8)) f |= 2;
        if (f) atomicOr(flag, f);
    }
}

}  // namespace

// -------------------------------------------------------------- forward
template <int C>
__global__ void __launch_bounds__(256) forward_kernel(FwdArgs a)
{
    extern __shared__ double smem_raw[];
    const int tid = threadIdx.x;
    const int W = blockDim.x / kWave;
    const Smem sm = carve(smem_raw, W);

    for (;;) {
        if (tid == 0) {
            sm.misc[0] = atomicAdd(a.queue, 1);
            sm.misc[1] = 0;
        }
        __syncthreads();
        const int item = uniform(sm.misc[0]);
        if (item >= a.count) break;
        const int p = uniform(a.order[item]);
        const SysDesc d = uniform_load(a.sys + p);
        const SizeClass sc = uniform_load(a.classes + d.cls);
        const LaneCtx lc = make_lane_ctx(sc, tid);
        const RhsCoef rc = make_rhs_coef(0.5 * a.dt, sc.dx);
        const double dx = sc.dx;
        const int n = sc.n, s = lc.s, T = sc.T;
        const double xs = ((double)s - 0.5 * (double)(n - 1)) * dx;
        const double xl = ((double)(s - 1) - 0.5 * (double)(n - 1)) * dx;
        const double* src = a.psi0 ? a.psi0 + 2 * d.psi_off : a.gs + 2 * a.gs_off[d.cls];
        const size_t row = (size_t)p * (size_t)(a.nt + 1);
        const double* erow = a.E + row;
        double* acc_row = a.accel + row;
        double* x_row = a.xexp ? a.xexp + row : nullptr;
        double* n_row = a.norm ? a.norm + row : nullptr;

        cd v[C];
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = (s + k < n) ? ld_psi(src, s + k) : czero();
        cd gl = (s > 0 && s - 1 < n) ? ld_psi(src, s - 1) : czero();
        cd gr = (s + C < n) ? ld_psi(src, s + C) : czero();

        observe<C>(v, sc, lc, xs, sm.ring);
        __syncthreads();
        double n0 = 0.0;
        for (int w = 0; w < W; ++w) n0 += sm.ring[w * 3 + 2];
        n0 *= dx;

        int flushed = 0;
        for (int i = 0; i < a.nt; ++i) {
            forward_step<C>(v, gl, gr, erow[i], a.dt, xl, sc, lc, rc, sm.lds_f, sm.lds_b);
            if ((i + 1) % kFlush == 0) {
                __syncthreads();
                flush(i + 1 - kFlush, i, sm.ring, W, dx, erow, acc_row, x_row, n_row, n0,
                      sm.misc + 1);
                flushed = i + 1;
            }
            observe<C>(v, sc, lc, xs, sm.ring + ((i + 1) % kRing) * W * 3);
        }
        __syncthreads();
        flush(flushed, a.nt, sm.ring, W, dx, erow, acc_row, x_row, n_row, n0, sm.misc + 1);
        if (a.psi_final) {
            double* dst = a.psi_final + 2 * d.psi_off;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                if (s + k < n) {
                    dst[2 * (s + k)] = v[k].re;
                    dst[2 * (s + k) + 1] = v[k].im;
                }
            }
        }
        __syncthreads();
        if (tid == 0 && a.status) a.status[p] = sm.misc[1];
    }
}

// -------------------------------------------------------------- ground state
// Imaginary-time relaxation: psi <- L_tau^{-1} R_tau psi with dt -> -i dtau,
// renormalised to dx sum |psi|^2 = 1 each iteration, until successive
// iterates differ by less than tol.  The energy follows from the growth
// factor g = ||L_tau^{-1} R_tau psi|| of the converged eigenvector:
// g = (1 - dtau E/2)/(1 + dtau E/2).  One workgroup per candidate.
template <int C>
__global__ void __launch_bounds__(256) gs_kernel(GsArgs a)
{
    extern __shared__ double smem_raw[];
    const int cand = blockIdx.x;
    const SizeClass sc = uniform_load(a.classes + uniform(a.cls_of[cand]));
    const int tid = threadIdx.x;
    const int W = sc.T / kWave;
    const Smem sm = carve(smem_raw, W);
    const LaneCtx lc = make_lane_ctx(sc, tid);
    const RhsCoef rc = make_rhs_coef(0.5 * a.dtau, sc.dx);
    const double dx = sc.dx;
    const int n = sc.n, s = lc.s;
    double* out = a.psi_out + 2 * a.psi_off[cand];

    cd v[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double x = ((double)(s + k) - 0.5 * (double)(n - 1)) * dx;
        v[k] = (s + k < n) ? mkc(exp(-x * x), 0.0) : czero();
    }
    const double xl = ((double)(s - 1) - 0.5 * (double)(n - 1)) * dx;
    const double xr = ((double)(s + C) - 0.5 * (double)(n - 1)) * dx;
    cd gl = (s > 0 && s - 1 < n) ? mkc(exp(-xl * xl), 0.0) : czero();
    cd gr = (s + C < n) ? mkc(exp(-xr * xr), 0.0) : czero();

    double loc = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) loc += cabs2(v[k]);
    double tot = block_sum(loc, sm.red0, lc.lane, lc.wave, W);
    double scl = 1.0 / sqrt(dx * tot);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        v[k] = cscale(scl, v[k]);
        if (s + k < n) {
            out[2 * (s + k)] = v[k].re;
            out[2 * (s + k) + 1] = v[k].im;
        }
    }
    gl = cscale(scl, gl);
    gr = cscale(scl, gr);

    int it = 0;
    bool conv = false;
    double g = 1.0;
    while (it < a.max_iter) {
        cd cf, cb;
        cn_apply<C, false>(v, gl, gr, sc, lc, rc, sm.lds_f, sm.lds_b, cf, cb);
        gl = cmad(lc.ql, cf, cmul(lc.bl, v[0]));
        gr = cb;
        loc = 0.0;
#pragma unroll
        for (int k = 0; k < C; ++k) loc += cabs2(v[k]);
        tot = block_sum(loc, sm.red1, lc.lane, lc.wave, W);
        g = sqrt(dx * tot);
        scl = 1.0 / g;
        gl = cscale(scl, gl);
        gr = cscale(scl, gr);
        loc = 0.0;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[k] = cscale(scl, v[k]);
            if (s + k < n) {
                const cd old = ld_psi(out, s + k);
                loc += cabs2(mkc(v[k].re - old.re, v[k].im - old.im));
                out[2 * (s + k)] = v[k].re;
                out[2 * (s + k) + 1] = v[k].im;
            }
        }
        tot = block_sum(loc, sm.red0, lc.lane, lc.wave, W);
        ++it;
        if (sqrt(dx * tot) < a.tol) {
            conv = true;
            break;
        }
    }
    if (tid == 0) {
        a.energy[cand] = (2.0 / a.dtau) * (1.0 - g) / (1.0 + g);
        a.iters[cand] = conv ? it : -it;
    }
}

__global__ void reset_counters_kernel(int32_t* c, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

hipError_t launch_reset_counters(int32_t* counters, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_counters_kernel, dim3((n + 63) / 64), dim3(64), 0, st, counters, n);
    return hipGetLastError();
}

bool layout_supported(int C) { return C == 4 || C == 8 || C == 16; }

template <int C>
static int occ_fwd(int T)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, forward_kernel<C>, T,
                                                     smem_bytes(T / kWave)) != hipSuccess)
        return 0;
    return nb;
}

int forward_occupancy(int C, int T)
{
    switch (C) {
        case 4: return occ_fwd<4>(T);
        case 8: return occ_fwd<8>(T);
        case 16: return occ_fwd<16>(T);
        default: return 0;
    }
}

hipError_t launch_forward(int C, const FwdArgs& a, int T, int grid, hipStream_t st)
{
    const size_t sh = smem_bytes(T / kWave);
    switch (C) {
        case 4: hipLaunchKernelGGL(forward_kernel<4>, dim3(grid), dim3(T), sh, st, a); break;
        case 8: hipLaunchKernelGGL(forward_kernel<8>, dim3(grid), dim3(T), sh, st, a); break;
        case 16: hipLaunchKernelGGL(forward_kernel<16>, dim3(grid), dim3(T), sh, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ground_state(int C, const GsArgs& a, int T, hipStream_t st)
{
    const size_t sh = smem_bytes(T / kWave);
    switch (C) {
        case 4: hipLaunchKernelGGL(gs_kernel<4>, dim3(a.ncand), dim3(T), sh, st, a); break;
        case 8: hipLaunchKernelGGL(gs_kernel<8>, dim3(a.ncand), dim3(T), sh, st, a); break;
        case 16: hipLaunchKernelGGL(gs_kernel<16>, dim3(a.ncand), dim3(T), sh, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tdse
