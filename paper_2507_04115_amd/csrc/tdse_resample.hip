// tdse_resample.hip -- the input interface of the microscopic solver on
// gfx950: driving fields given at M coarse samples are brought to the
// solver's time step by zero-padding their spectrum (section "1D-TSDE
// Implementation (CTDSE)": the time axis is shifted to start at 0 and the
// field is interpolated to dt in the Fourier domain).
//
// With X_k = sum_j e_j exp(-2 pi i j k / M) the DFT of a row's coarse
// samples (first sample at t = 0, spacing dt_c, period T = M dt_c) and
// M' = T / dt the padded length, the zero-padded inverse transform is the
// trigonometric interpolant
//   E(i dt) = (1/M) [ X_0 + 2 sum_{0<k<M/2} Re(X_k z_k(i))
//                     + (M even) Re(X_{M/2}) Re(z_{M/2}(i)) ],
//   z_k(i) = exp(2 pi i k i / M'),
// the Nyquist bin of an even M split evenly between +M/2 and -M/2.  Both
// sums are evaluated directly (O(M^2/2) per row for the spectrum,
// O(M (nt+1)/2) for the fine samples): the rotations exp(2 pi i q/M) are
// advanced by complex multiplication and restarted exactly from the integer
// phase (q mod M) every kRestart terms, so the rounding of the recurrence
// stays near 1e-15.  Runs once per input field, outside the propagation.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

constexpr int kRestart = 64;       // exact restart interval of the rotations
constexpr int kRowsPerBlock = 8;   // rows per workgroup of the synthesis

// exp(sign 2 pi i q / period) for an integer phase 0 <= q < period.
__device__ __forceinline__ cd unit_root(int64_t q, int64_t period, double sign)
{
    double s, c;
    sincos_rr(sign * 6.283185307179586476925286766559 * ((double)q / (double)period), &s, &c);
    return mkc(c, s);
}

// X[b][k] = sum_j e[b][j] exp(-2 pi i j k / M), k = 0 .. M/2.  One thread
// per (row, k); the 64 lanes of a wavefront share the row, so e[b][j] is a
// uniform (scalar) load.
__global__ void __launch_bounds__(256) coarse_dft_kernel(ResampleArgs a)
{
    const int b = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nk = a.m / 2 + 1;
    const double* row = a.coarse + (size_t)b * a.m;
    const int64_t M = a.m;
    cd acc = czero();
    const cd w = unit_root(k < nk ? k : 0, M, -1.0);
    cd z = mkc(1.0, 0.0);
    for (int j0 = 0; j0 < a.m; j0 += kRestart) {
        z = unit_root(((int64_t)j0 * (k < nk ? k : 0)) % M, M, -1.0);
        const int j1 = min(a.m, j0 + kRestart);
        for (int j = j0; j < j1; ++j) {
            const double e = ldg(row + j);
            acc = mkc(fma(e, z.re, acc.re), fma(e, z.im, acc.im));
            z = cmul(z, w);
        }
    }
    if (k < nk) reinterpret_cast<cd*>(a.spec)[(size_t)b * nk + k] = acc;
}

// Fine samples of kRowsPerBlock rows: one thread per fine sample i, the
// rotation z_k(i) advanced along k (factor exp(2 pi i i / M')) and shared
// by the block's rows; X of those rows is uniform across the workgroup.
__global__ void __launch_bounds__(256) synth_kernel(ResampleArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b0 = blockIdx.y * kRowsPerBlock;
    const int nk = a.m / 2 + 1;
    const bool even = (a.m % 2) == 0;
    const int kmax = even ? a.m / 2 : (a.m - 1) / 2;  // last bin of the sum
    const int64_t Mp = a.mp;
    const int ii = i <= a.nt ? i : 0;
    const cd w = unit_root(ii % Mp, Mp, 1.0);
    const cd* X = reinterpret_cast<const cd*>(a.spec);
    double acc[kRowsPerBlock];
#pragma unroll
    for (int r = 0; r < kRowsPerBlock; ++r) {
        const int b = min(b0 + r, a.batch - 1);
        acc[r] = ldg(&X[(size_t)b * nk].re);  // X_0 (real)
    }
    for (int k0 = 1; k0 <= kmax; k0 += kRestart) {
        cd z = unit_root(((int64_t)k0 * ii) % Mp, Mp, 1.0);
        const int k1 = min(kmax + 1, k0 + kRestart);
        for (int k = k0; k < k1; ++k) {
            // weight 2 for the bins with a mirror image, 1 for the split
            // Nyquist bin of an even M (whose X is real)
            const bool nyq = even && k == a.m / 2;
#pragma unroll
            for (int r = 0; r < kRowsPerBlock; ++r) {
                const int b = min(b0 + r, a.batch - 1);
                const cd x = ldg(&X[(size_t)b * nk + k]);
                const double t = nyq ? x.re * z.re : fma(x.re, z.re, -x.im * z.im);
                acc[r] = fma(nyq ? 1.0 : 2.0, t, acc[r]);
            }
            z = cmul(z, w);
        }
    }
    if (i > a.nt) return;
    const double inv_m = 1.0 / (double)a.m;
#pragma unroll
    for (int r = 0; r < kRowsPerBlock; ++r) {
        const int b = b0 + r;
        if (b < a.batch) a.fine[(size_t)b * (a.nt + 1) + i] = acc[r] * inv_m;
    }
}

hipError_t launch_resample(const ResampleArgs& a, hipStream_t st)
{
    const int nk = a.m / 2 + 1;
    hipLaunchKernelGGL(coarse_dft_kernel, dim3((nk + 255) / 256, a.batch), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(synth_kernel, dim3((a.nt + 1 + 255) / 256, (a.batch + kRowsPerBlock - 1) / kRowsPerBlock),
                       dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
