// tdse_farfield.hip -- far field of the XUV emission of the medium, and the
// adjoint of the band spectrum, so that a loss on the far field can be
// carried back to the field samples of every system.
//
// Far field (section "XUV Propagation (Spectral Approach)", Eq. of the far
// field in a homogeneous generating medium, mu0 left to the caller): with
// p = (i, j) running over the n_rho x n_z source points (rho'_i, z'_j),
// d_j = z - z'_j and k = k(omega_q),
//   E(rho_m, omega_q) = -(exp(i k z)/(4 pi)) sum_p w_p / d_j
//        exp(i (k (rho'_i^2 + rho_m^2) / (2 d_j) - k z'_j)) J0(k rho_m rho'_i / d_j) S_p(omega_q).
// w_p are the quadrature weights of rho' drho' dz' times the gas density.
// The map S -> E is linear; its adjoint gives dl/dS from dl/dE.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

namespace {

constexpr int kFarThreads = 256;
constexpr int kObsTile = 8;  // observation points per workgroup

// Propagator of source p at observation rho for wave number k, without the
// -(exp(i k z)/(4 pi)) prefactor.
__device__ __forceinline__ cd far_kernel(double k, double rho, double R, double Z, double w,
                                         double z_obs)
{
    const double d = z_obs - Z;
    const double ph = k * (R * R + rho * rho) / (2.0 * d) - k * Z;
    double s, c;
    sincos(ph, &s, &c);
    const double f = w / d * j0(k * rho * R / d);
    return mkc(f * c, f * s);
}

__device__ __forceinline__ cd far_prefactor(double k, double z_obs)
{
    double s, c;
    sincos(k * z_obs, &s, &c);
    const double f = -1.0 / (4.0 * M_PI);
    return mkc(f * c, f * s);
}

}  // namespace

// One workgroup per (tile of kObsTile observation points, frequency); the
// threads stride over the sources, each source spectrum value is loaded once
// and used for the whole tile; a tree reduction in LDS per observation point.
__global__ void __launch_bounds__(kFarThreads) far_field_kernel(FarArgs a)
{
    __shared__ double red[2 * kObsTile][kFarThreads];
    const int m0 = blockIdx.x * kObsTile, q = blockIdx.y;
    const int nm = min(kObsTile, a.n_obs - m0);
    const int P = a.n_rho * a.n_z;
    const double k = a.kwave[q];
    double rho[kObsTile];
#pragma unroll
    for (int t = 0; t < kObsTile; ++t) rho[t] = t < nm ? a.rho_obs[m0 + t] : 0.0;
    double sre[kObsTile], sim[kObsTile];
#pragma unroll
    for (int t = 0; t < kObsTile; ++t) sre[t] = sim[t] = 0.0;
    for (int p = threadIdx.x; p < P; p += kFarThreads) {
        const int i = p / a.n_z, j = p - i * a.n_z;
        const double R = a.rho_src[i], Z = a.z_src[j], w = a.weights[p];
        const cd src = mkc(a.in[2 * ((size_t)p * a.nk + q)], a.in[2 * ((size_t)p * a.nk + q) + 1]);
#pragma unroll
        for (int t = 0; t < kObsTile; ++t) {
            if (t < nm) {
                const cd kk = far_kernel(k, rho[t], R, Z, w, a.z_obs);
                sre[t] = fma(kk.re, src.re, fma(-kk.im, src.im, sre[t]));
                sim[t] = fma(kk.re, src.im, fma(kk.im, src.re, sim[t]));
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kObsTile; ++t) {
        red[2 * t][threadIdx.x] = sre[t];
        red[2 * t + 1][threadIdx.x] = sim[t];
    }
    __syncthreads();
    for (int o = kFarThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int t = 0; t < 2 * kObsTile; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + o];
        __syncthreads();
    }
    if ((int)threadIdx.x < nm) {
        const int t = threadIdx.x;
        const cd e = cmul(far_prefactor(k, a.z_obs), mkc(red[2 * t][0], red[2 * t + 1][0]));
        a.out[2 * ((size_t)(m0 + t) * a.nk + q)] = e.re;
        a.out[2 * ((size_t)(m0 + t) * a.nk + q) + 1] = e.im;
    }
}

// Adjoint: one thread per (source, frequency); S_bar[p][q] =
// sum_m conj(pre_q K_mpq) E_bar[m][q].
__global__ void __launch_bounds__(kFarThreads) far_field_adjoint_kernel(FarArgs a)
{
    const int P = a.n_rho * a.n_z;
    const int p = blockIdx.x * kFarThreads + threadIdx.x, q = blockIdx.y;
    if (p >= P) return;
    const int i = p / a.n_z, j = p - i * a.n_z;
    const double k = a.kwave[q];
    const double R = a.rho_src[i], Z = a.z_src[j], w = a.weights[p];
    double sre = 0.0, sim = 0.0;
    for (int m = 0; m < a.n_obs; ++m) {
        const cd kk = far_kernel(k, a.rho_obs[m], R, Z, w, a.z_obs);
        const cd eb = mkc(a.in[2 * ((size_t)m * a.nk + q)], a.in[2 * ((size_t)m * a.nk + q) + 1]);
        // conj(kk) * eb
        sre = fma(kk.re, eb.re, fma(kk.im, eb.im, sre));
        sim = fma(kk.re, eb.im, fma(-kk.im, eb.re, sim));
    }
    const cd r = cmul(cconj(far_prefactor(k, a.z_obs)), mkc(sre, sim));
    a.out[2 * ((size_t)p * a.nk + q)] = r.re;
    a.out[2 * ((size_t)p * a.nk + q) + 1] = r.im;
}

// Band adjoint: accel_bar[b][i] = dt w_i sum_k Re(conj(G_bk) exp(-i omega_k t_i)),
// w_i = sin^2(pi i / nt), omega_k t_i = 2 pi k i / (nt+1); one thread per
// sample, the phase advanced over k by rotation from an exact start.
__global__ void __launch_bounds__(256) band_adjoint_kernel(BandAdjArgs a)
{
    const int b = blockIdx.y;
    const int64_t M = (int64_t)a.nt + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double* g = a.amp_bar + 2 * (size_t)b * a.nk;
    double s = 0.0;
    if (a.nk > 0) {
        double sp, cp, sr, cr;
        sincos(-2.0 * M_PI * (double)(((int64_t)a.k_lo * i) % M) / (double)M, &sp, &cp);
        sincos(-2.0 * M_PI * (double)i / (double)M, &sr, &cr);
        cd ph = mkc(cp, sp);
        const cd rot = mkc(cr, sr);
        for (int kk = 0; kk < a.nk; ++kk) {
            s = fma(g[2 * kk], ph.re, fma(g[2 * kk + 1], ph.im, s));  // Re(conj(G) ph)
            ph = cmul(ph, rot);
        }
    }
    const double sw = sin(M_PI * (double)i / (double)a.nt);
    a.accel_bar[(size_t)b * M + i] = a.dt * sw * sw * s;
}

hipError_t launch_far_field(const FarArgs& a, bool adjoint, hipStream_t st)
{
    if (a.n_obs < 1 || a.nk < 1 || a.n_rho < 1 || a.n_z < 1) return hipErrorInvalidValue;
    if (!adjoint) {
        hipLaunchKernelGGL(far_field_kernel, dim3((a.n_obs + kObsTile - 1) / kObsTile, a.nk),
                           dim3(kFarThreads), 0, st, a);
    } else {
        const int P = a.n_rho * a.n_z;
        hipLaunchKernelGGL(far_field_adjoint_kernel, dim3((P + kFarThreads - 1) / kFarThreads, a.nk),
                           dim3(kFarThreads), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_band_adjoint(const BandAdjArgs& a, hipStream_t st)
{
    const int64_t M = (int64_t)a.nt + 1;
    hipLaunchKernelGGL(band_adjoint_kernel, dim3((unsigned)((M + 255) / 256), a.batch), dim3(256),
                       0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
