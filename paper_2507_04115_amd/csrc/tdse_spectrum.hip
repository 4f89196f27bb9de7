// tdse_spectrum.hip -- electron energy distribution of a wavefunction.
//
// Section "Analysing the Time-Dependent Electron Energy Density": with the
// field-free Hamiltonian H0 = M2^{-1}(-D2/2) + V of the solver's Numerov
// scheme,
//   P(E) = (eps / pi) dx sum_j |phi_j|^2,   (E - i eps - H0) phi = psi,
// the normalisation 1/(pi eps) making int P dE = dx sum |psi|^2.  Multiplied
// by M2 the system is tridiagonal,
//   ((E - i eps) M2 - A) phi = M2 psi,   A = -D2/2 + M2 diag(V):
//   diagonal   (E - i eps) 10/12 - 1/dx^2 - 10/12 V_j
//   T[j, j-1]  (E - i eps) /12 + 1/(2 dx^2) - V_{j-1}/12   (and T[j, j+1] with V_{j+1}).
// Its imaginary part -eps M2 is negative definite, so elimination without
// pivoting meets no zero pivot.  One lane per (system, energy): forward
// elimination storing (c'_j, d'_j) in the caller's workspace (interleaved by
// lane, so the stores are coalesced), then back substitution accumulating
// |phi_j|^2.  Lanes of a wavefront mostly share the system, so psi and V
// are broadcast loads.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

__global__ void __launch_bounds__(256) energy_spectrum_kernel(SpecArgs a)
{
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= a.lanes) return;
    const int64_t items = (int64_t)a.batch * a.n_energy;
    for (int64_t it = lane; it < items; it += a.lanes) {
        const int b = (int)(it / a.n_energy);
        const int e = (int)(it - (int64_t)b * a.n_energy);
        const SysDesc d = a.sys[b];
        const SizeClass& sc = a.classes[d.cls];
        const int n = sc.n, C = sc.C;
        const double dx = sc.dx;
        const double* v = sc.pt.v;
        const double* psi = a.psi + 2 * d.psi_off;
        const double E = a.energies[e], eps = a.eps;
        const double k2 = 1.0 / (dx * dx);
        const double off_re = E / 12.0 + 0.5 * k2, off_im = -eps / 12.0;
        const double dia_re = E * (10.0 / 12.0) - k2, dia_im = -eps * (10.0 / 12.0);
        cd* w = a.work;
        const int64_t L = a.lanes;

        // forward elimination
        cd cp = czero(), dp = czero();
        cd pm = czero(), p0 = ld_psi(psi, 0);
        double vm = 0.0, v0 = v[pidx(0, 0, C)];
        for (int j = 0; j < n; ++j) {
            const bool last = j + 1 == n;
            const cd pp = last ? czero() : ld_psi(psi, j + 1);
            const double vp = last ? 0.0 : v[pidx((j + 1) / C, (j + 1) % C, C)];
            const cd dia = mkc(dia_re - (10.0 / 12.0) * v0, dia_im);
            const cd low = j > 0 ? mkc(off_re - vm / 12.0, off_im) : czero();
            const cd up = last ? czero() : mkc(off_re - vp / 12.0, off_im);
            const cd rhs = mkc((pm.re + 10.0 * p0.re + pp.re) / 12.0, (pm.im + 10.0 * p0.im + pp.im) / 12.0);
            const cd inv = cinv(cadd(dia, cscale(-1.0, cmul(low, cp))));
            cp = cmul(up, inv);
            dp = cmul(cadd(rhs, cscale(-1.0, cmul(low, dp))), inv);
            w[2 * ((int64_t)j * L + lane)] = cp;
            w[2 * ((int64_t)j * L + lane) + 1] = dp;
            pm = p0;
            p0 = pp;
            vm = v0;
            v0 = vp;
        }
        // back substitution with |phi|^2 accumulated
        cd phi = dp;
        double acc = cabs2(phi);
        for (int j = n - 2; j >= 0; --j) {
            const cd c = w[2 * ((int64_t)j * L + lane)];
            const cd dd = w[2 * ((int64_t)j * L + lane) + 1];
            phi = cadd(dd, cscale(-1.0, cmul(c, phi)));
            acc += cabs2(phi);
        }
        a.out[it] = eps / M_PI * dx * acc;
    }
}

hipError_t launch_energy_spectrum(const SpecArgs& a, hipStream_t st)
{
    const unsigned blocks = (unsigned)((a.lanes + 255) / 256);
    hipLaunchKernelGGL(energy_spectrum_kernel, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
