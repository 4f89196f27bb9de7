// tdse_spectrum.hip -- analysis of the microscopic response: electron energy
// distribution of a wavefunction, Gabor transform of the source term,
// ground-state and volumetric populations along a propagation.
//
// Section "Analysing the Time-Dependent Electron Energy Density": with the
// field-free Hamiltonian H0 = M2^{-1}(-D2/2) + V of the solver's Numerov
// scheme,
//   P(E) = (eps / pi) dx sum_j |phi_j|^2,   (E - i eps - H0) phi = psi,
// the normalisation 1/(pi eps) making int P dE = dx sum |psi|^2.  Multiplied
// by M2 the system is tridiagonal,
//   ((E - i eps) M2 - A) phi = b = M2 psi,   A = -D2/2 + M2 diag(V):
//   diagonal   (E - i eps) 10/12 - 1/dx^2 - 10/12 V_j
//   T[j, j-1]  (E - i eps) /12 + 1/(2 dx^2) - V_{j-1}/12   (and T[j, j+1] with V_{j+1}).
// Its imaginary part -eps M2 is negative definite, so elimination without
// pivoting meets no zero pivot.
//
// The matrix depends on the grid size and the energy only: its elimination
// factors are formed once per (size, energy) pair and shared by every
// system.  With pivots p_j, 1/p_j = inv_j, m_j = -T[j, j-1] inv_j and
// c'_j = T[j, j+1] inv_j,
//   forward   d'_j  = b_j inv_j + m_j d'_{j-1}
//   backward  phi_j = d'_j - c'_j phi_{j+1},
// the norm accumulated in the backward sweep.  The backward sweep needs d'
// in reverse order: the forward sweep keeps only every kSpecGroup-th value
// (16 / kSpecGroup bytes per point and solve, in the caller's workspace),
// and the backward sweep recomputes each group of kSpecGroup values from
// its start value into registers before walking it backwards.  A wavefront
// works on a tile of 8 systems x 8 energies (systems ordered by size), so a
// factor load serves 8 lanes and a right-hand-side load 8 lanes.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

constexpr int kSpecGroup = 8;       // d' values recomputed per group
constexpr int kSpecTile = 8;        // systems (and energies) per wavefront tile

// b = M2 psi of every system (ragged, natural point order).
__global__ void __launch_bounds__(256) spectrum_rhs_kernel(SpecArgs a)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    for (int b = blockIdx.y; b < a.batch; b += gridDim.y) {
        const SysDesc d = a.sys[b];
        if (j >= d.n) continue;
        const double* psi = a.psi + 2 * d.psi_off;
        const cd p0 = ld_psi(psi, j);
        const cd pm = j > 0 ? ld_psi(psi, j - 1) : czero();
        const cd pp = j + 1 < d.n ? ld_psi(psi, j + 1) : czero();
        a.rhs[d.psi_off + j] = mkc((pm.re + 10.0 * p0.re + pp.re) / 12.0,
                                   (pm.im + 10.0 * p0.im + pp.im) / 12.0);
    }
}

// Elimination factors of one (size class, energy) pair, one lane per pair:
// fac[(j * pairs + pair) * 3 + {0, 1, 2}] = inv_j, m_j, -c'_j.
__global__ void __launch_bounds__(256) spectrum_factor_kernel(SpecArgs a)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= a.pairs) return;
    const int c = pair / a.n_energy, e = pair - c * a.n_energy;
    const SizeClass& sc = a.classes[c];
    const int n = sc.n, C = sc.C;
    const double* v = sc.pt.v;
    const double k2 = 1.0 / (sc.dx * sc.dx);
    const double E = a.energies[e];
    const double off_re = E / 12.0 + 0.5 * k2, off_im = -a.eps / 12.0;
    const double dia_re = E * (10.0 / 12.0) - k2, dia_im = -a.eps * (10.0 / 12.0);
    const int64_t P = a.pairs;
    cd cp = czero();
    double vm = 0.0, v0 = v[pidx(0, 0, C)];
    for (int j = 0; j < n; ++j) {
        const bool last = j + 1 == n;
        const double vp = last ? 0.0 : v[pidx((j + 1) / C, (j + 1) % C, C)];
        const cd dia = mkc(dia_re - (10.0 / 12.0) * v0, dia_im);
        const cd low = j > 0 ? mkc(off_re - vm / 12.0, off_im) : czero();
        const cd up = last ? czero() : mkc(off_re - vp / 12.0, off_im);
        const cd inv = cinv(cadd(dia, cscale(-1.0, cmul(low, cp))));
        cp = cmul(up, inv);
        cd* f = a.fac + 3 * ((int64_t)j * P + pair);
        f[0] = inv;
        f[1] = cscale(-1.0, cmul(low, inv));
        f[2] = cscale(-1.0, cp);
        vm = v0;
        v0 = vp;
    }
}

// One wavefront per tile of 8 systems x 8 energies (lane = 8 s + e); the
// wavefronts stride over the tiles.  Each lane keeps its d' group starts in
// its own column of its wavefront's block of the workspace ([group][lane],
// coalesced).
__global__ void __launch_bounds__(64) energy_spectrum_kernel(SpecArgs a)
{
    const int lane = threadIdx.x;
    const int64_t wave = blockIdx.x;
    const int64_t nwaves = gridDim.x;
    const int ts_count = (a.batch + kSpecTile - 1) / kSpecTile;
    const int te_count = (a.n_energy + kSpecTile - 1) / kSpecTile;
    const int64_t tiles = (int64_t)ts_count * te_count;
    const int64_t P = a.pairs;
    // this wavefront's group starts: [group][lane], contiguous per wavefront
    // so that each wavefront walks its own pages of the workspace
    const int64_t ckstride = kWave;
    const int64_t slots = (a.n_max + kSpecGroup - 1) / kSpecGroup - 1;
    cd* ck = a.work + wave * (slots > 0 ? slots : 1) * kWave + lane;
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        // energy tiles of one system tile are consecutive: neighbouring
        // wavefronts read the same right-hand sides
        const int te = (int)(tile % te_count), ts = (int)(tile / te_count);
        const int s_raw = ts * kSpecTile + lane / kSpecTile;
        const int e_raw = te * kSpecTile + lane % kSpecTile;
        const bool valid = s_raw < a.batch && e_raw < a.n_energy;
        const int b = a.order[min(s_raw, a.batch - 1)];
        const int ei = min(e_raw, a.n_energy - 1);
        const SysDesc d = a.sys[b];
        const int n = d.n;
        const int64_t pair = (int64_t)d.cls * a.n_energy + ei;
        const cd* f = a.fac + 3 * pair;
        const int64_t fs = 3 * P;  // factor stride per point
        const cd* rb = a.rhs + d.psi_off;
        const int ng = (n + kSpecGroup - 1) / kSpecGroup;
        const int nfull = n / kSpecGroup;  // groups of kSpecGroup points (no tail)
        // forward sweep, keeping d'_{j0 - 1} of every group j0 > 0; full
        // groups run without conditions, so their loads issue ahead
        cd dp = czero();
        for (int g = 0; g < ng; ++g) {
            const int j0 = g * kSpecGroup;
            if (g > 0) ck[(int64_t)(g - 1) * ckstride] = dp;
            const cd* fg = f + (int64_t)j0 * fs;
            if (g < nfull) {
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u)
                    dp = cmad(ldg(fg + u * fs + 1), dp, cmul(ldg(rb + j0 + u), ldg(fg + u * fs)));
            } else {
                for (int u = 0; j0 + u < n; ++u)
                    dp = cmad(ldg(fg + u * fs + 1), dp, cmul(ldg(rb + j0 + u), ldg(fg + u * fs)));
            }
        }
        // backward sweep group by group: recompute the group's d' from its
        // start value, then walk it backwards accumulating |phi|^2
        double acc = 0.0;
        cd phi = czero();
        for (int g = ng - 1; g >= 0; --g) {
            const int j0 = g * kSpecGroup;
            const cd* fg = f + (int64_t)j0 * fs;
            cd x = g > 0 ? ck[(int64_t)(g - 1) * ckstride] : czero();
            if (g < nfull) {
                cd dd[kSpecGroup];
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u) {
                    x = cmad(ldg(fg + u * fs + 1), x, cmul(ldg(rb + j0 + u), ldg(fg + u * fs)));
                    dd[u] = x;
                }
#pragma unroll
                for (int u = kSpecGroup - 1; u >= 0; --u) {
                    phi = cmad(ldg(fg + u * fs + 2), phi, dd[u]);
                    acc = fma(phi.re, phi.re, fma(phi.im, phi.im, acc));
                }
            } else {
                cd dd[kSpecGroup];
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u) {
                    if (j0 + u < n)
                        x = cmad(ldg(fg + u * fs + 1), x, cmul(ldg(rb + j0 + u), ldg(fg + u * fs)));
                    dd[u] = x;
                }
#pragma unroll
                for (int u = kSpecGroup - 1; u >= 0; --u) {
                    if (j0 + u < n) {
                        phi = cmad(ldg(fg + u * fs + 2), phi, dd[u]);
                        acc = fma(phi.re, phi.re, fma(phi.im, phi.im, acc));
                    }
                }
            }
        }
        if (valid) a.out[(int64_t)b * a.n_energy + ei] = a.eps / M_PI * a.classes[d.cls].dx * acc;
    }
}

size_t spectrum_factor_bytes(int n_max, int64_t pairs)
{
    return ((size_t)n_max * (size_t)pairs * 3 * sizeof(cd) + 255) & ~size_t(255);
}

size_t spectrum_slot_bytes(int n_max)
{
    const int ng = (n_max + kSpecGroup - 1) / kSpecGroup;
    return sizeof(cd) * (size_t)std::max(ng - 1, 1);
}

// Gabor transform (section "Physical Examples & tutorials", microscopic
// analysis): G[b][c][w] = |dt sum_i a_b,i exp(-(t_i - t_c)^2 / (2 sigma^2))
// exp(-i omega_w t_i)|^2.  Samples farther than kGaborReach sigma from t_c
// are skipped (their window is below 3e-20).  One workgroup per (t_c, row):
// the windowed samples go through LDS in chunks, each thread accumulates up
// to kGaborPerThread frequencies with a phase rotation started exactly at
// every chunk.
constexpr int kGaborChunk = 1024;
constexpr int kGaborPerThread = 4;
constexpr double kGaborReach = 9.5;

__global__ void __launch_bounds__(256) gabor_kernel(GaborArgs a)
{
    __shared__ double buf[kGaborChunk];
    const int c = blockIdx.x, b = blockIdx.y;
    const double tc = a.t_centres[c];
    const int64_t M = (int64_t)a.nt + 1;
    const double reach = kGaborReach * a.sigma;
    const int64_t i_lo = max((int64_t)0, (int64_t)floor((tc - reach) / a.dt));
    const int64_t i_hi = min(M - 1, (int64_t)ceil((tc + reach) / a.dt));
    const double* row = a.accel + (size_t)b * M;
    const double inv2s2 = 1.0 / (2.0 * a.sigma * a.sigma);
    double sre[kGaborPerThread], sim[kGaborPerThread], om[kGaborPerThread];
#pragma unroll
    for (int u = 0; u < kGaborPerThread; ++u) {
        const int w = threadIdx.x + u * blockDim.x;
        om[u] = w < a.n_w ? a.omegas[w] : 0.0;
        sre[u] = sim[u] = 0.0;
    }
    for (int64_t i0 = i_lo; i0 <= i_hi; i0 += kGaborChunk) {
        const int len = (int)min((int64_t)kGaborChunk, i_hi - i0 + 1);
        __syncthreads();
        for (int k = threadIdx.x; k < len; k += blockDim.x) {
            const double t = a.dt * (double)(i0 + k) - tc;
            buf[k] = row[i0 + k] * exp(-t * t * inv2s2);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kGaborPerThread; ++u) {
            if (threadIdx.x + u * (int)blockDim.x >= a.n_w) continue;
            double sp, cp, sr, cr;
            sincos(-om[u] * a.dt * (double)i0, &sp, &cp);
            sincos(-om[u] * a.dt, &sr, &cr);
            cd ph = mkc(cp, sp);
            const cd rot = mkc(cr, sr);
            for (int k = 0; k < len; ++k) {
                sre[u] = fma(buf[k], ph.re, sre[u]);
                sim[u] = fma(buf[k], ph.im, sim[u]);
                ph = cmul(ph, rot);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kGaborPerThread; ++u) {
        const int w = threadIdx.x + u * blockDim.x;
        if (w < a.n_w) {
            const double re = a.dt * sre[u], im = a.dt * sim[u];
            a.out[((size_t)b * a.n_tc + c) * a.n_w + w] = re * re + im * im;
        }
    }
}

// Populations (section "Microscopic Response in XUV regime (TDSE)", the
// analyses of psi it lists; the interface's example plots both against
// time): for the state psi of a stored record and the reference phi,
//   gs  = |dx sum_j conj(phi_j) psi_j|^2,
//   vol = dx sum_{|x_j| <= radius} |psi_j|^2,   x_j = (j - (n-1)/2) dx.
// One workgroup per (record, system).  The record is read in its own
// [k][t] order (point j = t C + k), so the loads are coalesced; phi is a
// gather from the plan's ground state (shared by all systems of a size, so
// it stays in the L2) or the caller's reference.
__global__ void __launch_bounds__(256) populations_kernel(PopArgs a)
{
    __shared__ double red[3][4];
    const int s = blockIdx.x, b = blockIdx.y;
    const SysDesc d = a.sys[b];
    const SizeClass& sc = a.classes[d.cls];
    const int C = sc.C, T = sc.T, n = sc.n;
    const double dx = sc.dx, half = 0.5 * (double)(n - 1);
    const size_t np2 = 2 * (size_t)(C + 2) * T;
    const double* rec = a.store + a.store_off[b] + np2 * (size_t)s;
    const double* ref = a.psi_ref ? a.psi_ref + 2 * d.psi_off : a.gs + 2 * a.gs_off[d.cls];
    double ore = 0.0, oim = 0.0, vol = 0.0;
    for (int idx = threadIdx.x; idx < C * T; idx += 256) {
        const int k = idx / T, t = idx - k * T;
        const int j = t * C + k;
        if (j >= n) continue;
        const double pr = rec[2 * (size_t)idx], pi = rec[2 * (size_t)idx + 1];
        const double fr = ref[2 * (size_t)j], fi = ref[2 * (size_t)j + 1];
        ore = fma(fr, pr, fma(fi, pi, ore));   // Re(conj(phi) psi)
        oim = fma(fr, pi, fma(-fi, pr, oim));  // Im(conj(phi) psi)
        if (fabs(((double)j - half) * dx) <= a.radius) vol = fma(pr, pr, fma(pi, pi, vol));
    }
    ore = wave_sum(ore);
    oim = wave_sum(oim);
    vol = wave_sum(vol);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == kSumLane) {
        red[0][w] = ore;
        red[1][w] = oim;
        red[2][w] = vol;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = dx * (red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        const double i = dx * (red[1][0] + red[1][1] + red[1][2] + red[1][3]);
        const size_t o = (size_t)b * a.nrec + s;
        if (a.gs_out) a.gs_out[o] = fma(r, r, i * i);
        if (a.vol_out) a.vol_out[o] = dx * (red[2][0] + red[2][1] + red[2][2] + red[2][3]);
    }
}

hipError_t launch_populations(const PopArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(populations_kernel, dim3(a.nrec, a.batch), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gabor(const GaborArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(gabor_kernel, dim3(a.n_tc, a.batch), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_energy_spectrum(const SpecArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(spectrum_factor_kernel, dim3((a.pairs + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(spectrum_rhs_kernel, dim3((a.n_max + 255) / 256, std::min(a.batch, 65535)),
                       dim3(256), 0, st, a);
    hipLaunchKernelGGL(energy_spectrum_kernel, dim3((unsigned)(a.lanes / kWave)), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
