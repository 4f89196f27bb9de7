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
// its start value into registers before walking it backwards.
//
// A wavefront solves one energy for a block of 64 systems of one size, one
// lane each: the factors are then the same for the whole wavefront and come
// in through scalar loads, and the right-hand sides b = M2 psi, stored point
// by point for the systems of a size ([j][system], one row of 16 bytes per
// system), arrive in one coalesced load per point.  So the vector memory
// path carries only the 16 bytes per point and solve that differ between
// lanes, twice (forward sweep, recomputation), plus the group starts.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

constexpr int kSpecGroup = 16;      // d' values recomputed per group

// Entry of `spec` that holds 64-system block `blk` (entries ordered by blk0).
__device__ __forceinline__ int spec_entry(const SpecClass* spec, int nspec, int blk)
{
    int lo = 0, hi = nspec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (scalar_load(&spec[mid].blk0) <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// b = M2 psi of every system, point-interleaved within its size:
// rhs[rhs_off + j * count + k] for the size's k-th system.  Lanes are
// systems of one block, so the stores are coalesced.
__global__ void __launch_bounds__(256) spectrum_rhs_kernel(SpecArgs a)
{
    const int j = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    for (int blk = blockIdx.y; blk < a.nblocks; blk += gridDim.y) {
        const SpecClass s = scalar_load(a.spec + spec_entry(a.spec, a.nspec, blk));
        const int k = (blk - s.blk0) * kWave + threadIdx.x % kWave;
        if (k >= s.count || j >= s.n) continue;
        const SysDesc d = a.sys[a.order[s.start + k]];
        const double* psi = a.psi + 2 * d.psi_off;
        const cd p0 = ld_psi(psi, j);
        const cd pm = j > 0 ? ld_psi(psi, j - 1) : czero();
        const cd pp = j + 1 < s.n ? ld_psi(psi, j + 1) : czero();
        a.rhs[s.rhs_off + (int64_t)j * s.count + k] =
            mkc((pm.re + 10.0 * p0.re + pp.re) / 12.0, (pm.im + 10.0 * p0.im + pp.im) / 12.0);
    }
}

// Elimination factors of one (size class, energy) pair per wavefront:
// fac[(pair * n_max + j) * 3 + {0, 1, 2}] = inv_j, m_j, -c'_j, contiguous
// along j for the scalar stream of the solve.
//
// The elimination is a serial chain, c'_j = up_j / (dia_j - low_j c'_{j-1})
// from c'_{-1} = 0: a Moebius map of c'_{j-1} with the matrix
// M_j = [[0, up_j], [-low_j, dia_j]] acting on (c', 1).  Lane l takes the
// points of one chunk of ceil(n / 64), composes its maps into one matrix
// (rescaled by powers of two, which changes neither the map nor any
// rounding), a scan over the lanes composes the chunks before each one, and
// the lane then runs the elimination itself over its chunk from the start
// value c'_{j0-1} that the composition gives.  The chain that was 4096 steps
// long per pair becomes 2 x 64 steps and a 6-level scan.  The potential is
// staged in LDS in natural point order (n doubles).
struct Moeb {
    cd a, b, c, d;  // [[a, b], [c, d]]
};
__device__ __forceinline__ cd cadd2(cd x, cd y) { return mkc(x.re + y.re, x.im + y.im); }
// x * y: the map y first, then x
__device__ __forceinline__ Moeb moeb_mul(const Moeb& x, const Moeb& y)
{
    Moeb r;
    r.a = cadd2(cmul(x.a, y.a), cmul(x.b, y.c));
    r.b = cadd2(cmul(x.a, y.b), cmul(x.b, y.d));
    r.c = cadd2(cmul(x.c, y.a), cmul(x.d, y.c));
    r.d = cadd2(cmul(x.c, y.b), cmul(x.d, y.d));
    return r;
}
__device__ __forceinline__ double cmaxabs(cd z) { return fmax(fabs(z.re), fabs(z.im)); }
__device__ __forceinline__ cd cldexp(cd z, int e) { return mkc(ldexp(z.re, e), ldexp(z.im, e)); }
// Scales the matrix by a power of two that brings its largest component near 1.
__device__ __forceinline__ void moeb_rescale(Moeb& m)
{
    const double big = fmax(fmax(cmaxabs(m.a), cmaxabs(m.b)), fmax(cmaxabs(m.c), cmaxabs(m.d)));
    if (!(big > 0.0) || !isfinite(big)) return;
    int ex;
    (void)frexp(big, &ex);
    m.a = cldexp(m.a, -ex);
    m.b = cldexp(m.b, -ex);
    m.c = cldexp(m.c, -ex);
    m.d = cldexp(m.d, -ex);
}
__device__ __forceinline__ cd shfl_up_cd(cd z, int d)
{
    return mkc(__shfl_up(z.re, d, kWave), __shfl_up(z.im, d, kWave));
}
__device__ __forceinline__ Moeb shfl_up_moeb(const Moeb& m, int d)
{
    Moeb r;
    r.a = shfl_up_cd(m.a, d);
    r.b = shfl_up_cd(m.b, d);
    r.c = shfl_up_cd(m.c, d);
    r.d = shfl_up_cd(m.d, d);
    return r;
}
constexpr int kFacRescale = 8;  // chunk-product steps between rescalings

__global__ void __launch_bounds__(kWave) spectrum_factor_kernel(SpecArgs a)
{
    extern __shared__ double vs[];  // V_j, natural order
    const int pair = blockIdx.x;
    const int lane = threadIdx.x;
    const int c = pair / a.n_energy, e = pair - c * a.n_energy;
    const SizeClass& sc = a.classes[c];
    const int n = sc.n, C = sc.C;
    for (int j = lane; j < n; j += kWave) vs[j] = ldg(sc.pt.v + pidx(j / C, j % C, C));
    __syncthreads();
    const double k2 = 1.0 / (sc.dx * sc.dx);
    const double E = a.energies[e];
    const double off_re = E / 12.0 + 0.5 * k2, off_im = -a.eps / 12.0;
    const double dia_re = E * (10.0 / 12.0) - k2, dia_im = -a.eps * (10.0 / 12.0);
    // the row of the Numerov matrix at point j
    auto row = [&](int j, cd& low, cd& dia, cd& up) {
        dia = mkc(dia_re - (10.0 / 12.0) * vs[j], dia_im);
        low = j > 0 ? mkc(off_re - vs[j - 1] / 12.0, off_im) : czero();
        up = j + 1 < n ? mkc(off_re - vs[j + 1] / 12.0, off_im) : czero();
    };
    const int L = (n + kWave - 1) / kWave;
    const int j0 = min(n, lane * L), j1 = min(n, j0 + L);
    // this chunk's map
    Moeb P{mkc(1.0, 0.0), czero(), czero(), mkc(1.0, 0.0)};
    for (int j = j0; j < j1; ++j) {
        cd low, dia, up;
        row(j, low, dia, up);
        Moeb Q;
        Q.a = cmul(up, P.c);
        Q.b = cmul(up, P.d);
        Q.c = cadd2(cmul(dia, P.c), cscale(-1.0, cmul(low, P.a)));
        Q.d = cadd2(cmul(dia, P.d), cscale(-1.0, cmul(low, P.b)));
        P = Q;
        if ((j - j0) % kFacRescale == kFacRescale - 1) moeb_rescale(P);
    }
    moeb_rescale(P);
    // inclusive scan over the lanes: the maps of chunks 0 .. lane, composed
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Moeb prev = shfl_up_moeb(P, d);
        if (lane >= d) {
            P = moeb_mul(P, prev);
            moeb_rescale(P);
        }
    }
    // c'_{j0-1}: the composed maps of the chunks before this one applied to 0
    const cd num = shfl_up_cd(P.b, 1), den = shfl_up_cd(P.d, 1);
    cd cp = lane > 0 ? cmul(num, cinv(den)) : czero();
    cd* f = a.fac + 3 * ((int64_t)pair * a.n_max + j0);
    for (int j = j0; j < j1; ++j, f += 3) {
        cd low, dia, up;
        row(j, low, dia, up);
        const cd inv = cinv(cadd(dia, cscale(-1.0, cmul(low, cp))));
        cp = cmul(up, inv);
        f[0] = inv;
        f[1] = cscale(-1.0, cmul(low, inv));
        f[2] = cscale(-1.0, cp);
    }
}

// d'_j of one lane from d'_{j-1}: factors from the scalar stream, b_j from
// the lane's column.
__device__ __forceinline__ cd spec_step(const cd* f, const cd* b, cd dp)
{
    return cmad(scalar_load(f + 1), dp, cmul(ldg(b), scalar_load(f)));
}

// One wavefront per tile (energy e, block of 64 systems of one size); the
// wavefronts stride over the tiles, energy-major, so that the blocks of one
// energy run side by side.  Each lane keeps its d' group starts in its own
// column of its wavefront's block of the workspace ([group][lane],
// coalesced).
__global__ void __launch_bounds__(64) energy_spectrum_kernel(SpecArgs a)
{
    const int lane = threadIdx.x;
    const int64_t wave = blockIdx.x;
    const int64_t nwaves = gridDim.x;
    const int64_t tiles = (int64_t)a.nblocks * a.n_energy;
    const int64_t slots = (a.n_max + kSpecGroup - 1) / kSpecGroup - 1;
    cd* ck = a.work + wave * (slots > 0 ? slots : 1) * kWave + lane;
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int e = (int)(tile / a.nblocks);
        const int blk = (int)(tile - (int64_t)e * a.nblocks);
        const SpecClass s = scalar_load(a.spec + spec_entry(a.spec, a.nspec, blk));
        const int k = (blk - s.blk0) * kWave + lane;
        const bool valid = k < s.count;
        const int n = s.n;
        // lanes past the last system repeat it (in bounds, nothing written)
        const cd* rb = a.rhs + s.rhs_off + (valid ? k : s.count - 1);
        const int64_t rs = s.count;  // right-hand side stride per point
        const cd* f = a.fac + 3 * ((int64_t)s.cls * a.n_energy + e) * a.n_max;
        const int ng = (n + kSpecGroup - 1) / kSpecGroup;
        const int nfull = n / kSpecGroup;  // groups of kSpecGroup points (no tail)
        // forward sweep, keeping d'_{j0 - 1} of every group j0 > 0; full
        // groups run without conditions, so their loads issue ahead
        cd dp = czero();
        for (int g = 0; g < ng; ++g) {
            const int j0 = g * kSpecGroup;
            if (g > 0) ck[(int64_t)(g - 1) * kWave] = dp;
            const cd* fg = f + 3 * (int64_t)j0;
            const cd* bg = rb + j0 * rs;
            if (g < nfull) {
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u) dp = spec_step(fg + 3 * u, bg + u * rs, dp);
            } else {
                for (int u = 0; j0 + u < n; ++u) dp = spec_step(fg + 3 * u, bg + u * rs, dp);
            }
        }
        // backward sweep group by group: recompute the group's d' from its
        // start value, then walk it backwards accumulating |phi|^2
        double acc = 0.0;
        cd phi = czero();
        // each group's start value is read one group ahead, so that its
        // memory latency overlaps the group before it
        cd x_next = ng > 1 ? ck[(int64_t)(ng - 2) * kWave] : czero();
        for (int g = ng - 1; g >= 0; --g) {
            const int j0 = g * kSpecGroup;
            const cd* fg = f + 3 * (int64_t)j0;
            const cd* bg = rb + j0 * rs;
            cd x = x_next;
            x_next = g > 1 ? ck[(int64_t)(g - 2) * kWave] : czero();
            cd dd[kSpecGroup];
            if (g < nfull) {
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u) {
                    x = spec_step(fg + 3 * u, bg + u * rs, x);
                    dd[u] = x;
                }
#pragma unroll
                for (int u = kSpecGroup - 1; u >= 0; --u) {
                    phi = cmad(scalar_load(fg + 3 * u + 2), phi, dd[u]);
                    acc = fma(phi.re, phi.re, fma(phi.im, phi.im, acc));
                }
            } else {
#pragma unroll
                for (int u = 0; u < kSpecGroup; ++u) {
                    if (j0 + u < n) x = spec_step(fg + 3 * u, bg + u * rs, x);
                    dd[u] = x;
                }
#pragma unroll
                for (int u = kSpecGroup - 1; u >= 0; --u) {
                    if (j0 + u < n) {
                        phi = cmad(scalar_load(fg + 3 * u + 2), phi, dd[u]);
                        acc = fma(phi.re, phi.re, fma(phi.im, phi.im, acc));
                    }
                }
            }
        }
        if (valid)
            a.out[(int64_t)a.order[s.start + k] * a.n_energy + e] =
                a.eps / M_PI * a.classes[s.cls].dx * acc;
    }
}

// Trapezoid integral of each row of a spectrum over the grid points at or
// above e_lo: one wavefront per row, lanes striding over the intervals, a
// fixed-order wave sum.
__global__ void __launch_bounds__(kWave) energy_integral_kernel(int32_t n_energy,
                                                                const double* energies,
                                                                const double* spectrum,
                                                                double e_lo, double* out)
{
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const double* p = spectrum + (int64_t)b * n_energy;
    double acc = 0.0;
    for (int q = lane; q + 1 < n_energy; q += kWave) {
        const double e0 = energies[q], e1 = energies[q + 1];
        if (e0 >= e_lo && e1 >= e_lo) acc = fma(0.5 * (e1 - e0), p[q] + p[q + 1], acc);
    }
    acc = wave_sum(acc);
    if (lane == kSumLane) out[b] = acc;
}

hipError_t launch_energy_integral(int batch, int n_energy, const double* energies,
                                  const double* spectrum, double e_lo, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(energy_integral_kernel, dim3(batch), dim3(kWave), 0, st, n_energy, energies,
                       spectrum, e_lo, out);
    return hipGetLastError();
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
    const size_t vbytes = sizeof(double) * (size_t)a.n_max;
    if (vbytes > (size_t)kMaxLds) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(spectrum_factor_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    hipLaunchKernelGGL(spectrum_factor_kernel, dim3(a.pairs), dim3(kWave), vbytes, st, a);
    hipLaunchKernelGGL(spectrum_rhs_kernel, dim3((a.n_max + 3) / 4, std::min(a.nblocks, 65535)),
                       dim3(256), 0, st, a);
    hipLaunchKernelGGL(energy_spectrum_kernel, dim3((unsigned)(a.lanes / kWave)), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
