// tdse_tables.hip -- plan tables of one size class, built on the device.
//
// The Crank-Nicolson left-hand side L = M2 + h A (section "1D-TSDE
// Implementation (CTDSE)", second substep) does not depend on time because
// the field enters only through the third (phase) substep.  Its
// factorisation is therefore computed once per (n, dx, h, a) and reused by
// every step of every system of that size.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

__device__ __forceinline__ double soft_core(double x, double a, double z)
{
    return z == 0.0 ? 0.0 : -z / sqrt(fma(x, x, a * a));
}
__device__ __forceinline__ double soft_core_slope(double x, double a, double z)
{
    if (z == 0.0) return 0.0;
    const double s = fma(x, x, a * a);
    return z * x / (s * sqrt(s));
}
// Absorber on the outer fraction `frac` of the grid at each side: the grid
// spans 2 x_max, so it starts at x_a = x_max - 2 frac x_max.  1 for
// |x| <= x_a, cos(pi/2 (|x|-x_a)/(x_max-x_a))^power up to x_max, and 0 at
// |x| >= x_max.
__device__ __forceinline__ double absorber(double ax, double xmax, double frac, double power)
{
    const double xa = xmax - 2.0 * frac * xmax;
    if (frac <= 0.0 || ax <= xa) return 1.0;
    if (ax >= xmax) return 0.0;
    return pow(cos(0.5 * M_PI * (ax - xa) / (xmax - xa)), power);
}

// One workgroup per size class.
__global__ void __launch_bounds__(256) build_tables_kernel(const SizeClass* classes,
                                                           const TableParams* params,
                                                           double* metrics /* [cls][2][7] */,
                                                           cd* scratch /* [cls][2][T] */,
                                                           int max_t)
{
    const SizeClass sc = classes[blockIdx.x];
    const TableParams P = params[blockIdx.x];
    const int n = sc.n, C = sc.C, T = sc.T, np = C * T;
    const double dx = P.dx;
    const double xmax = 0.5 * (double)(n - 1) * dx;
    cd* ca = scratch + (size_t)blockIdx.x * 2 * max_t;  // chunk products of alpha
    cd* cb = ca + max_t;                                 // chunk products of beta

    // 1. potential, slope, absorber and om at every (padded) point
    const double habs = sqrt(P.h.re * P.h.re + P.h.im * P.h.im);
    const double kw = 12.0 * habs;
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        const int idx = pidx(j / C, j % C, C);
        if (j < n) {
            const double x = ((double)j - 0.5 * (double)(n - 1)) * dx;
            const double vj = soft_core(x, P.a, P.z);
            sc.pt.v[idx] = vj;
            sc.pt.om[idx] = kw * (vj / 12.0 - 0.5 / (dx * dx));
            sc.pt.dv[idx] = soft_core_slope(x, P.a, P.z);
            sc.pt.m[idx] = absorber(fabs(x), xmax, P.mask_frac, P.mask_pow);
        } else {
            sc.pt.v[idx] = 0.0;
            sc.pt.om[idx] = 0.0;
            sc.pt.dv[idx] = 0.0;
            sc.pt.m[idx] = 0.0;
        }
    }
    __syncthreads();

    // 2. LU factorisation without pivoting (sequential in j)
    if (threadIdx.x == 0) {
        const double m2d = 10.0 / 12.0, m2o = 1.0 / 12.0;
        const double inv_dx2 = 1.0 / (dx * dx);
        cd q_prev = czero(), u_prev = czero(), l_prev = czero();
        for (int j = 0; j < np; ++j) {
            const int idx = pidx(j / C, j % C, C);
            cd q = czero();
            if (j < n) {
                const double vj = sc.pt.v[idx];
                // diagonal of L: 10/12 + h (1/dx^2 + 10/12 V_j)
                const double ad = inv_dx2 + m2d * vj;
                cd d = mkc(m2d + P.h.re * ad, P.h.im * ad);
                if (j > 0) {
                    const cd ell = cmul(l_prev, q_prev);          // l_{j-1} / p_{j-1}
                    d = mkc(d.re - (ell.re * u_prev.re - ell.im * u_prev.im),
                            d.im - (ell.re * u_prev.im + ell.im * u_prev.re));
                }
                q = cinv(d);
                if (j + 1 < n) {
                    const double xn = ((double)(j + 1) - 0.5 * (double)(n - 1)) * dx;
                    const double vn = soft_core(xn, P.a, P.z);
                    // superdiagonal (j, j+1): 1/12 + h (-1/(2dx^2) + V_{j+1}/12)
                    const double au = -0.5 * inv_dx2 + m2o * vn;
                    u_prev = mkc(m2o + P.h.re * au, P.h.im * au);
                    // subdiagonal (j+1, j): 1/12 + h (-1/(2dx^2) + V_j/12)
                    const double al = -0.5 * inv_dx2 + m2o * vj;
                    l_prev = mkc(m2o + P.h.re * al, P.h.im * al);
                }
                q_prev = q;
            }
            sc.pt.q[idx] = cscale(1.0 / 12.0, q);
        }
    }
    __syncthreads();

    // 2b. elimination factors from the stored om and q, by the kernels' own
    // formula (so a kernel that loads them gets the values it would compute):
    //   alpha_j = -(1 + h' om_{j-1}) q_{j-1},  beta_j = -(1 + h' om_{j+1}) q_j
    const bool rt = P.h.im != 0.0;
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        const int idx = pidx(j / C, j % C, C);
        cd alpha = czero(), beta = czero();
        if (j < n) {
            if (j > 0) {
                const int ip = pidx((j - 1) / C, (j - 1) % C, C);
                alpha = rt ? elim<true>(sc.pt.om[ip], sc.pt.q[ip]) : elim<false>(sc.pt.om[ip], sc.pt.q[ip]);
            }
            if (j + 1 < n) {
                const int in = pidx((j + 1) / C, (j + 1) % C, C);
                beta = rt ? elim<true>(sc.pt.om[in], sc.pt.q[idx]) : elim<false>(sc.pt.om[in], sc.pt.q[idx]);
            }
        }
        sc.pt.alpha[idx] = alpha;
        sc.pt.beta[idx] = beta;
    }
    __syncthreads();

    // 3. per lane: chunk products of alpha and beta, absorber flags
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        cd pr = mkc(1.0, 0.0);
        int flags = 0;
        for (int k = 0; k < C; ++k) {
            pr = cmul(sc.pt.alpha[pidx(t, k, C)], pr);
            if (sc.pt.m[pidx(t, k, C)] != 1.0) flags |= 1;
        }
        ca[t] = pr;
        pr = mkc(1.0, 0.0);
        for (int k = C - 1; k >= 0; --k) pr = cmul(sc.pt.beta[pidx(t, k, C)], pr);
        cb[t] = pr;
        if (t > 0 && sc.pt.m[pidx(t - 1, C - 1, C)] != 1.0) flags |= 2;
        if (t + 1 < T && sc.pt.m[pidx(t + 1, 0, C)] != 1.0) flags |= 4;
        sc.lt.hasmask[t] = flags;
    }
    __syncthreads();

    // 4. scan window products and truncation metrics
    __shared__ double red[2][kMaxLevels + 1][256];
    for (int t0 = 0; t0 < T; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        double mA[kMaxLevels + 1], mB[kMaxLevels + 1];
        for (int lev = 0; lev <= kMaxLevels; ++lev) mA[lev] = mB[lev] = 0.0;
        if (t < T) {
            const int ws = (t / kWave) * kWave, we = ws + kWave - 1;
            for (int lev = 0; lev < kMaxLevels; ++lev) {
                const int w = 1 << lev;
                cd pa = mkc(1.0, 0.0), qb = mkc(1.0, 0.0);
                for (int u = max(t - w + 1, ws); u <= t; ++u) pa = cmul(ca[u], pa);
                for (int u = min(t + w - 1, we); u >= t; --u) qb = cmul(cb[u], qb);
                sc.lt.pa[lev * T + t] = pa;
                sc.lt.qb[lev * T + t] = qb;
            }
            cd pw = mkc(1.0, 0.0), qw = mkc(1.0, 0.0);
            for (int u = ws; u <= t; ++u) pw = cmul(ca[u], pw);
            for (int u = we; u >= t; --u) qw = cmul(cb[u], qw);
            sc.lt.pw[t] = pw;
            sc.lt.qw[t] = qw;
            // full windows of 2^lev lanes (crossing wave boundaries): the term a
            // scan with `lev` levels would drop is bounded by these products
            for (int lev = 0; lev <= kMaxLevels; ++lev) {
                const int w = 1 << lev;
                if (t - w + 1 >= 0) {
                    cd p = mkc(1.0, 0.0);
                    for (int u = t - w + 1; u <= t; ++u) p = cmul(ca[u], p);
                    mA[lev] = sqrt(cabs2(p));
                }
                if (t + w - 1 < T) {
                    cd p = mkc(1.0, 0.0);
                    for (int u = t; u <= t + w - 1; ++u) p = cmul(cb[u], p);
                    mB[lev] = sqrt(cabs2(p));
                }
            }
        }
        for (int lev = 0; lev <= kMaxLevels; ++lev) {
            red[0][lev][threadIdx.x] = mA[lev];
            red[1][lev][threadIdx.x] = mB[lev];
        }
        __syncthreads();
        if (threadIdx.x < 2 * (kMaxLevels + 1)) {
            const int which = threadIdx.x / (kMaxLevels + 1), lev = threadIdx.x % (kMaxLevels + 1);
            double mx = t0 == 0 ? 0.0 : metrics[(blockIdx.x * 2 + which) * (kMaxLevels + 1) + lev];
            for (int i = 0; i < (int)blockDim.x; ++i) mx = fmax(mx, red[which][lev][i]);
            metrics[(blockIdx.x * 2 + which) * (kMaxLevels + 1) + lev] = mx;
        }
        __syncthreads();
    }
}

hipError_t launch_build_tables(const SizeClass* d_classes, const TableParams* d_params, int ncls,
                               double* d_metrics, cd* d_scratch, int max_t, hipStream_t st)
{
    hipLaunchKernelGGL(build_tables_kernel, dim3(ncls), dim3(256), 0, st, d_classes, d_params,
                       d_metrics, d_scratch, max_t);
    return hipGetLastError();
}

}  // namespace tdse
