// tdse_forward.hip -- persistent batched forward propagation and the
// imaginary-time ground state on gfx950.
//
// Layout: a workgroup holds S subgroups of T = 64 W lanes; each subgroup owns
// one system at a time and lane t keeps grid points [t C, t C + C) of psi in
// VGPRs for the whole time loop, plus one ghost value on each side, and up
// to 8 points per lane also the pivot factors q of its chunk.  The systems of
// one size in a workgroup share one copy of the size class's om and dV/dx
// tables in LDS (16 bytes per point), staged once per bin; where they do not
// fit, om alone or neither is staged (TAB).  Per step (section
// "1D-TSDE Implementation (CTDSE)", three substeps):
//   1. r = 12 R psi in place                      (first substep)
//   2. L y = r by a partitioned Thomas solve      (second substep):
//      lane-local recurrences, carries across lanes by a Kogge-Stone scan
//      within the wavefront and one LDS exchange between wavefronts
//   3. psi_j = m_j exp(-i dt E_i x_j) y_j         (third substep + absorber)
//   4. per-lane partial sums of |psi|^2, x|psi|^2, V'|psi|^2, wavefront sums,
//      a ring of per-wave partials in LDS flushed every 32 samples as
//      coalesced rows of accel/xexp/norm.
// Only E_i (8 B per system-step) is read from HBM inside the loop and only
// the three observables (24 B per system-step) are written.
#include "tdse_device.hpp"
#include "tdse_kernels.hpp"

namespace tdse {

// s_getreg operand of the XCC_ID hardware register (id 20), bits 3:0: the
// accelerator complex die a wave runs on (size - 1 = 3 goes in bits 15:11).
constexpr int kHwRegXccId = 20;

size_t sub_smem_bytes(int W)
{
    size_t b = sizeof(cd) * 2 * kMaxWaves + sizeof(double) * 2 * kMaxWaves + sizeof(cd) * kFlush +
               sizeof(double) * kRing * W * 3 + 4 * sizeof(int);
    return (b + 15) & ~size_t(15);
}

// -------------------------------------------------------------- forward
// Phase ratios of steps [i0, i0 + F) below nt into the subgroup's LDS block,
// one step per lane of its first wavefront: the per-step sincos of
// phase_ratio runs once per F steps instead of once per step.  Written after
// a barrier that follows every read of the previous block; the step's solve
// takes two more barriers before its phase reads them.
__device__ __forceinline__ void fill_ratios(cd* ratio, const double* erow, int i0, int nt, int F,
                                            double dt, double dx, int wsys, int lane)
{
    if (wsys == 0 && lane < F && i0 + lane < nt) ratio[lane] = phase_ratio(erow[i0 + lane], dt, dx);
}

// Persistent: each workgroup takes bins from the run of its XCD, then from
// the other runs (a.queue).  A bin is a set of
// systems of one lane layout that together fill the workgroup's lanes (plus a
// padding system where they do not); every subgroup runs the whole time loop
// of its system with the same barrier sequence as the others.
// X selects what the time loop records besides the outputs: kFwdPlain
// nothing; kFwdPop the ground-state and volumetric populations at every
// sample (six ring values per wavefront and sample, flushed every
// kFlush / 2); kFwdStore the adjoint's checkpoints, the state record (chunk
// and ghosts) of every K-th step and the norm row, in each system's part of
// the checkpoint store.
constexpr int kFwdPlain = 0;
constexpr int kFwdPop = 1;
constexpr int kFwdStore = 2;

// NARROW: workgroups of at most 512 threads, 2 waves per SIMD with 256
// registers per lane instead of 4 with 128.  At 8 points per lane the wide
// instances spill about 20 registers per lane; at 16 the narrow ones also
// keep the pivot factors in registers, as the shorter chunks do.
template <int C, bool NARROW>
struct FwdQRegs {
    static constexpr bool value = NARROW ? C <= 16 : QInRegs<C>::value;
};

template <int C, int TAB, bool AB = false, int X = kFwdPlain, bool NARROW = false>
__global__ void __launch_bounds__(NARROW ? 512 : 1024) forward_kernel(FwdArgs a)
{
    constexpr bool QREG = FwdQRegs<C, NARROW>::value;
    constexpr bool POP = X == kFwdPop;
    constexpr bool STORE = X == kFwdStore;
    constexpr int NV = POP ? 6 : 3;                   // ring values per wavefront and sample
    constexpr int RING = POP ? kRing / 2 : kRing;     // samples in the ring (same LDS bytes)
    constexpr int FLUSH = POP ? kFlush / 2 : kFlush;  // samples per output flush
    extern __shared__ double smem_raw[];
    char* const smem = reinterpret_cast<char*>(smem_raw);
    const int tid = threadIdx.x;
    const int wv = uniform(tid / kWave);  // wavefront within the workgroup
    int* wg_item = reinterpret_cast<int*>(smem + a.item_off);
    const int nt = a.nt;

    for (;;) {
        if (tid == 0) {
            // the run of the XCD this workgroup runs on first (its tables
            // stay in that XCD's L2), then what is left in the other runs;
            // everything is read here so that nothing stays live in the loop
            const int home = __builtin_amdgcn_s_getreg((3 << 11) | kHwRegXccId) & (kXcds - 1);
            const int32_t* bound = a.queue + kXcds;
            int item = a.nbins;
            for (int k = 0; k < kXcds; ++k) {
                const int x = (home + k) & (kXcds - 1);
                const int lo = bound[x], hi = bound[x + 1];
                if (lo >= hi) continue;
                const int i = atomicAdd(a.queue + x, 1);
                if (lo + i < hi) {
                    item = lo + i;
                    break;
                }
            }
            wg_item[0] = item;
        }
        __syncthreads();
        const int b = uniform(wg_item[0]);
        if (b >= a.nbins) break;
        const BinDesc* bd = a.bins + b;
        const int j = scalar_load(bd->sub_of_wave + wv);
        const BinSub bs = scalar_load(bd->sub + j);
        const SizeClass* const clsp = a.classes + bs.cls;
        const SizeClass sc = scalar_load(clsp);
        const int T = sc.T, W = T / kWave;
        const int wsys = wv - bs.wave0;  // wavefront within the system
        const int t = wsys * kWave + (tid & (kWave - 1));
        double* const tab = reinterpret_cast<double*>(smem + bs.tab_off);
        const SubSmem sm = carve_sub(smem + bs.sub_off, W);
        const bool active = bs.p >= 0;  // uniform within the subgroup
        const int p = active ? bs.p : 0;
        const double dx = sc.dx;
        const int n = sc.n, s = t * C;
        if (TAB != kTabGlobal && bs.stage) {
            const int np = C * T;
            for (int i = t; i < np; i += T) {
                tab[i] = sc.pt.om[i];
                if (TAB == kTabLds) tab[np + i] = sc.pt.dv[i];
            }
        }
        if (t == 0) sm.misc[1] = 0;
        __syncthreads();

        const SysDesc d = uniform_load(a.sys + p);
        const double* src = nullptr;
        if (active) src = a.psi0 ? a.psi0 + 2 * d.psi_off : a.gs + 2 * a.gs_off[bs.cls];
        const size_t row = (size_t)p * (size_t)(nt + 1);
        const double* erow = a.E + row;
        double* acc_row = a.accel + row;
        double* x_row = a.xexp ? a.xexp + row : nullptr;
        double* n_row = a.norm ? a.norm + row : nullptr;
        double* gs_row = (POP && a.gs_pop) ? a.gs_pop + row : nullptr;
        double* vol_row = (POP && a.vol_pop) ? a.vol_pop + row : nullptr;
        // checkpoint store of the system: records of (C+2) T complex values
        // at steps 0, K, 2K, ..., then the norm row
        const int K = STORE ? a.k_ckpt : 1;
        const size_t np2 = 2 * (size_t)(C + 2) * T;
        double* st_norm = nullptr;
        if (STORE && active) st_norm = a.store + uniform_load(a.store_off + p) + np2 * (size_t)(nt / K + 1);
        // reference state of the ground-state population (inactive subgroups
        // read one valid element)
        const double* phi = a.gs;
        int n_pop = 1;
        if (POP && active) {
            phi = a.pop_ref ? a.pop_ref + 2 * d.psi_off : a.gs + 2 * a.gs_off[bs.cls];
            n_pop = n;
        }

        cd v[C];
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = (active && s + k < n) ? ld_psi(src, s + k) : czero();
        cd gl = (active && s > 0 && s - 1 < n) ? ld_psi(src, s - 1) : czero();
        cd gr = (active && s + C < n) ? ld_psi(src, s + C) : czero();

        LaneFactors<C, QREG, AB> f;
        {
            const StepView<TAB> sv = step_view<TAB>(clsp, wsys, tab);
            f = load_factors<C, QREG, AB>(sv.sc, sv.lc);
            if constexpr (POP)
                observe_pop<C>(v, sv.tb, T, sv.lc, sv.xs, dx, n_pop, phi, a.pop_radius, sm.ring);
            else
                observe<C>(v, sv.tb, T, sv.lc, sv.xs, dx, sm.ring);
        }
        fill_ratios(sm.ratio, erow, 0, nt, FLUSH, a.dt, dx, wsys, tid & (kWave - 1));
        __syncthreads();
        double n0 = 0.0;
        for (int w = 0; w < W; ++w) n0 += sm.ring[w * NV + 2];
        n0 *= dx;

        int flushed = 0;
        for (int i = 0; i < nt; ++i) {
            const StepView<TAB> sv = step_view<TAB>(clsp, wsys, tab);
            if constexpr (STORE) {
                if (active && i % K == 0)
                    store_state<C>(a.store + uniform_load(a.store_off + p) + np2 * (size_t)(i / K),
                                   sv.sc.T, 16u * (unsigned)sv.lc.t, v, gl, gr);
            }
            forward_step<C>(v, gl, gr, f, erow[i], RatioLds{sm.ratio + i % FLUSH}, a.dt, sv.xl,
                            sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
            if ((i + 1) % FLUSH == 0) {
                __syncthreads();
                if (active)
                    flush<POP>(i + 1 - FLUSH, i, t, T, sm.ring, W, dx, erow, acc_row, x_row, n_row,
                               n0, sm.misc + 1, gs_row, vol_row, STORE ? st_norm : nullptr);
                fill_ratios(sm.ratio, erow, i + 1, nt, FLUSH, a.dt, dx, wsys, tid & (kWave - 1));
                flushed = i + 1;
            }
            double* slot = sm.ring + ((i + 1) % RING) * W * NV;
            if constexpr (POP)
                observe_pop<C>(v, sv.tb, sv.sc.T, sv.lc, sv.xs, sv.sc.dx, n_pop, phi, a.pop_radius,
                               slot);
            else
                observe<C>(v, sv.tb, sv.sc.T, sv.lc, sv.xs, sv.sc.dx, slot);
        }
        __syncthreads();
        if constexpr (STORE) {
            if (active && nt % K == 0)
                store_state<C>(a.store + uniform_load(a.store_off + p) + np2 * (size_t)(nt / K), T,
                               16u * (unsigned)t, v, gl, gr);
        }
        if (active) {
            flush<POP>(flushed, nt, t, T, sm.ring, W, dx, erow, acc_row, x_row, n_row, n0,
                       sm.misc + 1, gs_row, vol_row, STORE ? st_norm : nullptr);
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
        }
        __syncthreads();
        if (active && t == 0 && a.status) a.status[p] = sm.misc[1];
    }
}

// -------------------------------------------------------------- ground state
// Imaginary-time relaxation: psi <- L_tau^{-1} R_tau psi with dt -> -i dtau,
// renormalised to dx sum |psi|^2 = 1 each iteration, until successive
// iterates differ by less than tol.  The energy follows from the growth
// factor g = ||L_tau^{-1} R_tau psi|| of the converged eigenvector:
// g = (1 - dtau E/2)/(1 + dtau E/2).  One workgroup per candidate; all
// candidates of a launch share one lane layout.
template <int C>
__global__ void __launch_bounds__(1024) gs_kernel(GsArgs a)
{
    extern __shared__ double smem_raw[];
    const int cand = blockIdx.x;
    const SizeClass* const clsp = a.classes + uniform(a.cls_of[cand]);
    const SizeClass sc = uniform_load(clsp);
    const int tid = threadIdx.x;
    const int W = sc.T / kWave;
    const SubSmem sm = carve_sub(reinterpret_cast<char*>(smem_raw), W);
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const double dx = sc.dx;
    const int n = sc.n, s = tid * C;
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

    // workgroup sum in fixed wave order; consecutive sums alternate slot arrays
    auto block_sum = [&](double x, double* slots) {
        x = wave_sum(x);
        if (lane == kSumLane) slots[wave] = x;
        __syncthreads();
        double r = 0.0;
        for (int w = 0; w < W; ++w) r += slots[w];
        return r;
    };

    double loc = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) loc += cabs2(v[k]);
    double tot = block_sum(loc, sm.red0);
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
    const LaneFactors<C> f = load_factors<C>(sc, make_lane_ctx(sc, tid, uniform(tid / kWave)));
    while (it < a.max_iter) {
        const StepView<false> sv = step_view<false>(clsp, uniform(tid / kWave), smem_raw);
        cn_apply<C, false>(v, gl, gr, f, sv.tb, sv.sc, sv.lc, sv.rc, sm.lds_f, sm.lds_b);
        loc = 0.0;
#pragma unroll
        for (int k = 0; k < C; ++k) loc += cabs2(v[k]);
        tot = block_sum(loc, sm.red1);
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
        tot = block_sum(loc, sm.red0);
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

__global__ void reset_queues_kernel(int32_t* q, int nq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq * kXcds) q[(i / kXcds) * kQueueInts + i % kXcds] = 0;
}

hipError_t launch_reset_queues(int32_t* queues, int nq, hipStream_t st)
{
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_queues_kernel, dim3((nq * kXcds + 63) / 64), dim3(64), 0, st, queues, nq);
    return hipGetLastError();
}

hipError_t launch_reset_counters(int32_t* counters, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_counters_kernel, dim3((n + 63) / 64), dim3(64), 0, st, counters, n);
    return hipGetLastError();
}

bool layout_supported(int C) { return C == 4 || C == 8 || C == 12 || C == 16; }

template <int C, int TAB, bool NARROW = false>
static int occ_fwd(int threads, size_t sh)
{
    int nb = 0;
    void (*k)(FwdArgs) = forward_kernel<C, TAB, false, kFwdPlain, NARROW>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)) != hipSuccess ||
        threads > fa.maxThreadsPerBlock)
        return 0;  // beyond the kernel's launch bounds
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, sh) != hipSuccess) return 0;
    return nb;
}

// Layouts with narrow instances, used for workgroups of at most 512 threads.
bool forward_narrow(int C, int threads) { return (C == 8 || C == 16) && threads <= 512; }

// Instantiated layouts: C in {4, 8, 12, 16} with tables in global memory or
// in LDS; om alone in LDS only for 12 and 16 points per lane (the grids whose
// full tables do not fit).  12 points per lane (forward only) fill 1024-lane
// workgroups at N = 12288, where 16 points leave a quarter of them idle.
bool forward_tab_supported(int C, int tab)
{
    if (!layout_supported(C)) return false;
    return tab == kTabGlobal || tab == kTabLds || (tab == kTabOmLds && C >= 12);
}

int forward_occupancy(int C, int threads, size_t smem, int tab)
{
    if (smem > (size_t)kMaxLds || threads < kWave || threads > 1024 || threads % kWave) return 0;
    if (forward_narrow(C, threads)) {
        switch (C * 4 + tab) {
            case 32: return occ_fwd<8, kTabGlobal, true>(threads, smem);
            case 33: return occ_fwd<8, kTabLds, true>(threads, smem);
            case 64: return occ_fwd<16, kTabGlobal, true>(threads, smem);
            case 65: return occ_fwd<16, kTabLds, true>(threads, smem);
            case 66: return occ_fwd<16, kTabOmLds, true>(threads, smem);
            default: return 0;
        }
    }
    switch (C * 4 + tab) {
        case 16: return occ_fwd<4, kTabGlobal>(threads, smem);
        case 17: return occ_fwd<4, kTabLds>(threads, smem);
        case 32: return occ_fwd<8, kTabGlobal>(threads, smem);
        case 33: return occ_fwd<8, kTabLds>(threads, smem);
        case 48: return occ_fwd<12, kTabGlobal>(threads, smem);
        case 49: return occ_fwd<12, kTabLds>(threads, smem);
        case 50: return occ_fwd<12, kTabOmLds>(threads, smem);
        case 64: return occ_fwd<16, kTabGlobal>(threads, smem);
        case 65: return occ_fwd<16, kTabLds>(threads, smem);
        case 66: return occ_fwd<16, kTabOmLds>(threads, smem);
        default: return 0;
    }
}

template <int C, int TAB, bool AB, bool NARROW = false>
static int regs_fwd()
{
    hipFuncAttributes fa;
    void (*k)(FwdArgs) = forward_kernel<C, TAB, AB, kFwdPlain, NARROW>;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)) != hipSuccess) return 0;
    return fa.numRegs;
}

int forward_vgprs(int C, int tab, bool ab, int threads)
{
    if (forward_narrow(C, threads)) {
        switch (C * 4 + tab) {
            case 32: return regs_fwd<8, kTabGlobal, false, true>();
            case 33: return regs_fwd<8, kTabLds, false, true>();
            case 64: return regs_fwd<16, kTabGlobal, false, true>();
            case 65: return regs_fwd<16, kTabLds, false, true>();
            case 66: return regs_fwd<16, kTabOmLds, false, true>();
            default: return 0;
        }
    }
    if (C >= 12 && ab) {
        switch (C * 4 + tab) {
            case 48: return regs_fwd<12, kTabGlobal, true>();
            case 49: return regs_fwd<12, kTabLds, true>();
            case 50: return regs_fwd<12, kTabOmLds, true>();
            case 64: return regs_fwd<16, kTabGlobal, true>();
            case 65: return regs_fwd<16, kTabLds, true>();
            case 66: return regs_fwd<16, kTabOmLds, true>();
            default: return 0;
        }
    }
    switch (C * 4 + tab) {
        case 16: return regs_fwd<4, kTabGlobal, false>();
        case 17: return regs_fwd<4, kTabLds, false>();
        case 32: return regs_fwd<8, kTabGlobal, false>();
        case 33: return regs_fwd<8, kTabLds, false>();
        case 48: return regs_fwd<12, kTabGlobal, false>();
        case 49: return regs_fwd<12, kTabLds, false>();
        case 50: return regs_fwd<12, kTabOmLds, false>();
        case 64: return regs_fwd<16, kTabGlobal, false>();
        case 65: return regs_fwd<16, kTabLds, false>();
        case 66: return regs_fwd<16, kTabOmLds, false>();
        default: return 0;
    }
}

template <int X>
static hipError_t launch_forward_t(int C, int tab, const FwdArgs& a, int threads, size_t smem,
                                   int grid, hipStream_t st)
{
    const dim3 b(threads);
    // narrow instances hold q in registers and form the elimination factors
    if (forward_narrow(C, threads)) {
        switch (C * 4 + tab) {
            case 32: hipLaunchKernelGGL((forward_kernel<8, kTabGlobal, false, X, true>), dim3(grid), b, smem, st, a); break;
            case 33: hipLaunchKernelGGL((forward_kernel<8, kTabLds, false, X, true>), dim3(grid), b, smem, st, a); break;
            case 64: hipLaunchKernelGGL((forward_kernel<16, kTabGlobal, false, X, true>), dim3(grid), b, smem, st, a); break;
            case 65: hipLaunchKernelGGL((forward_kernel<16, kTabLds, false, X, true>), dim3(grid), b, smem, st, a); break;
            case 66: hipLaunchKernelGGL((forward_kernel<16, kTabOmLds, false, X, true>), dim3(grid), b, smem, st, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    // 12 and 16 points per lane: elimination factors from their tables
    // (a.ab) or formed from q and om
    if (C >= 12 && a.ab) {
        switch (C * 4 + tab) {
            case 48: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabGlobal, true, X>), dim3(grid), b, smem, st, a); } break;
            case 49: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabLds, true, X>), dim3(grid), b, smem, st, a); } break;
            case 50: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabOmLds, true, X>), dim3(grid), b, smem, st, a); } break;
            case 64: hipLaunchKernelGGL((forward_kernel<16, kTabGlobal, true, X>), dim3(grid), b, smem, st, a); break;
            case 65: hipLaunchKernelGGL((forward_kernel<16, kTabLds, true, X>), dim3(grid), b, smem, st, a); break;
            case 66: hipLaunchKernelGGL((forward_kernel<16, kTabOmLds, true, X>), dim3(grid), b, smem, st, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (C * 4 + tab) {
        case 16: hipLaunchKernelGGL((forward_kernel<4, kTabGlobal, false, X>), dim3(grid), b, smem, st, a); break;
        case 17: hipLaunchKernelGGL((forward_kernel<4, kTabLds, false, X>), dim3(grid), b, smem, st, a); break;
        case 32: hipLaunchKernelGGL((forward_kernel<8, kTabGlobal, false, X>), dim3(grid), b, smem, st, a); break;
        case 33: hipLaunchKernelGGL((forward_kernel<8, kTabLds, false, X>), dim3(grid), b, smem, st, a); break;
        case 48: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabGlobal, false, X>), dim3(grid), b, smem, st, a); } break;
        case 49: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabLds, false, X>), dim3(grid), b, smem, st, a); } break;
        case 50: if constexpr (X != kFwdStore) { hipLaunchKernelGGL((forward_kernel<12, kTabOmLds, false, X>), dim3(grid), b, smem, st, a); } break;
        case 64: hipLaunchKernelGGL((forward_kernel<16, kTabGlobal, false, X>), dim3(grid), b, smem, st, a); break;
        case 65: hipLaunchKernelGGL((forward_kernel<16, kTabLds, false, X>), dim3(grid), b, smem, st, a); break;
        case 66: hipLaunchKernelGGL((forward_kernel<16, kTabOmLds, false, X>), dim3(grid), b, smem, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward(int C, int tab, const FwdArgs& a, int threads, size_t smem, int grid,
                          hipStream_t st)
{
    if (smem > (size_t)kMaxLds || threads < kWave || threads > 1024 || threads % kWave ||
        (size_t)a.item_off + 16 > smem)
        return hipErrorInvalidValue;
    if (a.store) {
        if (a.gs_pop || a.vol_pop || C == 12 || a.k_ckpt < 1) return hipErrorInvalidValue;
        return launch_forward_t<kFwdStore>(C, tab, a, threads, smem, grid, st);
    }
    if (a.gs_pop || a.vol_pop) return launch_forward_t<kFwdPop>(C, tab, a, threads, smem, grid, st);
    return launch_forward_t<kFwdPlain>(C, tab, a, threads, smem, grid, st);
}

hipError_t launch_ground_state(int C, const GsArgs& a, int T, hipStream_t st)
{
    const size_t sh = sub_smem_bytes(T / kWave) + 16;
    switch (C) {
        case 4: hipLaunchKernelGGL(gs_kernel<4>, dim3(a.ncand), dim3(T), sh, st, a); break;
        case 8: hipLaunchKernelGGL(gs_kernel<8>, dim3(a.ncand), dim3(T), sh, st, a); break;
        case 12: hipLaunchKernelGGL(gs_kernel<12>, dim3(a.ncand), dim3(T), sh, st, a); break;
        case 16: hipLaunchKernelGGL(gs_kernel<16>, dim3(a.ncand), dim3(T), sh, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tdse
