// libtdse.cpp -- host side of the libtdse C-ABI (include/libtdse.h): argument
// validation, plans (size classes, device tables, ground states, work
// queues, workspaces), hipGraph capture and replay, the ground-state and
// soft-core-fit drivers.  All numerical work runs in the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include <unistd.h>

#include "libtdse.h"
#include "tdse_internal.hpp"
#include "tdse_kernels.hpp"

using namespace tdse;

namespace {

thread_local std::string g_last_error;

tdse_status fail(tdse_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(TDSE_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                            \
    } while (0)

constexpr double kTruncEps = 1.3877787807814457e-17;  // 2^-56
constexpr int kMaxN = 16384;
constexpr int kMinN = 16;

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int num_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// ------------------------------------------------------------ device arena
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
    template <class T>
    T* take(size_t count)
    {
        size_t bytes = (sizeof(T) * count + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};

// Lane layout for a grid of n points: C points per lane, T lanes.
struct Layout {
    int C, T;
};

int env_int(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

double env_double(const char* name, double dflt)
{
    const char* v = std::getenv(name);
    return (v && *v) ? std::strtod(v, nullptr) : dflt;
}

Layout default_layout(int n)
{
    // measured on MI355X: 8 points per lane with two systems per workgroup
    // beats 16 points (register spills) and 4 (per-lane overheads)
    int C = n > 8192 ? 16 : (n > 512 ? 8 : 4);
    const int fc = env_int("TDSE_LAYOUT_C", 0);  // experiment override
    if (fc == 4 || fc == 8 || fc == 12 || fc == 16) C = fc;  // 12: forward-only plans
    int T = ((n + C - 1) / C + kWave - 1) / kWave * kWave;
    if (T < kWave) T = kWave;
    return {C, T};
}

size_t class_bytes(const Layout& L)
{
    const size_t np = (size_t)L.C * L.T, T = L.T;
    size_t b = 0;
    auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
    for (int i = 0; i < 4; ++i) add(np * sizeof(double));
    for (int i = 0; i < 3; ++i) add(np * sizeof(cd));
    for (int i = 0; i < 2; ++i) add(kMaxLevels * T * sizeof(cd));
    for (int i = 0; i < 2; ++i) add(T * sizeof(cd));
    add(T * sizeof(int32_t));
    return b;
}

void carve_class(Arena& ar, SizeClass& sc)
{
    const size_t np = (size_t)sc.C * sc.T, T = sc.T;
    sc.pt.v = ar.take<double>(np);
    sc.pt.om = ar.take<double>(np);
    sc.pt.dv = ar.take<double>(np);
    sc.pt.m = ar.take<double>(np);
    sc.pt.q = ar.take<cd>(np);
    sc.pt.alpha = ar.take<cd>(np);
    sc.pt.beta = ar.take<cd>(np);
    sc.lt.pa = ar.take<cd>(kMaxLevels * T);
    sc.lt.qb = ar.take<cd>(kMaxLevels * T);
    sc.lt.pw = ar.take<cd>(T);
    sc.lt.qw = ar.take<cd>(T);
    sc.lt.hasmask = ar.take<int32_t>(T);
}

// Device memory of the set-up helpers: from hipMalloc (base == nullptr), or
// carved from a fixed region that the caller owns (the allocation-free
// ground state's static workspace), 256-byte aligned.
struct DevMem {
    char* base = nullptr;
    size_t size = 0, used = 0;
    bool heap() const { return base == nullptr; }
    hipError_t take(void** p, size_t bytes)
    {
        if (heap()) return hipMalloc(p, bytes);
        const size_t b = (bytes + 255) & ~size_t(255);
        if (used + b > size) return hipErrorOutOfMemory;
        *p = base + used;
        used += b;
        return hipSuccess;
    }
    void give(void* p)
    {
        if (heap() && p) (void)hipFree(p);
    }
};

// A set of size classes with their device tables.
struct ClassSet {
    std::vector<SizeClass> h;
    SizeClass* d = nullptr;
    char* mem = nullptr;
    bool owned = true;  // d and mem came from hipMalloc

    void release()
    {
        if (owned) {
            if (d) (void)hipFree(d);
            if (mem) (void)hipFree(mem);
        }
        d = nullptr;
        mem = nullptr;
        h.clear();
    }
};

// Builds tables for every entry of `params`/`layouts` and picks the scan
// depth of each class from the measured decay of the carry products.
tdse_status build_classes(ClassSet& cs, const std::vector<int>& ns,
                          const std::vector<Layout>& layouts, const std::vector<TableParams>& params,
                          hipStream_t st, DevMem* dm = nullptr)
{
    DevMem heap;
    DevMem& m = dm ? *dm : heap;
    cs.owned = m.heap();
    const int ncls = (int)ns.size();
    cs.h.assign(ncls, SizeClass{});
    size_t total = 0;
    int max_t = 0;
    for (int c = 0; c < ncls; ++c) {
        total += class_bytes(layouts[c]);
        max_t = std::max(max_t, layouts[c].T);
    }
    const size_t scratch_bytes = (size_t)ncls * 2 * max_t * sizeof(cd);
    const size_t metric_bytes = (size_t)ncls * 2 * (kMaxLevels + 1) * sizeof(double);
    const size_t param_bytes = (size_t)ncls * sizeof(TableParams);
    HIP_TRY(m.take(reinterpret_cast<void**>(&cs.mem), total + 3 * 256));
    Arena ar{cs.mem, total, 0};
    for (int c = 0; c < ncls; ++c) {
        SizeClass& sc = cs.h[c];
        sc.n = ns[c];
        sc.C = layouts[c].C;
        sc.T = layouts[c].T;
        sc.levels = kMaxLevels;
        sc.xwaves = sc.T / kWave;
        sc.dx = params[c].dx;
        const double habs =
            std::sqrt(params[c].h.re * params[c].h.re + params[c].h.im * params[c].h.im);
        sc.dofs10 = 7.2 * habs / (params[c].dx * params[c].dx);
        carve_class(ar, sc);
    }
    HIP_TRY(m.take(reinterpret_cast<void**>(&cs.d), sizeof(SizeClass) * ncls));
    char* tmp = nullptr;
    HIP_TRY(m.take(reinterpret_cast<void**>(&tmp), scratch_bytes + metric_bytes + param_bytes + 3 * 256));
    cd* d_scratch = reinterpret_cast<cd*>(tmp);
    double* d_metrics = reinterpret_cast<double*>(tmp + ((scratch_bytes + 255) & ~size_t(255)));
    TableParams* d_params = reinterpret_cast<TableParams*>(
        tmp + ((scratch_bytes + 255) & ~size_t(255)) + ((metric_bytes + 255) & ~size_t(255)));
    tdse_status rc = TDSE_OK;
    std::vector<double> metrics((size_t)ncls * 2 * (kMaxLevels + 1));
    do {
        if (hipMemcpyAsync(cs.d, cs.h.data(), sizeof(SizeClass) * ncls, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(d_params, params.data(), param_bytes, hipMemcpyHostToDevice, st) !=
                hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "copy of table parameters failed");
            break;
        }
        if (launch_build_tables(cs.d, d_params, ncls, d_metrics, d_scratch, max_t, st) !=
            hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "table kernel launch failed");
            break;
        }
        if (hipMemcpyAsync(metrics.data(), d_metrics, metric_bytes, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "table kernel failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        for (int c = 0; c < ncls; ++c) {
            SizeClass& sc = cs.h[c];
            const double* mA = &metrics[(size_t)(c * 2 + 0) * (kMaxLevels + 1)];
            const double* mB = &metrics[(size_t)(c * 2 + 1) * (kMaxLevels + 1)];
            int lev = -1;
            for (int l = 0; l <= kMaxLevels; ++l) {
                if (mA[l] < kTruncEps && mB[l] < kTruncEps) {
                    lev = l;
                    break;
                }
            }
            if (lev >= 0 && lev <= kMaxLevels) {
                sc.levels = std::min(lev, kMaxLevels);
                sc.xwaves = 1;
            } else {
                sc.levels = kMaxLevels;  // exact scan: every carry kept
                sc.xwaves = sc.T / kWave;
            }
            if (!std::isfinite(mA[0]) || !std::isfinite(mB[0])) {
                rc = fail(TDSE_E_NONFINITE, "non-finite factorisation for n=%d", sc.n);
                break;
            }
        }
        if (rc != TDSE_OK) break;
        if (hipMemcpyAsync(cs.d, cs.h.data(), sizeof(SizeClass) * ncls, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(TDSE_E_DEVICE, "copy of size classes failed");
    } while (0);
    m.give(tmp);
    return rc;
}

TableParams real_time_params(const tdse_params* p)
{
    TableParams t;
    t.dx = p->dx;
    t.a = p->a;
    t.z = p->charge_z;
    t.mask_frac = p->mask_fraction;
    t.mask_pow = p->mask_power;
    t.h = cd{0.0, 0.5 * p->dt};
    return t;
}

TableParams imag_time_params(double dx, double a, double z, double dtau)
{
    TableParams t;
    t.dx = dx;
    t.a = a;
    t.z = z;
    t.mask_frac = 0.0;
    t.mask_pow = 1.0;
    t.h = cd{0.5 * dtau, 0.0};
    return t;
}

// Runs the ground-state kernel for candidates that all share one layout.
tdse_status run_ground_states(const ClassSet& cs, const std::vector<int>& cls_of, double dtau,
                              int max_iter, double tol, double* d_psi, const int64_t* h_psi_off,
                              std::vector<double>& energy, std::vector<int>& iters, hipStream_t st,
                              DevMem* dm = nullptr)
{
    DevMem heap;
    DevMem& m = dm ? *dm : heap;
    const int nc = (int)cls_of.size();
    char* tmp = nullptr;
    const size_t b_cls = ((sizeof(int32_t) * nc + 255) & ~size_t(255));
    const size_t b_off = ((sizeof(int64_t) * nc + 255) & ~size_t(255));
    const size_t b_e = ((sizeof(double) * nc + 255) & ~size_t(255));
    HIP_TRY(m.take(reinterpret_cast<void**>(&tmp), b_cls + b_off + b_e + sizeof(int32_t) * nc));
    int32_t* d_cls = reinterpret_cast<int32_t*>(tmp);
    int64_t* d_off = reinterpret_cast<int64_t*>(tmp + b_cls);
    double* d_e = reinterpret_cast<double*>(tmp + b_cls + b_off);
    int32_t* d_it = reinterpret_cast<int32_t*>(tmp + b_cls + b_off + b_e);
    tdse_status rc = TDSE_OK;
    std::vector<int32_t> c32(cls_of.begin(), cls_of.end());
    energy.assign(nc, 0.0);
    iters.assign(nc, 0);
    std::vector<int32_t> it32(nc);
    do {
        if (hipMemcpyAsync(d_cls, c32.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(d_off, h_psi_off, sizeof(int64_t) * nc, hipMemcpyHostToDevice, st) !=
                hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "ground-state argument copy failed");
            break;
        }
        GsArgs g{};
        g.classes = cs.d;
        g.cls_of = d_cls;
        g.ncand = nc;
        g.dtau = dtau;
        g.max_iter = max_iter;
        g.tol = tol;
        g.psi_out = d_psi;
        g.psi_off = d_off;
        g.energy = d_e;
        g.iters = d_it;
        const SizeClass& s0 = cs.h[cls_of[0]];
        if (launch_ground_state(s0.C, g, s0.T, st) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "ground-state launch failed");
            break;
        }
        if (hipMemcpyAsync(energy.data(), d_e, sizeof(double) * nc, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(it32.data(), d_it, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "ground-state kernel failed: %s",
                      hipGetErrorString(hipGetLastError()));
            break;
        }
        for (int i = 0; i < nc; ++i) iters[i] = it32[i];
    } while (0);
    m.give(tmp);
    return rc;
}

// Device bytes build_classes and run_ground_states take for one ground state
// of layout L (each piece rounded to 256 bytes as DevMem::take does).
size_t ground_state_device_bytes(const Layout& L)
{
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t scratch_bytes = 2 * (size_t)L.T * sizeof(cd);
    const size_t metric_bytes = 2 * (kMaxLevels + 1) * sizeof(double);
    return r(class_bytes(L) + 3 * 256) + r(sizeof(SizeClass)) +
           r(scratch_bytes + metric_bytes + sizeof(TableParams) + 3 * 256) +
           r(3 * 256 + sizeof(int32_t));
}

tdse_status check_params(const tdse_params* p, bool need_time)
{
    if (!p) return fail(TDSE_E_INVALID, "params is NULL");
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(TDSE_E_INVALID, "dx must be > 0");
    if (need_time && (!(p->dt > 0.0) || !std::isfinite(p->dt)))
        return fail(TDSE_E_INVALID, "dt must be > 0");
    if (!std::isfinite(p->a) || (p->charge_z != 0.0 && !(p->a > 0.0)))
        return fail(TDSE_E_INVALID, "soft-core a must be > 0");
    if (!std::isfinite(p->charge_z)) return fail(TDSE_E_INVALID, "charge_z must be finite");
    if (need_time && (!(p->mask_fraction >= 0.0) || p->mask_fraction >= 0.5))
        return fail(TDSE_E_INVALID, "mask_fraction must be in [0, 0.5)");
    if (need_time && p->mask_fraction > 0.0 && !(p->mask_power > 0.0))
        return fail(TDSE_E_INVALID, "mask_power must be > 0");
    if (need_time && p->nt < 0) return fail(TDSE_E_INVALID, "nt must be >= 0");
    if (p->flags != 0) return fail(TDSE_E_INVALID, "flags must be 0");
    return TDSE_OK;
}

}  // namespace

// ==================================================================== plan
// ==================================================================== plan
// One launch of the persistent kernels: the systems of one size class.
struct Launch {
    int cls;
    int C, T, S;          // points per lane, lanes per system, systems per workgroup
    int tab;              // table placement of the forward launch (kTab*)
    int count, grid;
    double tuned_rate = 0.0;  // autotuner probe rate (0: default layout)
    int32_t* d_order;     // the class's systems
    // adjoint
    int aS = 1, agrid = 0;
    bool alds = false;
    int64_t slot_doubles = 0;
    int64_t work_off = 0;  // doubles into the adjoint workspace
    int32_t* d_order_adj = nullptr;
};

struct tdse_plan_s {
    tdse_params p{};
    int batch = 0;
    uint32_t options = 0;
    int adjoint_k = 0;
    std::vector<int> n_per;
    std::vector<int64_t> psi_off;
    std::vector<int> cls_of;            // per system
    ClassSet cls;                       // real-time tables, one class per distinct n
    std::map<int, int> cls_of_n;
    std::vector<double> gs_energy;      // per class
    std::vector<int64_t> gs_off;        // per class
    double* d_gs = nullptr;
    int64_t* d_gs_off = nullptr;
    SysDesc* d_sys = nullptr;
    std::vector<Launch> launches;       // one per class, longest work first
    std::vector<int> launch_of_cls;
    int32_t* d_order_all = nullptr;     // 2*batch: forward order, adjoint order
    int32_t* d_counters = nullptr;      // adjoint: launches + 2*launches (compaction); then one
                                        // kQueueInts queue per system (plain) and per forward group
    int32_t* d_ident = nullptr;
    // electron energy distribution: the sizes in system order, their blocks
    // of 64 systems and the length of the point-interleaved right-hand sides
    SpecClass* d_spec = nullptr;
    int spec_n = 0, spec_blocks = 0;
    int64_t spec_rhs = 0;
    // graph replay; graph_state: 0 not captured yet, 1 replaying a graph,
    // 2 capture failed (or was switched off) and calls launch directly
    int graph_state = 0;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev;
    hipGraphExec_t gexec = nullptr;
    std::vector<const void*> gkey;
    // adjoint workspace
    double* d_adj = nullptr;
    size_t adj_bytes = 0;
    // stored checkpoints (TDSE_OPT_STORE_CHECKPOINTS): per system
    double* d_store = nullptr;
    int64_t* d_store_off = nullptr;
    size_t store_bytes = 0;
    uint64_t ckpt_gen = 0;  // bumped by every call that rewrites the store
    // forward: one persistent launch per lane layout over workgroup bins
    struct FwdGroup {
        int C = 0;
        int tab = kTabLds;
        int threads = 0;  // workgroup size = bin capacity in lanes
        size_t smem = 0;  // LDS bytes per workgroup
        int nbins = 0, grid = 0;
        BinDesc* d_bins = nullptr;
        double est = 0.0;   // estimated time of the group run alone (any unit)
        bool fills = true;  // its grid takes every workgroup slot of the GPU
        int branch = 0;     // graph branch stream the group is launched on
    };
    std::vector<FwdGroup> fgroups;
    std::vector<int> fgroup_launch_order;  // small grids, then by decreasing time per bin
    std::vector<int> fgroup_of_cls;
    BinDesc* d_bins = nullptr;             // every group's bins, then one bin per system (plain)
    std::vector<int> plain_threads;        // per system
    std::vector<size_t> plain_smem;
    int ncls_real = 0;                     // classes [0, ncls_real) are real, the rest padding
    int ctr_plain = 0, ctr_fwd = 0;        // offsets into d_counters
    // elimination factors from their tables in the forward / adjoint
    // launches of layouts without q in registers (FwdArgs::ab)
    bool fwd_ab = true, adj_ab = true;
};

namespace {

void plan_free(tdse_plan pl)
{
    if (!pl) return;
    if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
    for (auto e : pl->ev) (void)hipEventDestroy(e);
    for (auto s : pl->branch) (void)hipStreamDestroy(s);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    pl->cls.release();
    if (pl->d_gs) (void)hipFree(pl->d_gs);
    if (pl->d_gs_off) (void)hipFree(pl->d_gs_off);
    if (pl->d_sys) (void)hipFree(pl->d_sys);
    if (pl->d_order_all) (void)hipFree(pl->d_order_all);
    if (pl->d_counters) (void)hipFree(pl->d_counters);
    if (pl->d_ident) (void)hipFree(pl->d_ident);
    if (pl->d_spec) (void)hipFree(pl->d_spec);
    if (pl->d_adj) (void)hipFree(pl->d_adj);
    if (pl->d_store) (void)hipFree(pl->d_store);
    if (pl->d_store_off) (void)hipFree(pl->d_store_off);
    if (pl->d_bins) (void)hipFree(pl->d_bins);
    delete pl;
}

// LDS bytes of a forward workgroup holding S systems of one class.
size_t fwd_smem(int C, int T, int S, int tab)
{
    return (size_t)tab_lds_bytes(tab) * C * T + S * sub_smem_bytes(T / kWave) + 16;
}
int fwd_occupancy(int C, int T, int S, int tab)
{
    if (!forward_tab_supported(C, tab)) return 0;
    return forward_occupancy(C, S * T, fwd_smem(C, T, S, tab), tab);
}

// Table placements in order of preference: both tables in LDS, om alone in
// LDS (forward kernel only), both in global memory.
constexpr int kTabOrder[3] = {kTabLds, kTabOmLds, kTabGlobal};

// Systems per workgroup and table placement for a class: as many systems as
// fit in 1024 lanes whose registers and LDS fit one workgroup per CU, point
// tables in LDS whenever they fit.  Returns false if nothing fits.
bool choose_packing(int C, int T, int count, bool adjoint, int* S_out, int* tab_out, int* occ_out,
                    bool stored = false)
{
    int smax = std::max(1, std::min(1024 / T, count));
    // the adjoint prefers workgroups of at most 512 threads, whose instances
    // have twice the registers (TDSE_ADJ_WIDE=1: up to 1024, experiments)
    if (adjoint && T <= 512 && !env_int("TDSE_ADJ_WIDE", 0)) smax = std::max(1, std::min(512 / T, count));
    const int fs = env_int("TDSE_PACK_S", 0);          // experiment overrides
    const int fl = env_int("TDSE_PACK_LDS", -1);
    if (fs > 0) smax = std::min(smax, fs);
    for (int tab : kTabOrder) {
        if (fl >= 0 && tab != fl) continue;
        if (adjoint ? tab == kTabOmLds : !forward_tab_supported(C, tab)) continue;
        const bool lds = tab == kTabLds;
        for (int S = smax; S >= 1; --S) {
            const size_t sh = adjoint ? adjoint_smem_bytes(C, T, S, lds) : fwd_smem(C, T, S, tab);
            if (sh > (size_t)kMaxLds) continue;
            const int occ = adjoint ? adjoint_occupancy(C, T, S, lds, stored) : fwd_occupancy(C, T, S, tab);
            if (occ >= 1) {
                *S_out = S;
                *tab_out = tab;
                *occ_out = occ;
                return true;
            }
        }
    }
    return false;
}

// ------------------------------------------------------------ workgroup bins
// The forward kernel takes one bin per queue item: systems of one lane layout
// packed into the lanes of a workgroup (first fit decreasing in lanes, within
// the LDS budget).  Lanes no system needs go to padding subgroups of padding
// classes, each no wider than the bin's widest system: a padding subgroup
// stages no tables of its own but reads (and discards the results of) the
// staged tables of that widest system's class, which are long enough.
struct PackItem {
    int p, cls, T;
};

struct HostBin {
    std::vector<PackItem> subs;
    std::vector<int> classes;  // distinct classes, in order of appearance
    int lanes = 0;
    int tmax = 0;              // widest subgroup (lanes)
    size_t tab_bytes = 0, sub_bytes = 0;
};

// Lane counts of the padding subgroups of a bin of `cap` lanes.
std::vector<int> pad_chunks(const HostBin& b, int cap)
{
    std::vector<int> out;
    for (int idle = cap - b.lanes; idle > 0;) {
        const int t = std::min(idle, b.tmax);
        out.push_back(t);
        idle -= t;
    }
    return out;
}

// LDS bytes of a bin (staged tables of its classes, the scratch blocks of all
// subgroups, the queue slot) and its subgroup count, padding included.
size_t bin_total(const HostBin& b, int cap, int* nsub)
{
    size_t bytes = b.tab_bytes + b.sub_bytes + 16;
    const std::vector<int> pad = pad_chunks(b, cap);
    for (int t : pad) bytes += sub_smem_bytes(t / kWave);
    *nsub = (int)(b.subs.size() + pad.size());
    return bytes;
}

bool bin_try_add(HostBin& b, const PackItem& it, int cap, int C, int tab)
{
    if (b.lanes + it.T > cap) return false;
    HostBin t = b;
    t.subs.push_back(it);
    t.lanes += it.T;
    t.tmax = std::max(t.tmax, it.T);
    if (std::find(t.classes.begin(), t.classes.end(), it.cls) == t.classes.end()) {
        t.classes.push_back(it.cls);
        t.tab_bytes += (size_t)tab_lds_bytes(tab) * C * it.T;
    }
    t.sub_bytes += sub_smem_bytes(it.T / kWave);
    int nsub = 0;
    if (bin_total(t, cap, &nsub) > (size_t)kMaxLds || nsub > kMaxSubs) return false;
    b = std::move(t);
    return true;
}

// Packs items into bins of `cap` lanes; fails if an item alone does not fit.
bool pack_bins(std::vector<PackItem> items, int cap, int C, int tab, std::vector<HostBin>& bins)
{
    std::stable_sort(items.begin(), items.end(),
                     [](const PackItem& x, const PackItem& y) { return x.T > y.T; });
    bins.clear();
    size_t first_open = 0;  // bins before this one are full
    for (const PackItem& it : items) {
        bool placed = false;
        for (size_t i = first_open; i < bins.size() && !placed; ++i) placed = bin_try_add(bins[i], it, cap, C, tab);
        if (!placed) {
            bins.emplace_back();
            if (!bin_try_add(bins.back(), it, cap, C, tab)) return false;
        }
        while (first_open < bins.size() && bins[first_open].lanes == cap) ++first_open;
    }
    return true;
}

// Device descriptor of a bin.  pad_cls(lanes) gives the padding class of a
// padding subgroup.  Returns the LDS bytes the bin uses (queue slot included).
template <class PadCls>
size_t make_bin_desc(const HostBin& b, int cap, int C, int tab, const std::vector<SizeClass>& cls,
                     PadCls pad_cls, BinDesc* d)
{
    std::memset(d, 0, sizeof(BinDesc));
    size_t off = 0;
    const bool lds = tab != kTabGlobal;
    std::vector<size_t> toff(b.classes.size(), 0);
    size_t wide_tab = 0;  // tables of the widest class, read by padding subgroups
    int wide_T = 0;
    if (lds)
        for (size_t k = 0; k < b.classes.size(); ++k) {
            toff[k] = off;
            const int T = cls[b.classes[k]].T;
            if (T > wide_T) {
                wide_T = T;
                wide_tab = off;
            }
            off += (size_t)tab_lds_bytes(tab) * C * T;
        }
    int wave = 0, j = 0;
    std::vector<int> staged;
    auto add = [&](int p, int c, int T, size_t toff, bool stage) {
        BinSub& u = d->sub[j];
        u.p = p;
        u.cls = c;
        u.wave0 = wave;
        u.tab_off = (int32_t)toff;
        u.sub_off = (int32_t)off;
        u.stage = stage ? 1 : 0;
        off += sub_smem_bytes(T / kWave);
        for (int w = 0; w < T / kWave; ++w) d->sub_of_wave[wave + w] = j;
        wave += T / kWave;
        ++j;
    };
    for (const PackItem& it : b.subs) {
        const size_t k = std::find(b.classes.begin(), b.classes.end(), it.cls) - b.classes.begin();
        const bool first = std::find(staged.begin(), staged.end(), it.cls) == staged.end();
        if (first) staged.push_back(it.cls);
        add(it.p, it.cls, it.T, lds ? toff[k] : 0, lds && first);
    }
    for (int t : pad_chunks(b, cap)) add(-1, pad_cls(t), t, wide_tab, false);
    d->nsub = j;
    return off + 16;
}

// ------------------------------------------------------------ autotuner
// For one grid size, times the forward kernel over the candidate lane
// layouts -- points per lane C (the length of the lane-local Thomas chunks
// against the width of the cross-lane scan), systems per workgroup S, and
// point tables in LDS or in global memory -- on a probe batch that fills the
// GPU once, and keeps the fastest.  Results are cached per process.
struct TuneChoice {
    int C = 0, T = 0, S = 1;
    int tab = kTabLds;
    double rate = 0.0;  // grid-point-steps per second of the probe
};

using TuneKey = std::tuple<int, int, double, double, double, double, double, double>;
std::map<TuneKey, TuneChoice> g_tune_cache;
std::mutex g_tune_mutex;
std::string g_tune_file;        // on-disk cache (tdse_set_tune_cache), "" = none
bool g_tune_file_set = false;   // false: TDSE_TUNE_CACHE names the file

Layout layout_for(int n, int C)
{
    int T = ((n + C - 1) / C + kWave - 1) / kWave * kWave;
    if (T < kWave) T = kWave;
    return {C, T};
}

// ---- on-disk autotune cache -------------------------------------------
// One text line per choice:
//   tdse-tune 1 <arch> <n> <count> <dx> <dt> <a> <z> <mask_frac> <mask_pow> : <C> <T> <S> <tab> <rate> # <fnv>
// with the doubles as hexadecimal floats (exact) and <fnv> the FNV-1a hash
// of everything before " # ".  A line that does not parse, fails its hash,
// belongs to another device architecture or names a layout that does not
// fit is ignored: the size is probed again and the file rewritten.

uint64_t fnv1a(const std::string& t)
{
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : t) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string tune_file()
{
    if (g_tune_file_set) return g_tune_file;
    const char* v = std::getenv("TDSE_TUNE_CACHE");
    return (v && *v) ? std::string(v) : std::string();
}

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    for (char& c : a)
        if (c == ' ' || c == '#' || c == ':') c = '_';
    return a;
}

std::string tune_key_text(const std::string& arch, const TuneKey& k)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf), "tdse-tune 1 %s %d %d %a %a %a %a %a %a", arch.c_str(),
                  std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                  std::get<5>(k), std::get<6>(k), std::get<7>(k));
    return buf;
}

int fwd_occupancy(int C, int T, int S, int tab);

// A cached choice is used only if it is a layout the plan could have picked.
bool choice_fits(int n, bool adjoint, bool shared, const TuneChoice& c)
{
    if (!layout_supported(c.C) || (adjoint && c.C == 12)) return false;
    const Layout L = layout_for(n, c.C);
    if (L.T != c.T || L.T > 1024 || c.S < 1 || c.S * c.T > 1024) return false;
    if (shared && forward_narrow(c.C, c.S * c.T)) return false;
    if (!forward_tab_supported(c.C, c.tab)) return false;
    if (!(c.rate > 0.0) || !std::isfinite(c.rate)) return false;
    return fwd_occupancy(c.C, c.T, c.S, c.tab) >= 1;
}

// Reads the file's lines: valid ones into `lines` (key text -> full line),
// returns the number of lines that were not valid.
int read_tune_file(const std::string& path, std::map<std::string, std::string>& lines)
{
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return 0;
    int bad = 0;
    char buf[1024];
    while (std::fgets(buf, sizeof(buf), f)) {
        std::string line(buf);
        while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
        if (line.empty()) continue;
        const size_t h = line.rfind(" # ");
        const size_t c = line.find(" : ");
        unsigned long long fnv = 0;
        if (h == std::string::npos || c == std::string::npos || c > h ||
            std::sscanf(line.c_str() + h + 3, "%llx", &fnv) != 1 ||
            fnv1a(line.substr(0, h)) != (uint64_t)fnv) {
            ++bad;
            continue;
        }
        lines[line.substr(0, c)] = line;
    }
    std::fclose(f);
    return bad;
}

bool parse_choice(const std::string& line, TuneChoice* out)
{
    const size_t c = line.find(" : ");
    if (c == std::string::npos) return false;
    TuneChoice t;
    char tail[8] = {0};
    if (std::sscanf(line.c_str() + c + 3, "%d %d %d %d %la %1s", &t.C, &t.T, &t.S, &t.tab, &t.rate,
                    tail) != 6 || tail[0] != '#')
        return false;
    *out = t;
    return true;
}

// The cached choice for `key`, if the file holds a valid one.
bool tune_file_lookup(const TuneKey& key, int n, bool adjoint, bool shared, TuneChoice* out)
{
    const std::string path = tune_file();
    if (path.empty()) return false;
    std::map<std::string, std::string> lines;
    read_tune_file(path, lines);
    auto it = lines.find(tune_key_text(device_arch(), key));
    if (it == lines.end()) return false;
    TuneChoice c;
    if (!parse_choice(it->second, &c) || !choice_fits(n, adjoint, shared, c)) return false;
    *out = c;
    return true;
}

// Adds (or replaces) the choice for `key`, dropping invalid lines; the file
// is written whole and renamed into place, so readers never see half of it.
void tune_file_store(const TuneKey& key, const TuneChoice& c)
{
    const std::string path = tune_file();
    if (path.empty()) return;
    std::map<std::string, std::string> lines;
    read_tune_file(path, lines);
    const std::string k = tune_key_text(device_arch(), key);
    char buf[256];
    std::snprintf(buf, sizeof(buf), " : %d %d %d %d %a", c.C, c.T, c.S, c.tab, c.rate);
    const std::string body = k + buf;
    char h[32];
    std::snprintf(h, sizeof(h), " # %016llx", (unsigned long long)fnv1a(body));
    lines[k] = body + h;
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;  // a cache that cannot be written only costs the next probe
    bool ok = true;
    for (const auto& kv : lines) ok = ok && std::fprintf(f, "%s\n", kv.second.c_str()) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

constexpr int kProbeSteps = 128;

// Rate of one candidate (0 when it does not fit).  Probe inputs are zero:
// the kernel's instruction stream does not depend on the values.  The probe
// batch fills every workgroup slot once with bins of S systems.
tdse_status probe_forward(const tdse_params* p, int n, const Layout& L, int S, int tab, int count,
                          hipStream_t st, double* rate)
{
    *rate = 0.0;
    if (!forward_tab_supported(L.C, tab)) return TDSE_OK;
    const size_t smem = fwd_smem(L.C, L.T, S, tab);
    const int occ = forward_occupancy(L.C, S * L.T, smem, tab);
    if (occ < 1 || smem > (size_t)kMaxLds || count < S) return TDSE_OK;
    const int nb = std::max(1, std::min(count / S, occ * num_cus()));
    const int P = nb * S;
    const int ps = env_int("TDSE_PROBE_STEPS", 0);  // experiment override
    const int nt = ps > 0 ? ps : kProbeSteps;
    ClassSet cs;
    tdse_status rc = build_classes(cs, {n}, {L}, {real_time_params(p)}, st);
    if (rc != TDSE_OK) {
        cs.release();
        return rc;
    }
    const size_t b_e = ((sizeof(double) * (size_t)P * (nt + 1) + 255) & ~size_t(255));
    const size_t b_psi = ((sizeof(double) * 2 * (size_t)P * n + 255) & ~size_t(255));
    const size_t b_sys = ((sizeof(SysDesc) * (size_t)P + 255) & ~size_t(255));
    const size_t b_bin = ((sizeof(BinDesc) * (size_t)nb + 255) & ~size_t(255));
    char* mem = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if (hipMalloc(&mem, 2 * b_e + b_psi + b_sys + b_bin + 256) != hipSuccess) {
            rc = fail(TDSE_E_NOMEM, "autotune probe allocation failed");
            break;
        }
        double* E = reinterpret_cast<double*>(mem);
        double* acc = reinterpret_cast<double*>(mem + b_e);
        double* psi = reinterpret_cast<double*>(mem + 2 * b_e);
        SysDesc* sys = reinterpret_cast<SysDesc*>(mem + 2 * b_e + b_psi);
        BinDesc* bins = reinterpret_cast<BinDesc*>(mem + 2 * b_e + b_psi + b_sys);
        int32_t* ctr = reinterpret_cast<int32_t*>(mem + 2 * b_e + b_psi + b_sys + b_bin);
        std::vector<SysDesc> hs(P);
        for (int i = 0; i < P; ++i) {
            hs[i].cls = 0;
            hs[i].n = n;
            hs[i].psi_off = (int64_t)i * n;
        }
        std::vector<BinDesc> hb(nb);
        size_t used = 0;
        bool packed = true;
        for (int k = 0; k < nb && packed; ++k) {
            HostBin hbin;
            for (int i = 0; i < S && packed; ++i)
                packed = bin_try_add(hbin, PackItem{k * S + i, 0, L.T}, S * L.T, L.C, tab);
            used = std::max(used, make_bin_desc(hbin, S * L.T, L.C, tab, cs.h, [](int) { return 0; }, &hb[k]));
        }
        if (!packed) {
            rc = fail(TDSE_E_UNSUPPORTED, "autotune probe: %d systems of n=%d do not fit a workgroup", S, n);
            break;
        }
        if (used > smem) {
            rc = fail(TDSE_E_UNSUPPORTED, "autotune probe bins need %zu B of LDS, %zu planned", used, smem);
            break;
        }
        if (hipMemsetAsync(mem, 0, 2 * b_e + b_psi, st) != hipSuccess ||
            hipMemcpyAsync(sys, hs.data(), sizeof(SysDesc) * P, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(bins, hb.data(), sizeof(BinDesc) * nb, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "autotune probe setup failed");
            break;
        }
        // one queue: every bin in the first run
        int32_t qb[kQueueInts] = {};
        for (int x = 1; x <= kXcds; ++x) qb[kXcds + x] = nb;
        if (hipMemcpy(ctr, qb, sizeof(qb), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "autotune probe setup failed");
            break;
        }
        FwdArgs a{};
        a.ab = 1;  // one size: its tables fit the L2
        a.classes = cs.d;
        a.sys = sys;
        a.bins = bins;
        a.nbins = nb;
        a.item_off = (int32_t)(smem - 16);
        a.queue = ctr;
        a.nt = nt;
        a.dt = p->dt;
        a.E = E;
        a.psi0 = psi;
        a.accel = acc;
        const int grid = std::min(nb, occ * num_cus());
        float best_ms = 0.0f;
        for (int rep = 0; rep < 3 && rc == TDSE_OK; ++rep) {  // warm-up, then best of two
            float ms = 0.0f;
            if (launch_reset_queues(ctr, 1, st) != hipSuccess ||
                hipEventRecord(e0, st) != hipSuccess ||
                launch_forward(L.C, tab, a, S * L.T, smem, grid, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = fail(TDSE_E_DEVICE, "autotune probe launch failed: %s",
                          hipGetErrorString(hipGetLastError()));
            else if (rep > 0 && ms > 0.0f && (best_ms == 0.0f || ms < best_ms))
                best_ms = ms;
        }
        if (rc == TDSE_OK && best_ms > 0.0f) *rate = (double)P * n * nt / (best_ms * 1e-3);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (mem) (void)hipFree(mem);
    cs.release();
    return rc;
}

// Rate of the adjoint kernel (forward pass, checkpointed recompute and
// reverse sweep over kProbeSteps steps, checkpoints every 16 steps) for one
// layout, with its default packing; 0 when it does not fit.
// stored: time the reverse sweep alone from per-system checkpoints (the
// path of plans that store them; the forward kernel writes the
// checkpoints), else the adjoint call that recomputes them.
tdse_status probe_adjoint(const tdse_params* p, int n, const Layout& L, int count, bool stored,
                          hipStream_t st, double* rate)
{
    *rate = 0.0;
    int S = 1, occ = 0, tab = kTabGlobal;
    if (!choose_packing(L.C, L.T, count, true, &S, &tab, &occ, stored)) return TDSE_OK;
    const bool lds = tab == kTabLds;
    const int P = std::max(1, std::min(count, S * occ * num_cus()));
    const int nt = kProbeSteps, K = 16;
    const int grid = std::min((P + S - 1) / S, occ * num_cus());
    const int64_t rec = 2 * (int64_t)(L.C + 2) * L.T;
    const int64_t ck = rec * (nt / K + 1) + ((nt + 2) & ~int64_t(1));  // checkpoints + norm row
    // the two-chain reverse sweep (narrow, up to 8 points) keeps two segment buffers
    const int nbuf = (stored && adjoint_narrow(S * L.T) && L.C <= 8) ? 2 : 1;
    const int64_t slot = (stored ? rec : rec + ck) + nbuf * 2 * (int64_t)L.C * L.T * (K + 1);
    const size_t b_store = stored ? sizeof(double) * (size_t)ck * P : 0;
    const size_t b_soff = stored ? ((sizeof(int64_t) * (size_t)P + 255) & ~size_t(255)) : 0;
    ClassSet cs;
    tdse_status rc = build_classes(cs, {n}, {L}, {real_time_params(p)}, st);
    if (rc != TDSE_OK) {
        cs.release();
        return rc;
    }
    const size_t b_e = ((sizeof(double) * (size_t)P * (nt + 1) + 255) & ~size_t(255));
    const size_t b_psi = ((sizeof(double) * 2 * (size_t)P * n + 255) & ~size_t(255));
    const size_t b_sys = ((sizeof(SysDesc) * (size_t)P + 255) & ~size_t(255));
    const size_t b_ord = ((sizeof(int32_t) * (size_t)P + 255) & ~size_t(255));
    const size_t b_work = sizeof(double) * (size_t)slot * grid * S;
    char* mem = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if (hipMalloc(&mem, 3 * b_e + b_psi + b_sys + b_ord + 256 + b_work + b_soff + b_store) !=
            hipSuccess) {
            rc = fail(TDSE_E_NOMEM, "autotune probe allocation failed");
            break;
        }
        double* E = reinterpret_cast<double*>(mem);
        double* abar = reinterpret_cast<double*>(mem + b_e);
        double* grad = reinterpret_cast<double*>(mem + 2 * b_e);
        double* psi = reinterpret_cast<double*>(mem + 3 * b_e);
        SysDesc* sys = reinterpret_cast<SysDesc*>(mem + 3 * b_e + b_psi);
        int32_t* ord = reinterpret_cast<int32_t*>(mem + 3 * b_e + b_psi + b_sys);
        int32_t* ctr = reinterpret_cast<int32_t*>(mem + 3 * b_e + b_psi + b_sys + b_ord);
        double* work = reinterpret_cast<double*>(mem + 3 * b_e + b_psi + b_sys + b_ord + 256);
        std::vector<SysDesc> hs(P);
        std::vector<int32_t> ho(P);
        std::vector<double> ha((size_t)P * (nt + 1), 1e-3);  // every row takes the reverse sweep
        for (int i = 0; i < P; ++i) {
            hs[i].cls = 0;
            hs[i].n = n;
            hs[i].psi_off = (int64_t)i * n;
            ho[i] = i;
        }
        if (hipMemsetAsync(E, 0, b_e, st) != hipSuccess ||
            hipMemsetAsync(psi, 0, b_psi, st) != hipSuccess ||
            hipMemcpyAsync(abar, ha.data(), sizeof(double) * ha.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(sys, hs.data(), sizeof(SysDesc) * P, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(ord, ho.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(TDSE_E_DEVICE, "autotune probe setup failed");
            break;
        }
        FwdArgs a{};
        a.ab = 1;  // one size: its tables fit the L2
        a.classes = cs.d;
        a.sys = sys;
        a.order = ord;
        a.count = P;
        a.cls = 0;
        a.queue = ctr;
        a.nt = nt;
        a.sub_bytes = (int64_t)sub_smem_bytes(L.T / kWave);
        a.dt = p->dt;
        a.E = E;
        a.psi0 = psi;
        a.abar = abar;
        a.grad = grad;
        a.work = work;
        a.slot_doubles = slot;
        a.k_ckpt = K;
        if (stored) {
            // zero checkpoints: the kernel's work does not depend on the values
            int64_t* soff = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(work) + b_work);
            double* store = reinterpret_cast<double*>(reinterpret_cast<char*>(soff) + b_soff);
            std::vector<int64_t> ho_off(P);
            for (int i = 0; i < P; ++i) ho_off[i] = (int64_t)i * ck;
            if (hipMemcpyAsync(soff, ho_off.data(), sizeof(int64_t) * P, hipMemcpyHostToDevice, st) !=
                    hipSuccess ||
                hipMemsetAsync(store, 0, b_store, st) != hipSuccess) {
                rc = fail(TDSE_E_DEVICE, "autotune probe setup failed");
                break;
            }
            a.store = store;
            a.store_off = soff;
            a.mode = kAdjReverseOnly;
        }
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && rc == TDSE_OK; ++rep) {  // warm-up, then timed
            if (launch_reset_counters(ctr, 1, st) != hipSuccess ||
                (rep == 1 && hipEventRecord(e0, st) != hipSuccess) ||
                launch_adjoint(L.C, lds, a, L.T, S, grid, st) != hipSuccess ||
                (rep == 1 && hipEventRecord(e1, st) != hipSuccess) ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = fail(TDSE_E_DEVICE, "autotune adjoint probe failed: %s",
                          hipGetErrorString(hipGetLastError()));
        }
        if (rc == TDSE_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f)
            *rate = (double)P * n * nt / (ms * 1e-3);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (mem) (void)hipFree(mem);
    cs.release();
    return rc;
}

// For plans with the adjoint the score is the time of one forward and one
// adjoint pass per grid-point-step, with the adjoint's own default packing.
// shared: the plan holds several sizes, whose classes share 1024-lane
// workgroups (one persistent launch per lane layout); only candidates that
// run the wide instances are probed there.  Narrow packings are kept by
// single-size plans only: in a plan of several sizes a narrow choice for
// some of them split the forward pass into launches of both instance
// families, which measured 15 % slower than one family on the uneven
// workload although the per-size probes favoured the mix.
tdse_status autotune(const tdse_params* p, int n, int count, bool adjoint, bool stored,
                     bool shared, hipStream_t st, TuneChoice* out)
{
    // the count field of the key also says which adjoint path the plan takes
    // and whether its classes share workgroups
    int kc = adjoint ? (stored ? -(count + (1 << 29)) : -count) : count;
    if (shared) kc = kc >= 0 ? kc + (1 << 28) : kc - (1 << 28);
    const TuneKey key{n, kc, p->dx, p->dt, p->a, p->charge_z, p->mask_fraction, p->mask_power};
    {
        std::lock_guard<std::mutex> g(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return TDSE_OK;
        }
        TuneChoice c;
        if (tune_file_lookup(key, n, adjoint, shared, &c)) {
            g_tune_cache[key] = c;
            *out = c;
            return TDSE_OK;
        }
    }
    TuneChoice best;
    double best_cost = 0.0;  // seconds per grid-point-step (forward [+ adjoint])
    int best_waves = 0;      // wavefronts the best candidate keeps resident per CU
    for (int C : {4, 8, 12, 16}) {
        const Layout L = layout_for(n, C);
        if (L.T > 1024 || !layout_supported(C)) continue;
        if (adjoint && C == 12) continue;  // the adjoint kernel has no 12-point layout
        double adj_cost = 0.0;
        if (adjoint) {
            double ra = 0.0;
            tdse_status rc = probe_adjoint(p, n, L, count, stored, st, &ra);
            if (rc != TDSE_OK) return rc;
            if (env_int("TDSE_TUNE_LOG", 0))
                std::fprintf(stderr, "[tdse autotune] n=%d C=%d T=%d adjoint (%s): %.4e grid-point-steps/s\n",
                             n, C, L.T, stored ? "reverse from stored checkpoints" : "recomputing",
                             ra);
            if (ra <= 0.0) continue;
            adj_cost = 1.0 / ra;
        }
        const int smax = std::max(1, std::min(1024 / L.T, count));
        for (int tab : kTabOrder) {
            if (!forward_tab_supported(C, tab)) continue;
            // the two widest packings that fit, and the widest one of the
            // narrow instances (at most 512 threads) when they differ
            std::vector<int> cand;
            for (int S = smax; S >= 1 && cand.size() < 2; --S)
                if (fwd_occupancy(C, L.T, S, tab) >= 1 && !(shared && forward_narrow(C, S * L.T)))
                    cand.push_back(S);
            const int sn = std::min(512 / L.T, count);
            if (!shared && sn >= 1 && forward_narrow(C, sn * L.T) &&
                std::find(cand.begin(), cand.end(), sn) == cand.end() &&
                fwd_occupancy(C, L.T, sn, tab) >= 1)
                cand.push_back(sn);
            for (int S : cand) {
                double r = 0.0;
                tdse_status rc = probe_forward(p, n, L, S, tab, count, st, &r);
                if (rc != TDSE_OK) return rc;
                if (env_int("TDSE_TUNE_LOG", 0))
                    std::fprintf(stderr, "[tdse autotune] n=%d C=%d T=%d S=%d tab=%d: %.4e grid-point-steps/s\n",
                                 n, C, L.T, S, tab, r);
                if (r <= 0.0) continue;
                // narrow instances (2 waves per SIMD) come out of the short
                // probe up to 5 % better than over whole runs (focus workload:
                // +5 % in the probe, -4 % over the run): they must win by 6 %
                const double cost = (forward_narrow(C, S * L.T) ? 1.06 : 1.0) / r + adj_cost;
                // fewer systems per workgroup (tried after more) must win by
                // more than the probe's noise: over whole runs the wider
                // workgroup, which shares its staged tables, was 1.5 % faster
                // on the focus workload, while its 128-step probes came out
                // up to 1.5 % either way
                const bool narrower = best_cost > 0.0 && C == best.C && tab == best.tab && S < best.S;
                // candidates within 2 % of each other are a tie, which goes
                // to the one keeping more wavefronts resident per CU: at
                // N = 12288 the 12-point layout (16 wavefronts) and the
                // 16-point one (12) probe within 1-2 % of each other either
                // way round, while over whole runs the first is 4 % faster
                const int waves = fwd_occupancy(C, L.T, S, tab) * S * L.T / kWave;
                bool take;
                if (best_cost == 0.0)
                    take = true;
                else if (waves != best_waves && std::fabs(cost - best_cost) < 0.02 * best_cost)
                    take = waves > best_waves;
                else
                    take = cost < best_cost * (narrower ? 0.97 : 1.0);
                if (take) {
                    best_cost = cost;
                    best_waves = waves;
                    best = TuneChoice{C, L.T, S, tab, r};
                }
            }
        }
    }
    if (best_cost <= 0.0) return fail(TDSE_E_UNSUPPORTED, "no lane layout fits n=%d", n);
    std::lock_guard<std::mutex> g(g_tune_mutex);
    g_tune_cache[key] = best;
    tune_file_store(key, best);
    *out = best;
    return TDSE_OK;
}

constexpr double kGsDtau = 0.5;
constexpr double kGsTol = 1e-13;
constexpr int kGsMaxIter = 100000;

// Ground states of every class of a plan (imaginary-time tables built on the
// side with the plan's a and charge, mask off).
tdse_status plan_ground_states(tdse_plan pl, hipStream_t st)
{
    const int ncls = pl->ncls_real;  // padding classes need no ground state
    std::vector<int> ns(ncls);
    std::vector<Layout> lay(ncls);
    std::vector<TableParams> prm(ncls);
    pl->gs_off.assign(ncls + 1, 0);
    for (int c = 0; c < ncls; ++c) {
        ns[c] = pl->cls.h[c].n;
        lay[c] = {pl->cls.h[c].C, pl->cls.h[c].T};
        prm[c] = imag_time_params(pl->p.dx, pl->p.a, pl->p.charge_z, kGsDtau);
        pl->gs_off[c + 1] = pl->gs_off[c] + ns[c];
    }
    HIP_TRY(hipMalloc(&pl->d_gs, sizeof(double) * 2 * (size_t)pl->gs_off[ncls]));
    HIP_TRY(hipMalloc(&pl->d_gs_off, sizeof(int64_t) * (ncls + 1)));
    HIP_TRY(hipMemcpy(pl->d_gs_off, pl->gs_off.data(), sizeof(int64_t) * (ncls + 1),
                      hipMemcpyHostToDevice));
    ClassSet im;
    tdse_status rc = build_classes(im, ns, lay, prm, st);
    pl->gs_energy.assign(ncls, 0.0);
    if (rc == TDSE_OK) {
        // one launch per distinct layout (the kernel is specialised on C)
        for (int c = 0; c < ncls && rc == TDSE_OK; ++c) {
            std::vector<int> one{c};
            std::vector<double> e;
            std::vector<int> it;
            rc = run_ground_states(im, one, kGsDtau, kGsMaxIter, kGsTol, pl->d_gs,
                                   &pl->gs_off[c], e, it, st);
            if (rc == TDSE_OK && it[0] <= 0)
                rc = fail(TDSE_E_NOCONV, "ground state for n=%d did not converge", ns[c]);
            if (rc == TDSE_OK) pl->gs_energy[c] = e[0];
        }
    }
    im.release();
    return rc;
}

}  // namespace

extern "C" {

const char* tdse_version(void) { return "libtdse 0.3.0 (gfx950, fp64)"; }

tdse_status tdse_set_tune_cache(const char* path)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> g(g_tune_mutex);
    g_tune_cache.clear();
    g_tune_file_set = true;
    g_tune_file = path ? std::string(path) : std::string();
    return TDSE_OK;
}

const char* tdse_status_string(tdse_status s)
{
    switch (s) {
        case TDSE_OK: return "ok";
        case TDSE_E_INVALID: return "invalid argument";
        case TDSE_E_NOMEM: return "out of memory";
        case TDSE_E_DEVICE: return "device error";
        case TDSE_E_NOCONV: return "not converged";
        case TDSE_E_UNSUPPORTED: return "unsupported";
        case TDSE_E_NONFINITE: return "non-finite value";
        default: return "unknown status";
    }
}

const char* tdse_last_error(void) { return g_last_error.c_str(); }

tdse_status tdse_plan_create(const tdse_params* p, int32_t batch, const int32_t* n_per_system,
                             uint32_t options, int32_t adjoint_k, tdse_plan* out)
{
    g_last_error.clear();
    if (!out) return fail(TDSE_E_INVALID, "out is NULL");
    *out = nullptr;
    tdse_status st = check_params(p, true);
    if (st != TDSE_OK) return st;
    if (batch < 1) return fail(TDSE_E_INVALID, "batch must be >= 1");
    if (!n_per_system) return fail(TDSE_E_INVALID, "n_per_system is NULL");
    if (options & ~(TDSE_OPT_PLAIN | TDSE_OPT_NO_GRAPH | TDSE_OPT_AUTOTUNE | TDSE_OPT_STORE_CHECKPOINTS))
        return fail(TDSE_E_INVALID, "unknown option bits 0x%x", options);
    if (adjoint_k < 0) return fail(TDSE_E_INVALID, "adjoint_k must be >= 0");
    if ((options & TDSE_OPT_STORE_CHECKPOINTS) && (adjoint_k == 0 || (options & TDSE_OPT_PLAIN)))
        return fail(TDSE_E_INVALID, "TDSE_OPT_STORE_CHECKPOINTS needs adjoint_k > 0 and no TDSE_OPT_PLAIN");
    for (int b = 0; b < batch; ++b) {
        if (n_per_system[b] < kMinN) return fail(TDSE_E_INVALID, "n[%d] = %d < %d", b, n_per_system[b], kMinN);
        if (n_per_system[b] > kMaxN)
            return fail(TDSE_E_UNSUPPORTED, "n[%d] = %d exceeds %d", b, n_per_system[b], kMaxN);
    }
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(TDSE_E_UNSUPPORTED, "device arch %s is not gfx950", prop.gcnArchName);

    tdse_plan pl = new tdse_plan_s();
    pl->p = *p;
    pl->batch = batch;
    pl->options = options;
    pl->adjoint_k = adjoint_k;
    pl->n_per.assign(n_per_system, n_per_system + batch);
    pl->psi_off.assign(batch + 1, 0);
    for (int b = 0; b < batch; ++b) pl->psi_off[b + 1] = pl->psi_off[b] + pl->n_per[b];

    auto bail = [&](tdse_status rc) {
        plan_free(pl);
        return rc;
    };
    if (hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(TDSE_E_DEVICE, "stream creation failed"));
    hipStream_t s0 = pl->cap;

    // size classes, one per distinct n
    std::vector<int> ns;
    for (int b = 0; b < batch; ++b) {
        if (!pl->cls_of_n.count(pl->n_per[b])) {
            pl->cls_of_n[pl->n_per[b]] = (int)ns.size();
            ns.push_back(pl->n_per[b]);
        }
    }
    const int ncls = (int)ns.size();
    std::vector<Layout> lay(ncls);
    std::vector<TableParams> prm(ncls, real_time_params(p));
    std::vector<int> ccount(ncls, 0);
    for (int b = 0; b < batch; ++b) ++ccount[pl->cls_of_n[pl->n_per[b]]];
    const bool tune = (options & TDSE_OPT_AUTOTUNE) && !(options & TDSE_OPT_PLAIN);
    if (adjoint_k > 0 && !tune && env_int("TDSE_LAYOUT_C", 0) == 12)
        return bail(fail(TDSE_E_UNSUPPORTED,
                         "TDSE_LAYOUT_C=12 is a forward-only layout: the adjoint kernel has "
                         "4, 8 and 16 points per lane (create the plan with adjoint_k = 0)"));
    std::vector<TuneChoice> tuned(ncls);
    for (int c = 0; c < ncls; ++c) {
        if (tune) {
            st = autotune(p, ns[c], ccount[c], adjoint_k > 0,
                          (options & TDSE_OPT_STORE_CHECKPOINTS) != 0, ncls > 1, s0, &tuned[c]);
            if (st != TDSE_OK) return bail(st);
            lay[c] = {tuned[c].C, tuned[c].T};
        } else {
            lay[c] = default_layout(ns[c]);
        }
        if (lay[c].T > 1024 || !layout_supported(lay[c].C))
            return bail(fail(TDSE_E_UNSUPPORTED, "no lane layout for n=%d", ns[c]));
    }
    // systems of each class
    pl->ncls_real = ncls;
    pl->cls_of.resize(batch);
    std::vector<SysDesc> sys(batch);
    std::vector<std::vector<int32_t>> csys(ncls);
    for (int b = 0; b < batch; ++b) {
        const int c = pl->cls_of_n[pl->n_per[b]];
        pl->cls_of[b] = c;
        sys[b].cls = c;
        sys[b].n = pl->n_per[b];
        sys[b].psi_off = pl->psi_off[b];
        csys[c].push_back(b);
    }

    // forward packing of each class: systems per workgroup, table placement
    std::vector<int> cS(ncls, 1);
    std::vector<int> ctab(ncls, kTabLds);
    for (int c = 0; c < ncls; ++c) {
        if (tune) {
            cS[c] = tuned[c].S;
            ctab[c] = tuned[c].tab;
        } else {
            int S = 1, occ = 0, tb = kTabLds;
            if (!choose_packing(lay[c].C, lay[c].T, ccount[c], false, &S, &tb, &occ))
                return bail(fail(TDSE_E_UNSUPPORTED, "layout C=%d T=%d does not fit", lay[c].C, lay[c].T));
            cS[c] = S;
            ctab[c] = tb;
        }
    }
    // one persistent forward launch per (C, table placement): a single class
    // keeps its own packing, several classes share 1024-lane workgroups
    std::map<std::pair<int, int>, std::vector<int>> gcls;
    for (int c = 0; c < ncls; ++c) gcls[{lay[c].C, ctab[c]}].push_back(c);
    struct GroupBins {
        int C;
        int tab;
        int cap;
        std::vector<HostBin> bins;
    };
    std::vector<GroupBins> gbins;
    std::map<std::pair<int, int>, int> pad_cls;  // (C, lanes) -> padding class
    pl->fgroup_of_cls.assign(ncls, -1);
    auto add_group = [&](const std::vector<int>& classes, int C, int tab, int cap) -> bool {
        GroupBins g;
        g.C = C;
        g.tab = tab;
        g.cap = cap;
        std::vector<PackItem> items;
        for (int c : classes)
            for (int32_t b : csys[c]) items.push_back(PackItem{b, c, lay[c].T});
        if (!pack_bins(items, g.cap, g.C, g.tab, g.bins)) return false;
        for (int c : classes) pl->fgroup_of_cls[c] = (int)gbins.size();
        for (const HostBin& hb : g.bins)
            for (int t : pad_chunks(hb, g.cap)) pad_cls[{g.C, t}] = 0;
        gbins.push_back(std::move(g));
        return true;
    };
    for (const auto& kv : gcls) {
        const int C = kv.first.first;
        const int tab = kv.first.second;
        // several classes share full workgroups when their staged tables and a
        // padding subgroup fit the LDS; otherwise each class keeps its own
        bool ok = kv.second.size() > 1 && add_group(kv.second, C, tab, 1024);
        if (!ok)
            for (int c : kv.second)
                if (!add_group({c}, C, tab, cS[c] * lay[c].T))
                    return bail(fail(TDSE_E_UNSUPPORTED, "systems of n=%d do not fit a workgroup", ns[c]));
    }
    // padding classes (16 points, the needed lane counts) after the real ones
    std::vector<int> ns_all = ns;
    std::vector<Layout> lay_all = lay;
    std::vector<TableParams> prm_all = prm;
    for (auto& kv : pad_cls) {
        kv.second = (int)ns_all.size();
        ns_all.push_back(kMinN);
        lay_all.push_back(Layout{kv.first.first, kv.first.second});
        prm_all.push_back(real_time_params(p));
    }
    st = build_classes(pl->cls, ns_all, lay_all, prm_all, s0);
    if (st != TDSE_OK) return bail(st);
    st = plan_ground_states(pl, s0);
    if (st != TDSE_OK) return bail(st);

    // bin descriptors: each group's bins, then one bin per system (plain form)
    std::vector<BinDesc> hbins;
    std::vector<size_t> goff;
    for (const GroupBins& g : gbins) {
        tdse_plan_s::FwdGroup fg;
        fg.C = g.C;
        fg.tab = g.tab;
        fg.threads = g.cap;
        fg.nbins = (int)g.bins.size();
        goff.push_back(hbins.size());
        for (const HostBin& hb : g.bins) {
            hbins.emplace_back();
            const size_t used = make_bin_desc(hb, g.cap, g.C, g.tab, pl->cls.h,
                                              [&](int t) { return pad_cls[{g.C, t}]; },
                                              &hbins.back());
            fg.smem = std::max(fg.smem, used);
        }
        const int occ = forward_occupancy(fg.C, fg.threads, fg.smem, fg.tab);
        if (occ < 1)
            return bail(fail(TDSE_E_UNSUPPORTED, "forward workgroup of %d lanes with %zu B of LDS does not fit",
                             fg.threads, fg.smem));
        fg.grid = std::min(fg.nbins, occ * num_cus());
        fg.fills = fg.nbins >= occ * num_cus();
        pl->fgroups.push_back(fg);
    }
    // each group's time alone: its grid points over the rate its classes
    // reached when tuned (grid-point-steps per second), else its grid points
    for (int c = 0; c < ncls; ++c) {
        const double rate = (tune && tuned[c].rate > 0.0) ? tuned[c].rate : 1.0;
        pl->fgroups[pl->fgroup_of_cls[c]].est += (double)ccount[c] * (double)ns[c] / rate;
    }
    pl->plain_threads.assign(batch, 0);
    pl->plain_smem.assign(batch, 0);
    for (int b = 0; b < batch; ++b) {
        const int c = pl->cls_of[b];
        HostBin hb;
        if (!bin_try_add(hb, PackItem{b, c, lay[c].T}, lay[c].T, lay[c].C, ctab[c]))
            return bail(fail(TDSE_E_UNSUPPORTED, "system %d does not fit a workgroup", b));
        hbins.emplace_back();
        pl->plain_smem[b] = make_bin_desc(hb, lay[c].T, lay[c].C, ctab[c], pl->cls.h,
                                          [](int) { return 0; }, &hbins.back());
        pl->plain_threads[b] = lay[c].T;
    }
    if (hipMalloc(&pl->d_bins, sizeof(BinDesc) * hbins.size()) != hipSuccess)
        return bail(fail(TDSE_E_NOMEM, "plan allocation failed"));
    for (size_t g = 0; g < pl->fgroups.size(); ++g) pl->fgroups[g].d_bins = pl->d_bins + goff[g];
    if (hipMemcpy(pl->d_bins, hbins.data(), sizeof(BinDesc) * hbins.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return bail(fail(TDSE_E_DEVICE, "plan upload failed"));
    // Per-XCD queues: each group's bins (ordered by lane count, so the
    // systems of one grid size are contiguous) are cut into kXcds contiguous
    // runs, one per XCD; a workgroup takes bins from the run of the XCD it
    // runs on first, so in a group of several sizes each L2 holds the tables
    // of about 1/kXcds of them.  Every bin of a group fills the same
    // workgroup (padding included), so the runs hold equal numbers of bins.
    std::vector<int32_t> xq;  // per group: kXcds + 1 run bounds
    for (size_t g = 0; g < pl->fgroups.size(); ++g) {
        const int64_t nb = pl->fgroups[g].nbins;
        for (int x = 0; x <= kXcds; ++x) xq.push_back((int32_t)(nb * x / kXcds));
    }
    {
        // Layouts without q in registers read alpha and beta from their
        // tables (no FMAs; three tables per point in the L2 instead of one).
        // Measured faster than forming them from q and om for every
        // workload here, the 57-size uneven batch included once its bins are
        // spread by XCD; TDSE_AB_TABLES=0 forms them from q (experiments).
        pl->fwd_ab = pl->adj_ab = env_int("TDSE_AB_TABLES", 1) != 0;
    }

    // adjoint launches, one per class, longest work first: classes by
    // (n_pad * count) descending
    std::vector<int> corder(ncls);
    for (int c = 0; c < ncls; ++c) corder[c] = c;
    std::stable_sort(corder.begin(), corder.end(), [&](int x, int y) {
        const double wx = (double)lay[x].C * lay[x].T * csys[x].size();
        const double wy = (double)lay[y].C * lay[y].T * csys[y].size();
        return wx > wy;
    });
    const int nl = ncls;
    const int ng = (int)pl->fgroups.size();
    pl->ctr_plain = 3 * nl;
    pl->ctr_fwd = 3 * nl + kQueueInts * batch;
    if (hipMalloc(&pl->d_sys, sizeof(SysDesc) * batch) != hipSuccess ||
        hipMalloc(&pl->d_order_all, sizeof(int32_t) * 2 * batch) != hipSuccess ||
        hipMalloc(&pl->d_counters, sizeof(int32_t) * (3 * nl + kQueueInts * (batch + ng))) != hipSuccess ||
        hipMalloc(&pl->d_ident, sizeof(int32_t) * batch) != hipSuccess)
        return bail(fail(TDSE_E_NOMEM, "plan allocation failed"));
    {
        // run bounds of the queues (the counters are reset by every launch):
        // a plain launch's one bin sits in the first run
        std::vector<int32_t> qs((size_t)kQueueInts * (batch + ng), 0);
        for (int b = 0; b < batch; ++b)
            for (int x = 1; x <= kXcds; ++x) qs[(size_t)kQueueInts * b + kXcds + x] = 1;
        for (int g = 0; g < ng; ++g)
            for (int x = 0; x <= kXcds; ++x)
                qs[(size_t)kQueueInts * (batch + g) + kXcds + x] = xq[(size_t)(kXcds + 1) * g + x];
        if (hipMemcpy(pl->d_counters + pl->ctr_plain, qs.data(), sizeof(int32_t) * qs.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(TDSE_E_DEVICE, "plan upload failed"));
    }
    std::vector<int32_t> order_all;
    std::vector<SpecClass> spec;
    pl->launch_of_cls.assign(ncls, -1);
    const int64_t nt = p->nt;
    int64_t adj_total = 0;
    const bool store = (options & TDSE_OPT_STORE_CHECKPOINTS) != 0;
    std::vector<int64_t> store_off(batch, 0);
    int64_t store_total = 0;
    for (int c : corder) {
        Launch L{};
        L.cls = c;
        L.C = lay[c].C;
        L.T = lay[c].T;
        L.count = (int)csys[c].size();
        L.d_order = pl->d_order_all + order_all.size();
        L.d_order_adj = pl->d_order_all + batch + order_all.size();
        {
            SpecClass sp{};
            sp.cls = c;
            sp.n = pl->n_per[csys[c][0]];
            sp.start = (int32_t)order_all.size();
            sp.count = L.count;
            sp.blk0 = pl->spec_blocks;
            sp.rhs_off = pl->spec_rhs;
            pl->spec_blocks += (L.count + kWave - 1) / kWave;
            pl->spec_rhs += (int64_t)sp.n * L.count;
            spec.push_back(sp);
        }
        order_all.insert(order_all.end(), csys[c].begin(), csys[c].end());
        const tdse_plan_s::FwdGroup& fg = pl->fgroups[pl->fgroup_of_cls[c]];
        L.S = std::max(1, fg.threads / L.T);
        L.tab = fg.tab;
        L.grid = fg.grid;
        if (tune) L.tuned_rate = tuned[c].rate;
        if (adjoint_k > 0) {
            int aocc = 0;
            int atab = kTabGlobal;
            if (!choose_packing(L.C, L.T, L.count, true, &L.aS, &atab, &aocc, store))
                return bail(fail(TDSE_E_UNSUPPORTED, "adjoint layout C=%d T=%d does not fit", L.C, L.T));
            L.alds = atab == kTabLds;
            L.agrid = std::min((L.count + L.aS - 1) / L.aS, aocc * num_cus());
            const int64_t rec = 2 * (int64_t)(L.C + 2) * L.T;   // one state record
            const int64_t recs = 2 * (int64_t)L.C * L.T;        // one segment record
            const int64_t nseg = nt / adjoint_k + 1;
            const int64_t ck = rec * nseg + ((nt + 2) & ~int64_t(1));  // checkpoints + norm row
            // a slot holds the segment states and one parked costate record, and
            // the checkpoints unless they are stored per system
            // the two-chain reverse sweep (narrow, up to 8 points per lane)
            // keeps a second segment buffer after the parked costate
            const int nbuf = (store && adjoint_narrow(L.aS * L.T) && L.C <= 8) ? 2 : 1;
            L.slot_doubles = nbuf * recs * (adjoint_k + 1) + rec + (store ? 0 : ck);
            L.work_off = adj_total;
            adj_total += L.slot_doubles * (int64_t)L.agrid * L.aS;
            if (store)
                for (int32_t b : csys[c]) {
                    store_off[b] = store_total;
                    store_total += ck;
                }
        }
        pl->launch_of_cls[c] = (int)pl->launches.size();
        pl->launches.push_back(L);
    }
    std::vector<int32_t> ident(batch);
    for (int b = 0; b < batch; ++b) ident[b] = b;
    pl->spec_n = (int)spec.size();
    if (hipMalloc(&pl->d_spec, sizeof(SpecClass) * spec.size()) != hipSuccess)
        return bail(fail(TDSE_E_NOMEM, "plan allocation failed"));
    if (hipMemcpy(pl->d_spec, spec.data(), sizeof(SpecClass) * spec.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return bail(fail(TDSE_E_DEVICE, "plan upload failed"));
    if (hipMemcpy(pl->d_sys, sys.data(), sizeof(SysDesc) * batch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->d_order_all, order_all.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(pl->d_ident, ident.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) !=
            hipSuccess)
        return bail(fail(TDSE_E_DEVICE, "plan upload failed"));

    // graph branches (forward groups run concurrently).  A persistent launch
    // whose grid takes every workgroup slot can hold its CUs until its queue
    // is empty: a small grid launched after it waited for them (the uneven
    // batch's 37-workgroup group, 11 % on the whole solve).  Launch order:
    // first the groups whose grids leave slots free, then the rest by
    // decreasing time per bin, so that the longest bins start first and the
    // last launch to end, which no other work can overlap, has the shortest.
    // Branches in launch order.
    const int nbr = std::min<int>(4, ng);
    {
        std::vector<int> order(ng);
        for (int g = 0; g < ng; ++g) order[g] = g;
        auto per_bin = [&](int g) { return pl->fgroups[g].est / std::max(1, pl->fgroups[g].nbins); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const bool fx = pl->fgroups[x].fills, fy = pl->fgroups[y].fills;
            if (fx != fy) return !fx;
            return per_bin(x) > per_bin(y);
        });
        for (int i = 0; i < ng; ++i) pl->fgroups[order[i]].branch = i % std::max(nbr, 1);
        pl->fgroup_launch_order = order;
    }
    for (int i = 0; i < nbr; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(TDSE_E_DEVICE, "stream creation failed"));
        pl->branch.push_back(s);
    }
    for (int i = 0; i < nbr + 1; ++i) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(TDSE_E_DEVICE, "event creation failed"));
        pl->ev.push_back(e);
    }

    if (adjoint_k > 0) {
        pl->adj_bytes = sizeof(double) * (size_t)adj_total;
        // an optional cap on the adjoint workspace and checkpoint store
        // (TDSE_MAX_WORKSPACE_BYTES): exceeding it fails like an allocation
        // the device cannot satisfy, before anything is allocated
        const double cap = env_double("TDSE_MAX_WORKSPACE_BYTES", 0.0);
        const double want = (double)pl->adj_bytes + (store ? sizeof(double) * (double)store_total : 0.0);
        if (cap > 0.0 && want > cap)
            return bail(fail(TDSE_E_NOMEM, "adjoint workspace and checkpoint store of %.0f bytes "
                                           "exceed TDSE_MAX_WORKSPACE_BYTES = %.0f", want, cap));
        if (hipMalloc(&pl->d_adj, pl->adj_bytes) != hipSuccess)
            return bail(fail(TDSE_E_NOMEM, "adjoint workspace of %.1f GB not available",
                             pl->adj_bytes / 1e9));
    }
    if (store) {
        pl->store_bytes = sizeof(double) * (size_t)store_total;
        if (hipMalloc(&pl->d_store, pl->store_bytes) != hipSuccess)
            return bail(fail(TDSE_E_NOMEM, "checkpoint store of %.1f GB not available",
                             pl->store_bytes / 1e9));
        if (hipMalloc(&pl->d_store_off, sizeof(int64_t) * batch) != hipSuccess ||
            hipMemcpy(pl->d_store_off, store_off.data(), sizeof(int64_t) * batch,
                      hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(TDSE_E_NOMEM, "checkpoint store offsets not available"));
    }
    *out = pl;
    return TDSE_OK;
}

tdse_status tdse_plan_destroy(tdse_plan plan)
{
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    (void)hipDeviceSynchronize();
    plan_free(plan);
    return TDSE_OK;
}

tdse_status tdse_plan_psi_offsets(tdse_plan plan, int64_t* offsets)
{
    if (!plan || !offsets) return fail(TDSE_E_INVALID, "NULL argument");
    std::memcpy(offsets, plan->psi_off.data(), sizeof(int64_t) * (plan->batch + 1));
    return TDSE_OK;
}

tdse_status tdse_plan_layout(tdse_plan plan, int32_t n, int32_t* points_per_lane, int32_t* lanes,
                             int32_t* scan_levels)
{
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    auto it = plan->cls_of_n.find(n);
    if (it == plan->cls_of_n.end()) return fail(TDSE_E_INVALID, "n=%d is not in the plan", n);
    const SizeClass& sc = plan->cls.h[it->second];
    if (points_per_lane) *points_per_lane = sc.C;
    if (lanes) *lanes = sc.T;
    if (scan_levels) *scan_levels = sc.xwaves > 1 ? -sc.levels : sc.levels;
    return TDSE_OK;
}

tdse_status tdse_plan_launch_info(tdse_plan plan, int32_t n, int32_t* systems_per_workgroup,
                                  int32_t* lds_tables, double* tuned_rate)
{
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    auto it = plan->cls_of_n.find(n);
    if (it == plan->cls_of_n.end()) return fail(TDSE_E_INVALID, "n=%d is not in the plan", n);
    const Launch& L = plan->launches[plan->launch_of_cls[it->second]];
    if (systems_per_workgroup) *systems_per_workgroup = L.S;
    if (lds_tables) *lds_tables = L.tab;
    if (tuned_rate) *tuned_rate = L.tuned_rate;
    return TDSE_OK;
}

tdse_status tdse_plan_kernel_info(tdse_plan plan, int32_t n, int32_t* workgroup_lanes,
                                  int32_t* grid, int32_t* workgroups_per_cu, int32_t* lds_bytes,
                                  int32_t* vgprs)
{
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    auto it = plan->cls_of_n.find(n);
    if (it == plan->cls_of_n.end()) return fail(TDSE_E_INVALID, "n=%d is not in the plan", n);
    const int gi = plan->fgroup_of_cls[it->second];
    if (gi < 0 || gi >= (int)plan->fgroups.size())
        return fail(TDSE_E_INVALID, "n=%d has no forward launch (plain plan)", n);
    const tdse_plan_s::FwdGroup& g = plan->fgroups[gi];
    const bool ab = g.C >= 12 && plan->fwd_ab;
    if (workgroup_lanes) *workgroup_lanes = g.threads;
    if (grid) *grid = g.grid;
    if (workgroups_per_cu) *workgroups_per_cu = forward_occupancy(g.C, g.threads, g.smem, g.tab);
    if (lds_bytes) *lds_bytes = (int32_t)g.smem;
    if (vgprs) *vgprs = forward_vgprs(g.C, g.tab, ab, g.threads);
    return TDSE_OK;
}

tdse_status tdse_plan_ground_state(tdse_plan plan, int32_t n, double* psi_out, double* energy_out)
{
    if (!plan || !psi_out) return fail(TDSE_E_INVALID, "NULL argument");
    auto it = plan->cls_of_n.find(n);
    if (it == plan->cls_of_n.end()) return fail(TDSE_E_INVALID, "n=%d is not in the plan", n);
    const int c = it->second;
    HIP_TRY(hipMemcpy(psi_out, plan->d_gs + 2 * plan->gs_off[c], sizeof(double) * 2 * n,
                      hipMemcpyDeviceToDevice));
    if (energy_out) *energy_out = plan->gs_energy[c];
    return TDSE_OK;
}

static void fill_fwd_args(tdse_plan pl, FwdArgs& a, const double* E, const double* psi0,
                          double* accel, double* xexp, double* norm, double* psi_final,
                          int32_t* sys_status)
{
    a = FwdArgs{};
    a.classes = pl->cls.d;
    a.sys = pl->d_sys;
    a.nt = pl->p.nt;
    a.dt = pl->p.dt;
    a.E = E;
    a.psi0 = psi0;
    a.gs = pl->d_gs;
    a.gs_off = pl->d_gs_off;
    a.accel = accel;
    a.xexp = xexp;
    a.norm = norm;
    a.psi_final = psi_final;
    a.status = sys_status;
}

static tdse_status enqueue_forward(tdse_plan pl, const FwdArgs& base, hipStream_t st, bool branches)
{
    const int ng = (int)pl->fgroups.size();
    int32_t* ctr = pl->d_counters + pl->ctr_fwd;
    if (launch_reset_queues(ctr, ng, st) != hipSuccess)
        return fail(TDSE_E_DEVICE, "counter reset launch failed");
    auto one = [&](int g, hipStream_t s) -> tdse_status {
        const tdse_plan_s::FwdGroup& G = pl->fgroups[g];
        FwdArgs a = base;
        a.bins = G.d_bins;
        a.nbins = G.nbins;
        a.item_off = (int32_t)(G.smem - 16);
        a.queue = ctr + kQueueInts * g;
        a.ab = pl->fwd_ab ? 1 : 0;
        if (launch_forward(G.C, G.tab, a, G.threads, G.smem, G.grid, s) != hipSuccess)
            return fail(TDSE_E_DEVICE, "forward launch failed: %s", hipGetErrorString(hipGetLastError()));
        return TDSE_OK;
    };
    if (!branches || pl->branch.size() <= 1) {
        for (int g = 0; g < ng; ++g) {
            tdse_status rc = one(g, st);
            if (rc != TDSE_OK) return rc;
        }
        return TDSE_OK;
    }
    // fork the groups over the branch streams (captured as parallel graph branches)
    const int nb = (int)pl->branch.size();
    HIP_TRY(hipEventRecord(pl->ev[0], st));
    for (int b = 0; b < nb; ++b) HIP_TRY(hipStreamWaitEvent(pl->branch[b], pl->ev[0], 0));
    for (int g : pl->fgroup_launch_order) {
        tdse_status rc = one(g, pl->branch[pl->fgroups[g].branch % nb]);
        if (rc != TDSE_OK) return rc;
    }
    for (int b = 0; b < nb; ++b) {
        HIP_TRY(hipEventRecord(pl->ev[b + 1], pl->branch[b]));
        HIP_TRY(hipStreamWaitEvent(st, pl->ev[b + 1], 0));
    }
    return TDSE_OK;
}

// One adjoint-kernel launch per size class.  With accel_bar, the class's
// systems are first reordered so that rows needing the reverse sweep come
// first; the forward-only mode keeps the class order.
static tdse_status enqueue_adjoint(tdse_plan plan, const FwdArgs& base, const double* accel_bar,
                                   int32_t mode, hipStream_t st)
{
    const int nl = (int)plan->launches.size();
    if (launch_reset_counters(plan->d_counters, 3 * nl, st) != hipSuccess)
        return fail(TDSE_E_DEVICE, "counter reset launch failed");
    for (int l = 0; l < nl; ++l) {
        const Launch& L = plan->launches[l];
        FwdArgs a = base;
        a.abar = accel_bar;
        a.k_ckpt = plan->adjoint_k;
        a.mode = mode;
        a.store = plan->d_store;
        a.store_off = plan->d_store_off;
        a.order = L.d_order;
        if (accel_bar) {
            if (launch_compact_rows(accel_bar, plan->p.nt, L.d_order, L.count, L.d_order_adj,
                                    plan->d_counters + nl + 2 * l, st) != hipSuccess)
                return fail(TDSE_E_DEVICE, "row compaction launch failed");
            a.order = L.d_order_adj;
        }
        a.count = L.count;
        a.cls = L.cls;
        a.queue = plan->d_counters + l;
        a.sub_bytes = (int64_t)sub_smem_bytes(L.T / kWave);
        a.work = plan->d_adj + L.work_off;
        a.slot_doubles = L.slot_doubles;
        a.ab = plan->adj_ab ? 1 : 0;
        if (launch_adjoint(L.C, L.alds, a, L.T, L.aS, L.agrid, st) != hipSuccess)
            return fail(TDSE_E_DEVICE, "adjoint launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    return TDSE_OK;
}

// One system per launch, serially on the caller's stream (TDSE_OPT_PLAIN).
static tdse_status enqueue_plain(tdse_plan plan, const FwdArgs& base, hipStream_t st)
{
    int32_t* ctr = plan->d_counters + plan->ctr_plain;
    if (launch_reset_queues(ctr, plan->batch, st) != hipSuccess)
        return fail(TDSE_E_DEVICE, "counter reset launch failed");
    const BinDesc* pb = plan->d_bins;
    size_t off = 0;
    for (const auto& G : plan->fgroups) off += G.nbins;
    for (int b = 0; b < plan->batch; ++b) {
        const Launch& L = plan->launches[plan->launch_of_cls[plan->cls_of[b]]];
        FwdArgs a = base;
        a.bins = pb + off + b;
        a.nbins = 1;
        a.item_off = (int32_t)(plan->plain_smem[b] - 16);
        a.queue = ctr + kQueueInts * b;
        a.ab = plan->fwd_ab ? 1 : 0;
        if (launch_forward(L.C, L.tab, a, plan->plain_threads[b], plan->plain_smem[b], 1, st) !=
            hipSuccess)
            return fail(TDSE_E_DEVICE, "forward launch failed");
    }
    return TDSE_OK;
}

tdse_status tdse_propagate_batch_populations(tdse_plan plan, const double* E, const double* psi0,
                                             double* accel, double* xexp, double* norm,
                                             double* psi_final, int32_t* sys_status,
                                             const double* psi_ref, double radius,
                                             double* gs_pop, double* vol_pop, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (!E || !accel) return fail(TDSE_E_INVALID, "E and accel are required");
    if (!gs_pop && !vol_pop) return fail(TDSE_E_INVALID, "gs_pop or vol_pop is required");
    if (!(radius >= 0.0)) return fail(TDSE_E_INVALID, "radius must be >= 0");
    const void* ptrs[] = {E, psi0, accel, xexp, norm, psi_final, sys_status, psi_ref, gs_pop, vol_pop};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    if (plan->d_store)
        return fail(TDSE_E_UNSUPPORTED, "a plan that stores checkpoints samples populations at its "
                                        "stored states (tdse_plan_populations)");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    FwdArgs base;
    fill_fwd_args(plan, base, E, psi0, accel, xexp, norm, psi_final, sys_status);
    base.pop_ref = psi_ref;
    base.gs_pop = gs_pop;
    base.vol_pop = vol_pop;
    base.pop_radius = radius;
    if (plan->options & TDSE_OPT_PLAIN) return enqueue_plain(plan, base, st);
    return enqueue_forward(plan, base, st, false);
}

tdse_status tdse_propagate_batch(tdse_plan plan, const double* E, const double* psi0,
                                 double* accel, double* xexp, double* norm, double* psi_final,
                                 int32_t* sys_status, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (!E || !accel) return fail(TDSE_E_INVALID, "E and accel are required");
    const void* ptrs[] = {E, psi0, accel, xexp, norm, psi_final, sys_status};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    FwdArgs base;
    fill_fwd_args(plan, base, E, psi0, accel, xexp, norm, psi_final, sys_status);

    if (plan->d_store) {
        // the forward kernel also writes the checkpoints and norm rows that a
        // later tdse_adjoint_batch_stored reads, in the adjoint's lane layout
        base.store = plan->d_store;
        base.store_off = plan->d_store_off;
        base.k_ckpt = plan->adjoint_k;
        ++plan->ckpt_gen;
    }
    if (plan->options & TDSE_OPT_PLAIN) return enqueue_plain(plan, base, st);
    if ((plan->options & TDSE_OPT_NO_GRAPH) || plan->graph_state == 2)
        return enqueue_forward(plan, base, st, false);

    std::vector<const void*> key{E, psi0, accel, xexp, norm, psi_final, sys_status};
    if (!plan->gexec || key != plan->gkey) {
        if (plan->gexec) {
            (void)hipGraphExecDestroy(plan->gexec);
            plan->gexec = nullptr;
        }
        // a capture that fails (or is switched off with
        // TDSE_FORCE_CAPTURE_FAILURE) leaves the plan on direct launches,
        // which run the same kernels with the same arguments
        const bool forced = env_int("TDSE_FORCE_CAPTURE_FAILURE", 0) != 0;
        hipGraph_t graph = nullptr;
        hipError_t ec = forced ? hipErrorNotSupported
                               : hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
        if (ec == hipSuccess) {
            tdse_status rc = enqueue_forward(plan, base, plan->cap, true);
            ec = hipStreamEndCapture(plan->cap, &graph);
            if (rc != TDSE_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec == hipSuccess) {
                ec = hipGraphInstantiate(&plan->gexec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ec != hipSuccess) plan->gexec = nullptr;
            }
        }
        if (ec != hipSuccess) {
            (void)hipGetLastError();  // the failed capture's error is not the caller's
            plan->graph_state = 2;
            return enqueue_forward(plan, base, st, false);
        }
        plan->graph_state = 1;
        plan->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(plan->gexec, st));
    return TDSE_OK;
}

tdse_status tdse_plan_graph_state(tdse_plan plan, int32_t* state)
{
    if (!plan || !state) return fail(TDSE_E_INVALID, "NULL argument");
    *state = plan->graph_state;
    return TDSE_OK;
}

// ------------------------------------------------------------ ground state
tdse_status tdse_ground_state(const tdse_params* p, int32_t n, double dtau, int32_t max_iter,
                              double tol, double* psi_out, double* energy_out, void* stream)
{
    g_last_error.clear();
    tdse_status st = check_params(p, false);
    if (st != TDSE_OK) return st;
    if (n < kMinN || n > kMaxN) return fail(n > kMaxN ? TDSE_E_UNSUPPORTED : TDSE_E_INVALID, "n=%d out of range", n);
    if (!(dtau > 0.0) || max_iter < 1 || !(tol > 0.0) || !psi_out)
        return fail(TDSE_E_INVALID, "dtau > 0, max_iter >= 1, tol > 0 and psi_out are required");
    if (!aligned16(psi_out)) return fail(TDSE_E_INVALID, "psi_out must be 16-byte aligned");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    ClassSet cs;
    std::vector<int> ns{n};
    std::vector<Layout> lay{default_layout(n)};
    std::vector<TableParams> prm{imag_time_params(p->dx, p->a, p->charge_z, dtau)};
    st = build_classes(cs, ns, lay, prm, hs);
    if (st == TDSE_OK) {
        std::vector<int> one{0};
        int64_t off = 0;
        std::vector<double> e;
        std::vector<int> it;
        st = run_ground_states(cs, one, dtau, max_iter, tol, psi_out, &off, e, it, hs);
        if (st == TDSE_OK) {
            if (energy_out) *energy_out = e[0];
            if (it[0] <= 0) st = fail(TDSE_E_NOCONV, "not converged after %d iterations", -it[0]);
            else if (!std::isfinite(e[0])) st = fail(TDSE_E_NONFINITE, "non-finite energy");
        }
    }
    cs.release();
    return st;
}

tdse_status tdse_resample_field(int32_t batch, int32_t m, double dt_coarse, double dt, int32_t nt,
                                const double* e_coarse, double* work, size_t work_bytes,
                                double* e_fine, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || batch > 65535) return fail(TDSE_E_INVALID, "batch must be in [1, 65535]");
    if (m < 2 || m > (1 << 20)) return fail(TDSE_E_INVALID, "m must be in [2, 2^20]");
    if (nt < 0) return fail(TDSE_E_INVALID, "nt must be >= 0");
    if (!(dt_coarse > 0.0) || !(dt > 0.0)) return fail(TDSE_E_INVALID, "dt_coarse and dt must be > 0");
    const double ratio = (double)m * dt_coarse / dt;
    const double mp = std::round(ratio);
    if (!(std::fabs(ratio - mp) <= 1e-9 * ratio) || mp > 2147483647.0)
        return fail(TDSE_E_INVALID, "m dt_coarse / dt = %.12g is not an integer (the padded length)", ratio);
    if (mp < (double)m || mp < (double)nt + 1.0)
        return fail(TDSE_E_INVALID, "the padded length %.0f is below max(m, nt+1) = %d", mp,
                    std::max(m, nt + 1));
    if (!e_coarse || !work || !e_fine) return fail(TDSE_E_INVALID, "e_coarse, work and e_fine are required");
    if (!aligned16(work) || (reinterpret_cast<uintptr_t>(e_coarse) & 7u) ||
        (reinterpret_cast<uintptr_t>(e_fine) & 7u))
        return fail(TDSE_E_INVALID, "work must be 16-byte aligned, e_coarse and e_fine 8-byte aligned");
    const size_t need = (size_t)16 * (size_t)batch * (size_t)(m / 2 + 1);
    if (work_bytes < need) return fail(TDSE_E_INVALID, "work holds %zu bytes, needs %zu", work_bytes, need);
    ResampleArgs a{};
    a.batch = batch;
    a.m = m;
    a.nt = nt;
    a.mp = (int64_t)mp;
    a.coarse = e_coarse;
    a.spec = work;
    a.fine = e_fine;
    if (launch_resample(a, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(TDSE_E_DEVICE, "resampling launch failed: %s", hipGetErrorString(hipGetLastError()));
    return TDSE_OK;
}

// ------------------------------------------------ allocation-free ground state
// A fixed device workspace for tdse_ground_state_noalloc: the tables of one
// size class and the ground-state kernel's outputs (about 1.6 MB at the
// largest grid, n = 16384).  Every GPU the library runs on holds its own
// copy of the array until the process ends.  In host code `scratch` only
// stands in for the symbol: its device address on the current GPU comes
// from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocScratchBytes = size_t(2) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                  // held for the whole call: calls on one
char* g_scratch_ptr[kMaxDevices] = {};    // GPU from threads of this process run
                                          // one after the other

// The device address of `scratch` on the current GPU (looked up on the first
// call on that GPU).  Called with g_scratch_mu held.
tdse_status scratch_of_current_device(char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TDSE_E_UNSUPPORTED, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TDSE_E_DEVICE, "hipGetSymbolAddress of the static workspace failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return TDSE_OK;
}

}  // namespace

tdse_status tdse_ground_state_noalloc(const tdse_params* p, int32_t n, double dtau,
                                      int32_t max_iter, double tol, double* psi_out,
                                      double* energy_out, void* stream)
{
    g_last_error.clear();
    tdse_status st = check_params(p, false);
    if (st != TDSE_OK) return st;
    if (n < kMinN || n > kMaxN) return fail(n > kMaxN ? TDSE_E_UNSUPPORTED : TDSE_E_INVALID, "n=%d out of range", n);
    if (!(dtau > 0.0) || max_iter < 1 || !(tol > 0.0) || !psi_out)
        return fail(TDSE_E_INVALID, "dtau > 0, max_iter >= 1, tol > 0 and psi_out are required");
    if (!aligned16(psi_out)) return fail(TDSE_E_INVALID, "psi_out must be 16-byte aligned");
    const Layout L = default_layout(n);
    const size_t need = ground_state_device_bytes(L);
    if (need > kNoAllocScratchBytes)
        return fail(TDSE_E_NOMEM, "n=%d needs %zu bytes of the static workspace, which holds %zu", n,
                    need, kNoAllocScratchBytes);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    char* base = nullptr;
    st = scratch_of_current_device(&base);
    if (st != TDSE_OK) return st;
    DevMem dm{base, kNoAllocScratchBytes, 0};
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    ClassSet cs;
    std::vector<int> ns{n};
    std::vector<Layout> lay{L};
    std::vector<TableParams> prm{imag_time_params(p->dx, p->a, p->charge_z, dtau)};
    st = build_classes(cs, ns, lay, prm, hs, &dm);
    if (st == TDSE_OK) {
        std::vector<int> one{0};
        int64_t off = 0;
        std::vector<double> e;
        std::vector<int> it;
        st = run_ground_states(cs, one, dtau, max_iter, tol, psi_out, &off, e, it, hs, &dm);
        if (st == TDSE_OK) {
            if (energy_out) *energy_out = e[0];
            if (it[0] <= 0) st = fail(TDSE_E_NOCONV, "not converged after %d iterations", -it[0]);
            else if (!std::isfinite(e[0])) st = fail(TDSE_E_NONFINITE, "non-finite energy");
        }
    }
    cs.release();  // nothing to free: the tables live in the static workspace
    // the stream has been synchronised (the energy was read back), so the
    // workspace is free for the next call
    return st;
}

tdse_status tdse_soft_core_for_ip(double ip, int32_t n, double dx, double dtau, double tol,
                                  double a_lo, double a_hi, double* a_out, double* e_out)
{
    g_last_error.clear();
    if (!(ip > 0.0) || !(dx > 0.0) || !(dtau > 0.0) || !(tol > 0.0) || !a_out)
        return fail(TDSE_E_INVALID, "ip, dx, dtau, tol > 0 and a_out are required");
    if (!(a_lo > 0.0) || !(a_hi > a_lo)) return fail(TDSE_E_INVALID, "need 0 < a_lo < a_hi");
    if (n < kMinN || n > kMaxN) return fail(TDSE_E_INVALID, "n=%d out of range", n);
    const int K = 31;  // candidates per pass (plus the two bracket ends in the first)
    const Layout L = default_layout(n);
    double* d_psi = nullptr;
    HIP_TRY(hipMalloc(&d_psi, sizeof(double) * 2 * (size_t)n * (K + 2)));
    tdse_status st = TDSE_OK;
    double lo = a_lo, hi = a_hi, best_a = 0.5 * (a_lo + a_hi), best_e = 0.0;
    bool first = true, done = false;
    for (int round = 0; round < 40 && st == TDSE_OK && !done; ++round) {
        std::vector<double> cand;
        if (first) {
            cand.push_back(lo);
            cand.push_back(hi);
        }
        for (int k = 1; k <= K; ++k) cand.push_back(lo + (hi - lo) * k / (K + 1));
        const int nc = (int)cand.size();
        std::vector<int> ns(nc, n), cls(nc);
        std::vector<Layout> lay(nc, L);
        std::vector<TableParams> prm(nc);
        std::vector<int64_t> off(nc);
        for (int c = 0; c < nc; ++c) {
            prm[c] = imag_time_params(dx, cand[c], 1.0, dtau);
            cls[c] = c;
            off[c] = (int64_t)c * n;
        }
        ClassSet cs;
        st = build_classes(cs, ns, lay, prm, nullptr);
        std::vector<double> e;
        std::vector<int> it;
        if (st == TDSE_OK) st = run_ground_states(cs, cls, dtau, kGsMaxIter, kGsTol, d_psi, off.data(), e, it, nullptr);
        cs.release();
        if (st != TDSE_OK) break;
        for (int c = 0; c < nc; ++c) {
            if (it[c] <= 0 || !std::isfinite(e[c])) {
                st = fail(TDSE_E_NOCONV, "ground state at a=%.17g did not converge", cand[c]);
                break;
            }
        }
        if (st != TDSE_OK) break;
        if (first) {
            if (!(e[0] < -ip && e[1] > -ip)) {
                st = fail(TDSE_E_INVALID, "-ip is not bracketed: E(a_lo)=%.6f E(a_hi)=%.6f", e[0], e[1]);
                break;
            }
            first = false;
        }
        // closest candidate and the new bracket
        double new_lo = lo, new_hi = hi;
        for (int c = 0; c < nc; ++c) {
            if (std::fabs(e[c] + ip) < std::fabs(best_e + ip) || (round == 0 && c == 0)) {
                best_a = cand[c];
                best_e = e[c];
            }
            if (e[c] < -ip && cand[c] > new_lo) new_lo = cand[c];
            if (e[c] > -ip && cand[c] < new_hi) new_hi = cand[c];
        }
        lo = new_lo;
        hi = new_hi;
        if (std::fabs(best_e + ip) < tol) done = true;
        else if (hi - lo <= 4.0 * std::numeric_limits<double>::epsilon() * hi) {
            st = fail(TDSE_E_NOCONV, "bracket collapsed at |E+ip| = %.3g", std::fabs(best_e + ip));
        }
    }
    (void)hipFree(d_psi);
    if (st == TDSE_OK && !done) st = fail(TDSE_E_NOCONV, "soft-core fit did not reach tol");
    *a_out = best_a;
    if (e_out) *e_out = best_e;
    return st;
}

tdse_status tdse_adjoint_batch(tdse_plan plan, const double* E, const double* psi0,
                               const double* accel_bar, double* grad_E, double* accel,
                               int32_t* sys_status, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (plan->adjoint_k <= 0 || !plan->d_adj)
        return fail(TDSE_E_INVALID, "plan was created without adjoint support (adjoint_k = 0)");
    if (!E || !accel_bar || !grad_E) return fail(TDSE_E_INVALID, "E, accel_bar and grad_E are required");
    const void* ptrs[] = {E, psi0, accel_bar, grad_E, accel, sys_status};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    FwdArgs base;
    fill_fwd_args(plan, base, E, psi0, accel, nullptr, nullptr, nullptr, sys_status);
    base.grad = grad_E;
    tdse_status rc = enqueue_adjoint(plan, base, accel_bar, kAdjFull, reinterpret_cast<hipStream_t>(stream));
    if (rc == TDSE_OK && plan->d_store) ++plan->ckpt_gen;  // the store now holds this E's pass
    return rc;
}

tdse_status tdse_plan_checkpoint_generation(tdse_plan plan, uint64_t* generation)
{
    g_last_error.clear();
    if (!plan || !generation) return fail(TDSE_E_INVALID, "NULL argument");
    *generation = plan->ckpt_gen;
    return TDSE_OK;
}

tdse_status tdse_adjoint_batch_stored(tdse_plan plan, uint64_t generation, const double* E,
                                      const double* accel_bar, double* grad_E, int32_t* sys_status,
                                      void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (!plan->d_store)
        return fail(TDSE_E_INVALID, "plan was created without TDSE_OPT_STORE_CHECKPOINTS");
    if (generation == 0 || generation != plan->ckpt_gen)
        return fail(TDSE_E_INVALID, "stored checkpoints are of generation %llu, not %llu",
                    (unsigned long long)plan->ckpt_gen, (unsigned long long)generation);
    if (!E || !accel_bar || !grad_E) return fail(TDSE_E_INVALID, "E, accel_bar and grad_E are required");
    const void* ptrs[] = {E, accel_bar, grad_E, sys_status};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    FwdArgs base;
    fill_fwd_args(plan, base, E, nullptr, nullptr, nullptr, nullptr, nullptr, sys_status);
    base.grad = grad_E;
    return enqueue_adjoint(plan, base, accel_bar, kAdjReverseOnly, reinterpret_cast<hipStream_t>(stream));
}

static void band_of(int32_t nt, double dt, double omega0, double h_lo, double h_hi, int32_t* k_lo,
                    int32_t* nk)
{
    const int64_t M = (int64_t)nt + 1;
    const double dw = 2.0 * M_PI / ((double)M * dt);
    int64_t lo = -1, hi = -2;
    for (int64_t k = 0; k <= M / 2; ++k) {
        const double w = (double)k * dw;
        if (w >= h_lo * omega0 && w <= h_hi * omega0) {
            if (lo < 0) lo = k;
            hi = k;
        }
    }
    *k_lo = (int32_t)std::max<int64_t>(lo, 0);
    *nk = lo < 0 ? 0 : (int32_t)(hi - lo + 1);
}

tdse_status tdse_harmonic_band(int32_t nt, double dt, double omega0, double h_lo, double h_hi,
                               int32_t* k_lo, int32_t* nk)
{
    g_last_error.clear();
    if (nt < 1 || !(dt > 0.0) || !(omega0 > 0.0) || !(h_hi >= h_lo) || h_lo < 0.0 || !k_lo || !nk)
        return fail(TDSE_E_INVALID, "need nt >= 1, dt > 0, omega0 > 0, 0 <= h_lo <= h_hi");
    band_of(nt, dt, omega0, h_lo, h_hi, k_lo, nk);
    return TDSE_OK;
}

tdse_status tdse_harmonic_yield(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                                double h_hi, const double* accel, const double* row_weight,
                                double* work, double* yield, double* accel_bar, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || nt < 1 || !(dt > 0.0) || !(omega0 > 0.0) || !(h_hi >= h_lo) || h_lo < 0.0)
        return fail(TDSE_E_INVALID, "need batch >= 1, nt >= 1, dt > 0, omega0 > 0, 0 <= h_lo <= h_hi");
    if (!accel || !yield || !work) return fail(TDSE_E_INVALID, "accel, work and yield are required");
    const void* ptrs[] = {accel, row_weight, work, yield, accel_bar};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    YieldArgs a{};
    band_of(nt, dt, omega0, h_lo, h_hi, &a.k_lo, &a.nk);
    a.batch = batch;
    a.nt = nt;
    a.dt = dt;
    a.omega0 = omega0;
    a.h_lo = h_lo;
    a.h_hi = h_hi;
    a.accel = accel;
    a.row_weight = row_weight;
    a.amp = work;
    a.yield = yield;
    a.abar = accel_bar;
    HIP_TRY(launch_yield(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_plan_stored_state(tdse_plan plan, uint64_t generation, int32_t index,
                                   double* psi_out, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (!plan->d_store) return fail(TDSE_E_INVALID, "plan was created without TDSE_OPT_STORE_CHECKPOINTS");
    if (generation == 0 || generation != plan->ckpt_gen)
        return fail(TDSE_E_INVALID, "stored checkpoints are of generation %llu, not %llu",
                    (unsigned long long)plan->ckpt_gen, (unsigned long long)generation);
    const int nseg = plan->p.nt / plan->adjoint_k + 1;
    if (index < 0 || index >= nseg) return fail(TDSE_E_INVALID, "index %d outside [0, %d)", index, nseg);
    if (!psi_out || !aligned16(psi_out)) return fail(TDSE_E_INVALID, "psi_out must be a 16-byte aligned device pointer");
    const int n_max = *std::max_element(plan->n_per.begin(), plan->n_per.end());
    HIP_TRY(launch_stored_state(plan->cls.d, plan->d_sys, plan->batch, n_max, plan->d_store,
                                plan->d_store_off, index, psi_out, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_plan_populations(tdse_plan plan, uint64_t generation, const double* psi_ref,
                                  double radius, double* gs, double* vol, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (!plan->d_store) return fail(TDSE_E_INVALID, "plan was created without TDSE_OPT_STORE_CHECKPOINTS");
    if (generation == 0 || generation != plan->ckpt_gen)
        return fail(TDSE_E_INVALID, "stored checkpoints are of generation %llu, not %llu",
                    (unsigned long long)plan->ckpt_gen, (unsigned long long)generation);
    if (!gs && !vol) return fail(TDSE_E_INVALID, "gs and vol are both NULL");
    if (!std::isfinite(radius)) return fail(TDSE_E_INVALID, "radius must be finite");
    if (psi_ref && !aligned16(psi_ref)) return fail(TDSE_E_INVALID, "psi_ref must be 16-byte aligned");
    PopArgs a{};
    a.classes = plan->cls.d;
    a.sys = plan->d_sys;
    a.batch = plan->batch;
    a.nrec = plan->p.nt / plan->adjoint_k + 1;
    a.store = plan->d_store;
    a.store_off = plan->d_store_off;
    a.psi_ref = psi_ref;
    a.gs = plan->d_gs;
    a.gs_off = plan->d_gs_off;
    a.radius = radius;
    a.gs_out = gs;
    a.vol_out = vol;
    HIP_TRY(launch_populations(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_plan_energy_spectrum(tdse_plan plan, const double* psi, int32_t n_energy,
                                      const double* energies, double eps, double* spectrum,
                                      void* work, size_t work_bytes, void* stream)
{
    g_last_error.clear();
    if (!plan) return fail(TDSE_E_INVALID, "plan is NULL");
    if (n_energy < 1 || !(eps > 0.0) || !std::isfinite(eps))
        return fail(TDSE_E_INVALID, "need n_energy >= 1 and a finite eps > 0");
    if (!psi || !energies || !spectrum || !work)
        return fail(TDSE_E_INVALID, "psi, energies, spectrum and work are required");
    if (!aligned16(psi) || !aligned16(work)) return fail(TDSE_E_INVALID, "psi and work must be 16-byte aligned");
    const int n_max = *std::max_element(plan->n_per.begin(), plan->n_per.end());
    const int64_t pairs = (int64_t)plan->ncls_real * n_energy;
    if (pairs > std::numeric_limits<int32_t>::max())
        return fail(TDSE_E_INVALID, "too many (size, energy) pairs");
    const size_t fac = spectrum_factor_bytes(n_max, pairs);
    const size_t rhs = ((size_t)plan->spec_rhs * sizeof(cd) + 255) & ~size_t(255);
    const size_t per_lane = spectrum_slot_bytes(n_max);
    // tiles of one energy x 64 systems of one size, one wavefront each
    const int64_t tiles = (int64_t)plan->spec_blocks * n_energy;
    if (work_bytes < fac + rhs + kWave * per_lane)
        return fail(TDSE_E_INVALID,
                    "work must hold at least %zu bytes: %zu of elimination factors, %zu of right-hand "
                    "sides and 64 solves of %zu",
                    fac + rhs + kWave * per_lane, fac, rhs, per_lane);
    int64_t waves = (int64_t)std::min<size_t>((work_bytes - fac - rhs) / (kWave * per_lane),
                                              (size_t)1 << 16);
    waves = std::max<int64_t>(1, std::min<int64_t>(waves, tiles));
    SpecArgs a{};
    a.fac = reinterpret_cast<cd*>(work);
    a.pairs = (int32_t)pairs;
    a.classes = plan->cls.d;
    a.sys = plan->d_sys;
    a.order = plan->d_order_all;
    a.spec = plan->d_spec;
    a.nspec = plan->spec_n;
    a.nblocks = plan->spec_blocks;
    a.batch = plan->batch;
    a.n_energy = n_energy;
    a.n_max = n_max;
    a.psi = psi;
    a.energies = energies;
    a.eps = eps;
    a.out = spectrum;
    a.rhs = reinterpret_cast<cd*>(static_cast<char*>(work) + fac);
    a.work = reinterpret_cast<cd*>(static_cast<char*>(work) + fac + rhs);
    a.lanes = waves * kWave;
    HIP_TRY(launch_energy_spectrum(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_plan_energy_spectrum_work(tdse_plan plan, int32_t n_energy, int64_t lanes,
                                           size_t* bytes)
{
    g_last_error.clear();
    if (!plan || !bytes) return fail(TDSE_E_INVALID, "plan and bytes are required");
    if (n_energy < 1 || lanes < kWave) return fail(TDSE_E_INVALID, "need n_energy >= 1 and lanes >= 64");
    const int n_max = *std::max_element(plan->n_per.begin(), plan->n_per.end());
    *bytes = spectrum_factor_bytes(n_max, (int64_t)plan->ncls_real * n_energy) +
             (((size_t)plan->spec_rhs * sizeof(cd) + 255) & ~size_t(255)) +
             (size_t)((lanes + kWave - 1) / kWave * kWave) * spectrum_slot_bytes(n_max);
    return TDSE_OK;
}

tdse_status tdse_energy_integral(int32_t batch, int32_t n_energy, const double* energies,
                                 const double* spectrum, double e_lo, double* out, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || n_energy < 2) return fail(TDSE_E_INVALID, "need batch >= 1 and n_energy >= 2");
    if (std::isnan(e_lo) || e_lo == std::numeric_limits<double>::infinity())
        return fail(TDSE_E_INVALID, "e_lo must be finite or -inf");
    if (!energies || !spectrum || !out) return fail(TDSE_E_INVALID, "energies, spectrum and out are required");
    HIP_TRY(launch_energy_integral(batch, n_energy, energies, spectrum, e_lo, out,
                                   reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_gabor(int32_t batch, int32_t nt, double dt, const double* accel, int32_t n_tc,
                       const double* t_centres, int32_t n_w, const double* omegas, double sigma,
                       double* out, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || nt < 1 || !(dt > 0.0) || n_tc < 1 || n_tc > 65535 || n_w < 1 ||
        n_w > kGaborMaxFreqs || !(sigma > 0.0) || !std::isfinite(sigma))
        return fail(TDSE_E_INVALID, "need batch, nt, dt > 0, 1 <= n_tc <= 65535, 1 <= n_w <= %d, sigma > 0",
                    kGaborMaxFreqs);
    if (!accel || !t_centres || !omegas || !out) return fail(TDSE_E_INVALID, "every array is required");
    GaborArgs a{};
    a.batch = batch;
    a.nt = nt;
    a.n_tc = n_tc;
    a.n_w = n_w;
    a.dt = dt;
    a.sigma = sigma;
    a.accel = accel;
    a.t_centres = t_centres;
    a.omegas = omegas;
    a.out = out;
    HIP_TRY(launch_gabor(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_band_dft(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                          double h_hi, const double* accel, double* amp, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || nt < 1 || !(dt > 0.0) || !(omega0 > 0.0) || !(h_hi >= h_lo) || h_lo < 0.0)
        return fail(TDSE_E_INVALID, "need batch >= 1, nt >= 1, dt > 0, omega0 > 0, 0 <= h_lo <= h_hi");
    if (!accel || !amp) return fail(TDSE_E_INVALID, "accel and amp are required");
    if (!aligned16(accel) || !aligned16(amp)) return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    YieldArgs a{};
    band_of(nt, dt, omega0, h_lo, h_hi, &a.k_lo, &a.nk);
    a.batch = batch;
    a.nt = nt;
    a.dt = dt;
    a.accel = accel;
    a.amp = amp;
    HIP_TRY(launch_band_dft(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_band_dft_adjoint(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                                  double h_hi, const double* amp_bar, double* accel_bar, void* stream)
{
    g_last_error.clear();
    if (batch < 1 || nt < 1 || !(dt > 0.0) || !(omega0 > 0.0) || !(h_hi >= h_lo) || h_lo < 0.0)
        return fail(TDSE_E_INVALID, "need batch >= 1, nt >= 1, dt > 0, omega0 > 0, 0 <= h_lo <= h_hi");
    if (!amp_bar || !accel_bar) return fail(TDSE_E_INVALID, "amp_bar and accel_bar are required");
    if (!aligned16(amp_bar) || !aligned16(accel_bar))
        return fail(TDSE_E_INVALID, "device pointers must be 16-byte aligned");
    BandAdjArgs a{};
    band_of(nt, dt, omega0, h_lo, h_hi, &a.k_lo, &a.nk);
    a.batch = batch;
    a.nt = nt;
    a.dt = dt;
    a.amp_bar = amp_bar;
    a.accel_bar = accel_bar;
    HIP_TRY(launch_band_adjoint(a, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

static tdse_status far_field_common(int32_t n_rho, int32_t n_z, const double* rho_src,
                                    const double* z_src, const double* weights, int32_t nk,
                                    const double* kwave, const double* in, int32_t n_obs,
                                    const double* rho_obs, double z_obs, double* out, bool adjoint,
                                    void* stream)
{
    g_last_error.clear();
    if (n_rho < 1 || n_z < 1 || nk < 1 || n_obs < 1 || (int64_t)n_rho * n_z > (1 << 26))
        return fail(TDSE_E_INVALID, "need n_rho, n_z, nk, n_obs >= 1 and n_rho * n_z <= 2^26");
    if (!std::isfinite(z_obs)) return fail(TDSE_E_INVALID, "z_obs must be finite");
    const void* ptrs[] = {rho_src, z_src, weights, kwave, in, rho_obs, out};
    for (const void* q : ptrs)
        if (!q) return fail(TDSE_E_INVALID, "every array is required");
    if (!aligned16(in) || !aligned16(out)) return fail(TDSE_E_INVALID, "complex arrays must be 16-byte aligned");
    FarArgs a{};
    a.n_rho = n_rho;
    a.n_z = n_z;
    a.n_obs = n_obs;
    a.nk = nk;
    a.rho_src = rho_src;
    a.z_src = z_src;
    a.weights = weights;
    a.kwave = kwave;
    a.rho_obs = rho_obs;
    a.z_obs = z_obs;
    a.in = in;
    a.out = out;
    HIP_TRY(launch_far_field(a, adjoint, reinterpret_cast<hipStream_t>(stream)));
    return TDSE_OK;
}

tdse_status tdse_far_field(int32_t n_rho, int32_t n_z, const double* rho_src, const double* z_src,
                           const double* weights, int32_t nk, const double* kwave, const double* amp,
                           int32_t n_obs, const double* rho_obs, double z_obs, double* field,
                           void* stream)
{
    return far_field_common(n_rho, n_z, rho_src, z_src, weights, nk, kwave, amp, n_obs, rho_obs,
                            z_obs, field, false, stream);
}

tdse_status tdse_far_field_adjoint(int32_t n_rho, int32_t n_z, const double* rho_src,
                                   const double* z_src, const double* weights, int32_t nk,
                                   const double* kwave, const double* field_bar, int32_t n_obs,
                                   const double* rho_obs, double z_obs, double* amp_bar,
                                   void* stream)
{
    return far_field_common(n_rho, n_z, rho_src, z_src, weights, nk, kwave, field_bar, n_obs,
                            rho_obs, z_obs, amp_bar, true, stream);
}

}  // extern "C"
