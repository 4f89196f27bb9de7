// tdse_kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once
#include "tdse_internal.hpp"

namespace tdse {

constexpr int kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

// Parameters of one set of plan tables.
struct TableParams {
    double dx, a, z, mask_frac, mask_pow;
    cd h;  // i dt/2 (real time) or dtau/2 (imaginary time)
};

// Arguments of the persistent propagation kernels (forward and adjoint).
// One launch covers the systems of one size class.
struct FwdArgs {
    const SizeClass* classes;
    const SysDesc* sys;
    // forward: workgroup bins (one queue item each)
    const BinDesc* bins;
    int32_t nbins;
    int32_t item_off;       // LDS byte offset of the workgroup's queue slot
    // adjoint: the systems of one size class, one subgroup each
    const int32_t* order;   // systems of this launch, in queue order
    int32_t count;          // number of entries in `order`
    int32_t cls;            // size class of every system of this launch
    // adjoint: one work counter, reset to 0 before the launch.  forward:
    // kQueueInts ints, queue[x] the counter of XCD x (reset to 0 before the
    // launch) and queue[kXcds + x] .. queue[kXcds + x + 1] the bins of its run
    int32_t* queue;
    int32_t nt;
    int64_t sub_bytes;      // LDS bytes per subgroup
    double dt;
    const double* E;        // [batch][nt+1]
    const double* psi0;     // ragged, or NULL
    const double* gs;       // plan ground states, ragged by size class
    const int64_t* gs_off;  // per class offset into gs (complex elements)
    double* accel;
    double* xexp;
    double* norm;
    double* psi_final;
    int32_t* status;
    // adjoint only
    const double* abar;     // [batch][nt+1]
    double* grad;           // [batch][nt+1]
    double* work;           // per subgroup slot: [checkpoints, norm row,] segment states
    int64_t slot_doubles;   // doubles per slot
    int32_t k_ckpt;
    int32_t mode;           // kAdjFull, kAdjForwardOnly or kAdjReverseOnly
    // layouts without q in registers: read the elimination factors from
    // their tables (1) or form them from q and om (0)
    int32_t ab;
    // per-system checkpoints and norm rows (stored mode), or NULL: then they
    // live in the slot
    double* store;
    const int64_t* store_off;  // [batch] doubles into store
    // forward only: per-step populations (tdse_propagate_batch_populations),
    // written when either row pointer is set
    const double* pop_ref;     // ragged complex reference states, or NULL: the
                               // plan's ground states
    double* gs_pop;            // [batch][nt+1] or NULL
    double* vol_pop;           // [batch][nt+1] or NULL
    double pop_radius;
};

// Adjoint kernel modes: forward pass then reverse sweep; forward pass only
// (outputs and stored checkpoints); reverse sweep only, from the stored
// checkpoints of an earlier forward pass.
constexpr int32_t kAdjFull = 0;
constexpr int32_t kAdjForwardOnly = 1;
constexpr int32_t kAdjReverseOnly = 2;

struct GsArgs {
    const SizeClass* classes;
    const int32_t* cls_of;  // size class of each candidate
    int32_t ncand;
    double dtau;
    int32_t max_iter;
    double tol;
    double* psi_out;        // [ncand] ragged by psi_off
    const int64_t* psi_off;
    double* energy;         // [ncand]
    int32_t* iters;         // [ncand]; negative when not converged
};

// Far field of the medium (tdse_far_field) and its adjoint.
struct FarArgs {
    int32_t n_rho, n_z, n_obs, nk;
    const double* rho_src;  // [n_rho]
    const double* z_src;    // [n_z]
    const double* weights;  // [n_rho * n_z], source p = i * n_z + j
    const double* kwave;    // [nk]
    const double* rho_obs;  // [n_obs]
    double z_obs;
    const double* in;       // forward: S [P][nk] complex; adjoint: E_bar [n_obs][nk]
    double* out;            // forward: E [n_obs][nk] complex; adjoint: S_bar [P][nk]
};

// Adjoint of the band spectrum: accel_bar from amp_bar (tdse_band_dft_adjoint).
struct BandAdjArgs {
    int32_t batch, nt;
    double dt;
    int32_t k_lo, nk;
    const double* amp_bar;  // [batch][nk] complex
    double* accel_bar;      // [batch][nt+1]
};

// One grid size of a batch as the electron energy distribution sees it: its
// systems are order[start .. start+count), their right-hand sides stored
// point by point (rhs[rhs_off + j * count + k] for the k-th of them), in
// blocks of 64 systems numbered blk0 .. blk0 + ceil(count / 64) - 1.
struct SpecClass {
    int32_t cls;      // size class
    int32_t n;        // grid size
    int32_t start;    // first position in the plan's system order
    int32_t count;    // systems of this size
    int32_t blk0;     // first 64-system block
    int32_t pad_;
    int64_t rhs_off;  // complex elements into rhs
};

// Electron energy distribution (tdse_plan_energy_spectrum).
struct SpecArgs {
    const SizeClass* classes;
    const SysDesc* sys;
    const int32_t* order;    // systems grouped by size class
    const SpecClass* spec;   // [nspec], ordered by blk0
    int32_t nspec, nblocks;  // sizes, 64-system blocks over all sizes
    int32_t batch, n_energy, n_max;
    const double* psi;       // ragged complex, plan offsets
    const double* energies;  // [n_energy]
    double eps;
    double* out;             // [batch][n_energy]
    cd* fac;                 // [pairs][n_max][3] (1/p, -low/p, -c'), pair = class * n_energy + energy
    int32_t pairs;           // real classes * n_energy
    cd* rhs;                 // M2 psi, point-interleaved per size (SpecClass)
    cd* work;                // per wavefront: [groups - 1][64] start values of the d' groups
    int64_t lanes;           // solves in flight (a multiple of 64)
};

// Gabor transform of the source term (tdse_gabor).
struct GaborArgs {
    int32_t batch, nt, n_tc, n_w;
    double dt, sigma;
    const double* accel;      // [batch][nt+1]
    const double* t_centres;  // [n_tc]
    const double* omegas;     // [n_w]
    double* out;              // [batch][n_tc][n_w]
};

// Ground-state and volumetric populations of stored records (tdse_plan_populations).
struct PopArgs {
    const SizeClass* classes;
    const SysDesc* sys;
    int32_t batch, nrec;
    const double* store;       // per-system records
    const int64_t* store_off;  // [batch]
    const double* psi_ref;     // ragged complex, or null: the plan's ground states
    const double* gs;          // plan ground states, per class
    const int64_t* gs_off;
    double radius;
    double* gs_out;            // [batch][nrec], or null
    double* vol_out;           // [batch][nrec], or null
};

struct YieldArgs {
    int32_t batch, nt;
    double dt, omega0, h_lo, h_hi;
    int32_t k_lo, nk;       // band bins k_lo .. k_lo+nk-1
    const double* accel;
    const double* row_weight;
    double* amp;            // [batch][nk] complex scratch
    double* yield;
    double* abar;
};

// Field resampling by Fourier zero-padding (tdse_resample_field).
struct ResampleArgs {
    int32_t batch, m, nt;
    int64_t mp;             // padded length M' = M dt_coarse / dt
    const double* coarse;   // [batch][m]
    double* spec;           // [batch][m/2+1] complex: the DFT of each row
    double* fine;           // [batch][nt+1]
};

hipError_t launch_resample(const ResampleArgs& a, hipStream_t st);
hipError_t launch_far_field(const FarArgs& a, bool adjoint, hipStream_t st);
hipError_t launch_energy_spectrum(const SpecArgs& a, hipStream_t st);
// Bytes of the shared elimination factors of tdse_plan_energy_spectrum, and
// of one solve's slot of d' group starts.
size_t spectrum_factor_bytes(int n_max, int64_t pairs);
size_t spectrum_slot_bytes(int n_max);
hipError_t launch_gabor(const GaborArgs& a, hipStream_t st);
hipError_t launch_energy_integral(int batch, int n_energy, const double* energies,
                                  const double* spectrum, double e_lo, double* out, hipStream_t st);
hipError_t launch_populations(const PopArgs& a, hipStream_t st);
hipError_t launch_stored_state(const SizeClass* classes, const SysDesc* sys, int batch, int n_max,
                               const double* store, const int64_t* store_off, int index,
                               double* psi_out, hipStream_t st);
constexpr int kGaborMaxFreqs = 1024;  // frequencies per call (4 per thread of 256)
hipError_t launch_band_adjoint(const BandAdjArgs& a, hipStream_t st);

hipError_t launch_build_tables(const SizeClass* d_classes, const TableParams* d_params, int ncls,
                               double* d_metrics, cd* d_scratch, int max_t, hipStream_t st);
hipError_t launch_reset_counters(int32_t* counters, int n, hipStream_t st);
// Zeroes the kXcds counters of `nq` consecutive forward queues.
hipError_t launch_reset_queues(int32_t* queues, int nq, hipStream_t st);
bool layout_supported(int C);
size_t sub_smem_bytes(int W);

// Forward kernel over workgroup bins: C points per lane, `threads` lanes per
// workgroup, `smem` bytes of LDS (staged tables of the bin's classes, the
// subgroups' scratch blocks, the queue slot), table placement `tab`
// (kTabGlobal, kTabLds, kTabOmLds).  Occupancy is in workgroups per CU (0
// when it does not fit or the combination is not instantiated).
bool forward_tab_supported(int C, int tab);
int forward_occupancy(int C, int threads, size_t smem, int tab);
// Vector registers per lane of the forward kernel instance launched with
// `threads` per workgroup (0 if not instantiated).
int forward_vgprs(int C, int tab, bool ab, int threads);
// Whether workgroups of `threads` run the narrow instance (at most 512
// threads, 256 registers per lane, pivot factors in registers).
bool forward_narrow(int C, int threads);
hipError_t launch_forward(int C, int tab, const FwdArgs& a, int threads, size_t smem, int grid,
                          hipStream_t st);

size_t adjoint_smem_bytes(int C, int T, int S, bool lds_tables);
// Workgroups per CU of the adjoint kernel; `stored`: the packing must also
// fit the reverse-only instance (plans with stored checkpoints).
int adjoint_occupancy(int C, int T, int S, bool lds_tables, bool stored);
// Workgroups of at most 512 threads run the instances with 256 registers per
// lane (2 waves per SIMD); wider ones those with 128 (4 waves per SIMD).
bool adjoint_narrow(int threads);
hipError_t launch_adjoint(int C, bool lds_tables, const FwdArgs& a, int T, int S, int grid,
                          hipStream_t st);

// Orders the systems of one launch so that rows with a non-zero abar come
// first; counters (2 ints) must be zero.
hipError_t launch_compact_rows(const double* abar, int nt, const int32_t* order_in, int count,
                               int32_t* order_out, int32_t* counters, hipStream_t st);
hipError_t launch_ground_state(int C, const GsArgs& a, int T, hipStream_t st);
hipError_t launch_yield(const YieldArgs& a, hipStream_t st);
hipError_t launch_band_dft(const YieldArgs& a, hipStream_t st);

}  // namespace tdse
