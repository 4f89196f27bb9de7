// tdse_kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once
#include "tdse_internal.hpp"

namespace tdse {

// Parameters of one set of plan tables.
struct TableParams {
    double dx, a, z, mask_frac, mask_pow;
    cd h;  // i dt/2 (real time) or dtau/2 (imaginary time)
};

// Arguments of the persistent propagation kernels (forward and adjoint).
struct FwdArgs {
    const SizeClass* classes;
    const SysDesc* sys;
    const int32_t* order;   // systems of this launch, in queue order
    int32_t count;          // number of entries in `order` (all of one lane layout)
    int32_t* queue;         // work counter, reset to 0 before the launch
    int32_t nt;
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
    double* ckpt;           // per workgroup slot checkpoints
    double* seg;            // per workgroup slot segment states
    double* nrm_buf;        // per workgroup slot norm series
    int64_t slot_stride_ckpt;  // doubles per slot
    int64_t slot_stride_seg;
    int32_t k_ckpt;
};

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

hipError_t launch_build_tables(const SizeClass* d_classes, const TableParams* d_params, int ncls,
                               double* d_metrics, cd* d_scratch, int max_t, hipStream_t st);
hipError_t launch_reset_counters(int32_t* counters, int n, hipStream_t st);
// Occupancy (workgroups per CU) of the forward kernel for points-per-lane C
// and T lanes; 0 if the configuration is not built.
int forward_occupancy(int C, int T);
int adjoint_occupancy(int C, int T);
hipError_t launch_forward(int C, const FwdArgs& a, int T, int grid, hipStream_t st);
hipError_t launch_adjoint(int C, const FwdArgs& a, int T, int grid, hipStream_t st);
hipError_t launch_ground_state(int C, const GsArgs& a, int T, hipStream_t st);
hipError_t launch_yield(const YieldArgs& a, hipStream_t st);
bool layout_supported(int C);

}  // namespace tdse
