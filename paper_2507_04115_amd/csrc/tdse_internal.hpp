// tdse_internal.hpp -- structures shared by the host API (libtdse.cpp) and the
// gfx950 kernels (tdse_kernels.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdse {

struct cd {
    double re, im;
};

constexpr int kWave = 64;       // wavefront width on CDNA
constexpr int kMaxWaves = 16;   // lanes per system <= 1024
constexpr int kMaxLevels = 6;   // in-wave Kogge-Stone levels (2^6 = 64 lanes)
constexpr int kFlush = 32;      // samples per output flush
constexpr int kRing = 64;       // ring of per-wave partial sums (samples)

// Point tables of one size class, stored lane-interleaved: the value of
// grid point j = t*C + k (lane t, local index k) lives at [k*T + t], so the
// k-th loads of consecutive lanes are consecutive in memory.
//
// For the left-hand side L = M2 + h A of the Crank-Nicolson step (h = i dt/2
// in real time, dtau/2 in imaginary time) factorised without pivoting as
// L = (unit lower, subdiagonal l_j) (upper, pivots p_j, superdiagonal u_j):
//   alpha_j = -l_j            forward recurrence  z_j = r_j + alpha_j z_{j-1}
//   q_j     = 1 / (12 p_j)    scaling             w_j = q_j z_j
//   beta_j  = -u_j / p_j      backward recurrence y_j = w_j + beta_j y_{j+1}
// (the right-hand side is formed as 12 R psi, hence the 1/12 in q).
//   at_j    = prod_{m=s..j} alpha_m   within the lane's chunk [s, s+C)
//   bt_j    = prod_{m=j..s+C-1} beta_m
// Padding points (j >= n) have every coefficient 0 so they stay 0.
struct PointTables {
    double* v;      // V_j
    double* dv;     // dV/dx_j
    double* m;      // absorber mask m_j (0 on padding)
    cd* alpha;
    cd* at;
    cd* q;
    cd* beta;
    cd* bt;
};

// Per-lane constants (arrays of length T).
struct LaneTables {
    double* vl;    // V at s-1 (0 outside)
    double* vr;    // V at s+C
    double* ml;    // mask at s-1 (0 outside)
    double* mr;    // mask at s+C
    double* dvl;   // dV/dx at s-1
    double* dvr;   // dV/dx at s+C
    cd* ql;        // q at s-1
    cd* bl;        // beta at s-1
    cd* pa;        // [kMaxLevels][T]: prod of chunk products A over lanes [max(t-2^lev+1, ws), t]
    cd* pw;        // prod of A over [ws, t]   (ws = first lane of t's wave)
    cd* qb;        // [kMaxLevels][T]: prod of chunk products B over lanes [t, min(t+2^lev-1, we)]
    cd* qw;        // prod of B over [t, we]
    int32_t* hasmask;  // 1 if any mask value of the chunk differs from 1
};

// One size class: a distinct grid size n with its lane layout.
struct SizeClass {
    int32_t n;       // real grid size
    int32_t C;       // points per lane
    int32_t T;       // lanes per system (multiple of 64)
    int32_t levels;  // in-wave scan levels used (0..6)
    int32_t xwaves;  // previous/next waves chained in the cross-wave carry
    int32_t pad_;
    double dx;
    double x0;       // x of grid point 0 = -(n-1)/2 dx
    PointTables pt;
    LaneTables lt;
};

// Kernel-side description of one system of a batch.
struct SysDesc {
    int32_t cls;      // size class index
    int32_t n;
    int64_t psi_off;  // offset of the system's psi in ragged buffers (complex elements)
};

}  // namespace tdse
