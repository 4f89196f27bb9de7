// tdse_internal.hpp -- structures shared by the host API (libtdse.cpp) and the
// gfx950 kernels.  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdse {

struct alignas(16) cd {
    double re, im;
};

constexpr int kWave = 64;       // wavefront width on CDNA
constexpr int kMaxWaves = 16;   // lanes per system <= 1024
constexpr int kMaxLevels = 6;   // in-wave Kogge-Stone levels (2^6 = 64 lanes)
constexpr int kFlush = 32;      // samples per output flush
constexpr int kRing = 64;       // ring of per-wave partial sums (samples)
constexpr int kLdsTableBytes = 16;  // LDS bytes per grid point of the staged
                                    // tables (om and dV/dx)

// Placement of a size class's om and dV/dx tables in a workgroup: both read
// from global memory, both staged in LDS, or om staged in LDS and dV/dx read
// from global memory (for grids whose full tables do not fit).
constexpr int kTabGlobal = 0;
constexpr int kTabLds = 1;
constexpr int kTabOmLds = 2;
__host__ __device__ constexpr int tab_lds_bytes(int tab)
{
    return tab == kTabLds ? kLdsTableBytes : (tab == kTabOmLds ? 8 : 0);
}

__host__ __device__ inline int pbase(int t, int C) { return (t >> 6) * (C * 64) + (t & 63); }
__host__ __device__ inline int pidx(int t, int k, int C) { return pbase(t, C) + 64 * k; }

// Point tables of one size class, stored lane-interleaved by wavefront: the
// value of grid point j = t*C + k (lane t, local index k) lives at
// pidx(t, k, C) = (t/64)*64C + 64k + t%64.  The k-th accesses of the 64 lanes
// of a wavefront are consecutive (coalesced in HBM, bank-conflict free in
// LDS) and the offset of point k from the lane's base is the compile-time
// constant 64k, so every table access in the unrolled chunk loops is an
// immediate-offset load from one base register.
//
// The Crank-Nicolson left-hand side L = M2 + h A (h = i dt/2 in real time,
// dtau/2 in imaginary time) is factorised without pivoting as
// L = (unit lower, subdiagonal l_{j-1}/p_{j-1}) (upper, pivots p_j,
// superdiagonal u_j).  With the right-hand side formed as 12 R psi:
//   om_j  = 12 |h| (V_j/12 - 1/(2 dx^2))   (so 12 l_j = 1 + h' om_j,
//                                           12 u_j = 1 + h' om_{j+1},
//                                           h' = i or 1)
//   q_j   = 1 / (12 p_j)
//   alpha_j = -(1 + h' om_{j-1}) q_{j-1}    forward  z_j = r_j + alpha_j z_{j-1}
//   beta_j  = -(1 + h' om_{j+1}) q_j        backward y_j = q_j z_j + beta_j y_{j+1}
// alpha and beta build the lane carry products.  Where q is held in
// registers the kernels recompute them from om and q (two FMAs each, om read
// from LDS); where q would be read from memory they read alpha and beta
// instead, which costs the same 16 bytes and saves the FMAs.
// Padding points (j >= n) have q = 0, V = 0, dV = 0, m = 0, so they stay 0.
struct PointTables {
    double* v;      // V_j
    double* om;     // om_j
    double* dv;     // dV/dx_j
    double* m;      // absorber mask m_j (0 on padding)
    cd* q;
    cd* alpha;
    cd* beta;
};

// Per-lane constants (arrays of length T).
struct LaneTables {
    cd* pa;        // [kMaxLevels][T]: prod of chunk products A over lanes [max(t-2^lev+1, ws), t]
    cd* pw;        // prod of A over [ws, t]   (ws = first lane of t's wave)
    cd* qb;        // [kMaxLevels][T]: prod of chunk products B over lanes [t, min(t+2^lev-1, we)]
    cd* qw;        // prod of B over [t, we]
    int32_t* hasmask;  // absorber flags: bit 0 chunk, bit 1 point s-1, bit 2 point s+C
                       // (set where a mask value differs from 1)
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
    double dofs10;   // 7.2 |h| / dx^2 (|h| = dt/2 or dtau/2): a tenth of the
                     // diagonal of 12 |h| (-D2/2), used by the right-hand side
    PointTables pt;
    LaneTables lt;
};

// One workgroup's worth of work for the forward kernel: up to kMaxSubs
// systems of one lane layout, each on a contiguous run of wavefronts
// (a subgroup of T = 64 W lanes).  Lanes that no system needs run a padding
// system (p = -1) of a padding class with exactly that many lanes, so every
// wavefront takes the same sequence of barriers.  Packing systems of
// different sizes into full workgroups is what lets one persistent launch
// keep every SIMD busy on an uneven batch.
constexpr int kMaxSubs = 16;

struct BinSub {
    int32_t p;        // system, or -1 for padding
    int32_t cls;      // size class
    int32_t wave0;    // first wavefront of the subgroup in the workgroup
    int32_t tab_off;  // byte offset of the class's staged tables in LDS
    int32_t sub_off;  // byte offset of the subgroup's scratch block in LDS
    int32_t stage;    // 1: this subgroup copies its class's tables into LDS
    int32_t pad_[2];
};

constexpr int kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2
constexpr int kQueueInts = 2 * kXcds + 1;  // a forward work queue: counters, run bounds

struct BinDesc {
    int32_t nsub;
    int32_t pad_[3];
    int32_t sub_of_wave[kMaxSubs];  // subgroup of each wavefront
    BinSub sub[kMaxSubs];
};

// Kernel-side description of one system of a batch.
struct SysDesc {
    int32_t cls;      // size class index
    int32_t n;
    int64_t psi_off;  // offset of the system's psi in ragged buffers (complex elements)
};

}  // namespace tdse
