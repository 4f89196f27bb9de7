/*
 * libtdse.h -- C-ABI of libtdse, a gfx950 (MI355X) implementation of the
 * microscopic step of the multiscale high-harmonic-generation model of
 * arXiv 2507.04115: one independent 1D time-dependent Schrodinger equation
 * per macroscopic point, soft-core atom, length gauge, Numerov-corrected
 * Crank-Nicolson with a split-operator field phase, dipole acceleration out.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Atomic units.  Grid of n points x_j = (j - (n-1)/2) dx, j = 0..n-1,
 *    Dirichlet outside; time grid t_i = i dt, i = 0..nt (the paper's grids,
 *    section "1D-TSDE Implementation (CTDSE)", shifted to start at t = 0).
 *  - Wavefunctions are complex128 stored interleaved (re, im) as double[2n].
 *  - Field and output series are row-major double[batch][nt+1].
 *  - "dev" pointers are HIP device pointers (16-byte aligned); "host"
 *    pointers are ordinary host memory.  The caller owns every buffer.
 *  - Calls that take a `stream` (a hipStream_t passed as void*, NULL = the
 *    null stream) are asynchronous and stream-ordered unless stated; argument
 *    errors are reported before anything is launched.
 *  - Every call returns a tdse_status; on failure a thread-local detail
 *    string is available from tdse_last_error().
 *
 * No entry point allocates device memory except tdse_plan_create (which
 * sizes every workspace it will ever need), tdse_ground_state and
 * tdse_soft_core_for_ip (both synchronous set-up calls).
 */
#ifndef LIBTDSE_H
#define LIBTDSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t tdse_status;
#define TDSE_OK 0
#define TDSE_E_INVALID (-1)     /* bad argument; nothing was launched         */
#define TDSE_E_NOMEM (-2)       /* device or host allocation failed           */
#define TDSE_E_DEVICE (-3)      /* a HIP runtime call failed                  */
#define TDSE_E_NOCONV (-4)      /* ground state / soft-core fit not converged */
#define TDSE_E_UNSUPPORTED (-5) /* size or device outside what is built       */
#define TDSE_E_NONFINITE (-6)   /* a non-finite value was produced            */

/* Per-system status words written by the propagation calls (sys_status). */
#define TDSE_SYS_OK 0
#define TDSE_SYS_NONFINITE 1    /* an observable became NaN/Inf               */
#define TDSE_SYS_NORM_GROWTH 2  /* norm exceeded its initial value by >1e-8   */

const char* tdse_version(void);
const char* tdse_status_string(tdse_status s);
/* Detail of the last failing call on this thread ("" if none). */
const char* tdse_last_error(void);

/* ---------------------------------------------------------------- params */
/* Physical and numerical parameters of one batch.
 *  dx, dt          grid spacing and time step (> 0)
 *  a, charge_z     soft-core potential V(x) = -charge_z / sqrt(x^2 + a^2)
 *                  (section "Microscopic Response in XUV regime (TDSE)",
 *                  Eq. SC potential); charge_z = 0 gives a free particle
 *  mask_fraction   absorber on this fraction of the whole grid at each side,
 *                  in [0, 0.5) (0 disables; 0.1: the outer tenth of the grid
 *                  at each side, |x| > 0.8 x_max);
 *                  m(x) = cos(pi/2 (|x|-x_a)/(x_max-x_a))^mask_power for
 *                  x_a < |x| < x_max, x_a = (1 - 2 mask_fraction) x_max,
 *                  x_max = (n-1) dx / 2, 1 inside and 0 at the two outermost
 *                  points.  The paper's solver has no absorber; this one is
 *                  applied after the field substep.
 *  mask_power      exponent of the absorber (e.g. 0.125)
 *  nt              number of time steps; every series has nt+1 samples
 *  flags           reserved, must be 0 */
typedef struct {
    double dx;
    double dt;
    double a;
    double charge_z;
    double mask_fraction;
    double mask_power;
    int32_t nt;
    uint32_t flags;
} tdse_params;

/* ------------------------------------------------------ ground state, fit */
/* Imaginary-time relaxation (dt -> -i dtau in the Crank-Nicolson step, with
 * renormalisation to dx sum |psi|^2 = 1) of the field-free Hamiltonian
 * H0 = p^2/2 + V_C on the n-point grid of `p` (p->a, p->charge_z, p->dx;
 * the absorber and p->dt, p->nt are ignored).  The paper fixes a so that the
 * ground-state energy matches the atom's (section "Microscopic Response in
 * XUV regime (TDSE)", text after Eq. SC potential).
 *   dtau       imaginary time step, 0 < dtau < 2/|E_g| (e.g. 1.0)
 *   max_iter   iteration cap; tol: stop when successive normalised iterates
 *              differ by less than tol (dx-weighted L2)
 *   psi_out    dev, 2n doubles: real, positive at the centre
 *   energy_out host, may be NULL: ground-state energy E_g
 * Synchronous on `stream`.  TDSE_E_NOCONV if max_iter is reached. */
tdse_status tdse_ground_state(const tdse_params* p, int32_t n, double dtau, int32_t max_iter,
                              double tol, double* psi_out, double* energy_out, void* stream);

/* tdse_ground_state for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results (bitwise), but the
 * tables and the kernel's outputs live in a static device workspace of
 * 2 MiB that each GPU holds until the process ends, so the call makes no
 * hipMalloc, hipFree or allocating library call.  That covers every n up
 * to 16384; a layout needing more fails with TDSE_E_NOMEM before any launch.
 * Calls share their GPU's workspace: the library runs calls on one GPU from
 * threads of one process one after the other (the call is synchronous), and
 * overlapping use of the workspace by other means races. */
tdse_status tdse_ground_state_noalloc(const tdse_params* p, int32_t n, double dtau,
                                      int32_t max_iter, double tol, double* psi_out,
                                      double* energy_out, void* stream);

/* Soft-core parameter a in [a_lo, a_hi] whose ground-state energy on the
 * n-point grid of spacing dx equals -ip (E_g increases with a).  Multisection:
 * each round evaluates a batch of candidates on the device.
 *   tol        stop when |E_g(a) + ip| < tol
 *   a_out      host; e_out host, may be NULL.  Synchronous. */
tdse_status tdse_soft_core_for_ip(double ip, int32_t n, double dx, double dtau, double tol,
                                  double a_lo, double a_hi, double* a_out, double* e_out);

/* ------------------------------------------------------------------ plan */
typedef struct tdse_plan_s* tdse_plan;

/* Plan options (bit flags). */
#define TDSE_OPT_NONE 0u
#define TDSE_OPT_PLAIN 1u     /* propagate one system per launch (no queue)   */
#define TDSE_OPT_NO_GRAPH 2u  /* launch directly instead of replaying a graph */
#define TDSE_OPT_AUTOTUNE 4u  /* time the candidate layouts at plan creation  */
#define TDSE_OPT_STORE_CHECKPOINTS 8u /* forward stores adjoint checkpoints   */

/* Creates a plan for `batch` systems of sizes n_per_system[0..batch-1]
 * (host array, each 16 <= n <= 16384) sharing the parameters `p`.  The plan
 * precomputes, per distinct n, the grid tables and the factorisation of the
 * constant Crank-Nicolson matrix (section "1D-TSDE Implementation (CTDSE)":
 * the field is split off, so the tridiagonal left-hand side never changes),
 * computes the ground state for each distinct n (used when psi0 is NULL),
 * chooses a lane layout per n, and allocates every workspace the
 * propagation and adjoint calls need.  Synchronous (device 0 of the calling
 * thread's current device).  The plan is immutable; one plan must not be
 * used by two threads at once.
 *   adjoint_k  checkpoint interval of the adjoint in steps (>= 1); 0 creates a
 *              forward-only plan without the adjoint workspace
 * With TDSE_OPT_STORE_CHECKPOINTS (needs adjoint_k > 0, excludes
 * TDSE_OPT_PLAIN) the plan also holds, per system, the states at steps
 * 0, K, 2K, ... and the norm row of the last forward pass: about
 * 16 (C+2)/C n (nt/K + 1) + 8 (nt+1) bytes per system (C = points per lane).
 * tdse_propagate_batch then runs the adjoint kernel's forward pass, which
 * writes the same outputs and the store, and tdse_adjoint_batch_stored can
 * skip that pass. */
tdse_status tdse_plan_create(const tdse_params* p, int32_t batch, const int32_t* n_per_system,
                             uint32_t options, int32_t adjoint_k, tdse_plan* out);
tdse_status tdse_plan_destroy(tdse_plan plan);

/* Offsets (in complex elements) of each system's wavefunction inside a
 * ragged psi buffer: offsets[0] = 0, offsets[b+1] = offsets[b] + n_b.
 * host, batch+1 entries. */
tdse_status tdse_plan_psi_offsets(tdse_plan plan, int64_t* offsets);

/* Layout chosen for size n: points per lane, lanes per system, scan levels
 * (host outputs, any may be NULL). */
tdse_status tdse_plan_layout(tdse_plan plan, int32_t n, int32_t* points_per_lane,
                             int32_t* lanes, int32_t* scan_levels);

/* Launch parameters chosen for size n (host outputs, any may be NULL):
 * systems per workgroup, the placement of the per-point tables (om and
 * dV/dx) of the forward kernel -- 0 both read from global memory, 1 both
 * staged in LDS, 2 om staged in LDS and dV/dx read from global memory -- and
 * the probe rate in grid-point-steps/s measured by the autotuner (0 when
 * the plan was not created with TDSE_OPT_AUTOTUNE).  The autotuner times,
 * for each distinct n, every lane layout that fits (points per lane C in
 * {4, 8, 12, 16}, 12 only for plans without the adjoint, i.e. the length of
 * the lane-local Thomas chunks against the
 * width of the cross-lane scan; systems per workgroup; table placement) on
 * a probe batch that fills the GPU once, and keeps the fastest.  Results are
 * cached per process, and on disk when a cache file is set
 * (tdse_set_tune_cache, or the TDSE_TUNE_CACHE environment variable). */
tdse_status tdse_plan_launch_info(tdse_plan plan, int32_t n, int32_t* systems_per_workgroup,
                                  int32_t* lds_tables, double* tuned_rate);

/* Sets the file where the autotuner keeps its choices across processes (path
 * NULL or "": none; until this is called, the TDSE_TUNE_CACHE environment
 * variable names it) and clears the per-process cache.  Choices are keyed by
 * device architecture, n, batch count, dx, dt, a, charge and absorber; a
 * line that is unreadable, fails its checksum or names a layout that does
 * not fit is ignored, the size is timed again and the file rewritten (whole,
 * then renamed into place).  A file that cannot be written only costs the
 * next process its probes.  Thread-safe. */
tdse_status tdse_set_tune_cache(const char* path);

/* How the plan's forward calls run: 0 no call yet, 1 replay of a captured
 * hipGraph, 2 direct launches because graph capture failed (or was
 * switched off with the TDSE_FORCE_CAPTURE_FAILURE environment variable,
 * a failure-injection hook); direct launches run the same kernels with the
 * same arguments.  Plans with TDSE_OPT_NO_GRAPH, TDSE_OPT_PLAIN or stored
 * checkpoints never capture (state 0). */
tdse_status tdse_plan_graph_state(tdse_plan plan, int32_t* state);

/* Launch shape of the persistent forward kernel that propagates the systems
 * of size n (section "1D-TSDE Implementation (CTDSE)" is run by one such
 * launch per lane layout): lanes per workgroup, workgroups launched,
 * workgroups resident per CU, LDS bytes per workgroup and vector registers
 * per lane.  Resident wavefronts per SIMD = workgroups_per_cu *
 * workgroup_lanes / 64 / 4.  Any output pointer may be NULL.  Fails with
 * TDSE_E_INVALID on a plan created with TDSE_OPT_PLAIN or an n the plan does
 * not hold. */
tdse_status tdse_plan_kernel_info(tdse_plan plan, int32_t n, int32_t* workgroup_lanes,
                                  int32_t* grid, int32_t* workgroups_per_cu, int32_t* lds_bytes,
                                  int32_t* vgprs);

/* Device copy of the plan's ground state for size n (dev, 2n doubles) and its
 * energy (host, may be NULL).  Synchronous. */
tdse_status tdse_plan_ground_state(tdse_plan plan, int32_t n, double* psi_out,
                                   double* energy_out);

/* --------------------------------------------------------------- forward */
/* Propagates every system of the plan over nt steps (section "1D-TSDE
 * Implementation (CTDSE)", the three substeps: Crank-Nicolson right-hand
 * side, tridiagonal solve, field phase exp(-i dt E(t_i) x_j)), followed by
 * the absorber, and records at every sample i = 0..nt
 *   accel[b][i] = dx sum_j |psi_j|^2 (dV/dx_j + E_i)   (dipole acceleration,
 *                 section "Microscopic Response in XUV regime (TDSE)",
 *                 Eq. dipole acceleration)
 *   xexp[b][i]  = dx sum_j x_j |psi_j|^2,   norm[b][i] = dx sum_j |psi_j|^2
 * computed from psi^(i) (before step i).
 *   E          dev [batch][nt+1]: field samples E(t_i) of every system
 *   psi0       dev ragged complex (tdse_plan_psi_offsets), or NULL = the
 *              plan's ground states
 *   accel      dev [batch][nt+1], required; xexp, norm: same, may be NULL
 *   psi_final  dev ragged complex, may be NULL
 *   sys_status dev int32[batch], may be NULL (TDSE_SYS_* codes)
 * Asynchronous on `stream`. */
tdse_status tdse_propagate_batch(tdse_plan plan, const double* E, const double* psi0,
                                 double* accel, double* xexp, double* norm, double* psi_final,
                                 int32_t* sys_status, void* stream);

/* tdse_propagate_batch that also records, at every sample i = 0..nt, the
 * ground-state population and the volumetric population near the nucleus
 * (section "Microscopic Response in XUV regime (TDSE)", the analyses of psi
 * listed after the dipole acceleration, shown over time in the microscopic
 * insights of the physical examples):
 *   gs_pop[b][i]  = |dx sum_j conj(phi_j) psi^(i)_j|^2
 *   vol_pop[b][i] = dx sum_{|x_j| <= radius} |psi^(i)_j|^2,
 *                   x_j = (j - (n-1)/2) dx
 * reduced in the time loop with the other observables.
 *   psi_ref   dev ragged complex reference states phi (plan offsets), or
 *             NULL = the plan's ground state of each system's grid
 *   radius    >= 0 (a.u.)
 *   gs_pop, vol_pop  dev [batch][nt+1]; at least one of them
 * The other arguments and outputs are those of tdse_propagate_batch (same
 * values).  Launched directly (no graph replay).  TDSE_E_UNSUPPORTED on a
 * plan created with TDSE_OPT_STORE_CHECKPOINTS (its stored states have
 * tdse_plan_populations).  Asynchronous on `stream`. */
tdse_status tdse_propagate_batch_populations(tdse_plan plan, const double* E, const double* psi0,
                                             double* accel, double* xexp, double* norm,
                                             double* psi_final, int32_t* sys_status,
                                             const double* psi_ref, double radius,
                                             double* gs_pop, double* vol_pop, void* stream);

/* --------------------------------------------------------------- adjoint */
/* Gradient of a loss l(accel) with respect to every field sample.  Given
 * accel_bar[b][i] = dl/d accel[b][i], writes grad_E[b][i] = dl/dE_b(t_i).
 * The gradient is the exact discrete adjoint of tdse_propagate_batch (the
 * paper has no adjoint; this one follows from differentiating the forward
 * recursion step by step): the costate is propagated backward in time with
 * the adjoint of each substep, the forward wavefunction being recomputed
 * from checkpoints stored every plan->adjoint_k steps during a forward pass
 * that this call runs first.  On a plan with TDSE_OPT_STORE_CHECKPOINTS that
 * pass rewrites the plan's store (and advances its generation).
 *   E, psi0    as for tdse_propagate_batch
 *   accel_bar  dev [batch][nt+1]; rows that are entirely zero are skipped
 *              (their grad_E row is zero)
 *   grad_E     dev [batch][nt+1], overwritten
 *   accel      dev [batch][nt+1], may be NULL: forward accelerations
 *   sys_status dev int32[batch], may be NULL
 * Asynchronous on `stream`. */
tdse_status tdse_adjoint_batch(tdse_plan plan, const double* E, const double* psi0,
                               const double* accel_bar, double* grad_E, double* accel,
                               int32_t* sys_status, void* stream);

/* Generation of a plan's checkpoint store (host output): 0 until the first
 * tdse_propagate_batch, then advanced by every call that rewrites the store
 * (tdse_propagate_batch and tdse_adjoint_batch on a plan created with
 * TDSE_OPT_STORE_CHECKPOINTS).  Read it right after the forward call whose
 * checkpoints a later tdse_adjoint_batch_stored should use. */
tdse_status tdse_plan_checkpoint_generation(tdse_plan plan, uint64_t* generation);

/* The gradient of tdse_adjoint_batch from the checkpoints that the forward
 * pass of generation `generation` stored: the reverse sweep only (segment
 * recompute from the stored checkpoints, then the costate steps).  E must be
 * the field of that forward pass (the checkpoints already hold its psi0).
 * Fails with TDSE_E_INVALID, before any launch, when the plan has no store
 * or the store has been rewritten since (generation mismatch).
 *   accel_bar, grad_E, sys_status   as for tdse_adjoint_batch
 * Asynchronous on `stream`, ordered after the forward pass on the same
 * stream. */
tdse_status tdse_adjoint_batch_stored(tdse_plan plan, uint64_t generation, const double* E,
                                      const double* accel_bar, double* grad_E, int32_t* sys_status,
                                      void* stream);

/* The wavefunction of every system at step index * adjoint_k, as stored by
 * the forward pass of generation `generation` on a plan created with
 * TDSE_OPT_STORE_CHECKPOINTS (0 <= index <= nt / adjoint_k), copied into a
 * ragged complex buffer (tdse_plan_psi_offsets).  With it the time-dependent
 * analyses of the wavefunction (energy distribution, ground-state and
 * volumetric populations) can be taken along a propagation.  Fails with
 * TDSE_E_INVALID, before any launch, for a stale generation.  Asynchronous
 * on `stream`. */
tdse_status tdse_plan_stored_state(tdse_plan plan, uint64_t generation, int32_t index,
                                   double* psi_out, void* stream);

/* Ground-state and volumetric populations along a propagation: the
 * analyses of the wavefunction listed in section "Microscopic Response in
 * XUV regime (TDSE)" and plotted against time in the interactive
 * interface's example.  For every system b and stored state s (the state at
 * step s * adjoint_k, 0 <= s <= nt / adjoint_k, of the forward pass of
 * generation `generation` on a plan created with TDSE_OPT_STORE_CHECKPOINTS):
 *   gs[b][s]  = |dx sum_j conj(phi_j) psi_j|^2
 *   vol[b][s] = dx sum_{|x_j| <= radius} |psi_j|^2,  x_j = (j - (n-1)/2) dx
 *   psi_ref   device, ragged complex (tdse_plan_psi_offsets): phi per system,
 *             or NULL for the plan's ground state of the system's grid size
 *   radius    half-width of the region around the nucleus (a.u.); finite
 *   gs, vol   device float64 [batch][nt / adjoint_k + 1]; either may be NULL
 * Fails with TDSE_E_INVALID, before any launch, for a plan without a store,
 * a stale generation, both outputs NULL or a non-finite radius.
 * Asynchronous on `stream`. */
tdse_status tdse_plan_populations(tdse_plan plan, uint64_t generation, const double* psi_ref,
                                  double radius, double* gs, double* vol, void* stream);

/* ------------------------------------------------- energy distribution */
/* Electron energy distribution of every system's wavefunction (section
 * "Analysing the Time-Dependent Electron Energy Density"):
 *   spectrum[b][e] = (eps/pi) dx sum_j |phi_j|^2,  (E_e - i eps - H0) phi = psi_b,
 * H0 = M2^{-1}(-D2/2) + V the field-free Hamiltonian of the solver's Numerov
 * scheme (the inverse taken in that form: ((E - i eps) M2 - A) phi = M2 psi).
 * The factor 1/(pi eps) makes int P dE = dx sum |psi|^2, so the integral
 * over E > 0 is the ionisation probability.  Applied to psi_final of a
 * propagation (or to the states of a propagation split into segments) it
 * gives the time-dependent distribution.
 *   psi       dev ragged complex (tdse_plan_psi_offsets)
 *   energies  dev [n_energy];  eps > 0 (the resolution)
 *   spectrum  dev [batch][n_energy]
 *   work      dev scratch of work_bytes bytes, 16-byte aligned: first the
 *             elimination factors shared by the systems of one size (48 n_max
 *             bytes per grid size and energy, n_max = the plan's largest n),
 *             then M2 psi of every system (16 bytes per point), then
 *             n_max bytes per (system, energy) solve in flight (the start
 *             of every 16-point group of the forward sweep, recomputed from
 *             in the backward sweep), at least 64 of them; 256k keep the GPU
 *             busy.  A wavefront solves one energy for 64 systems of one
 *             size, so a size with fewer systems leaves lanes idle.
 *             tdse_plan_energy_spectrum_work gives the size for a number of
 *             solves in flight.  Contents on return are undefined.
 * Fails with TDSE_E_INVALID, before any launch, when work is too small.
 * Asynchronous on `stream`; allocates nothing. */
tdse_status tdse_plan_energy_spectrum(tdse_plan plan, const double* psi, int32_t n_energy,
                                      const double* energies, double eps, double* spectrum,
                                      void* work, size_t work_bytes, void* stream);

/* Bytes of work tdse_plan_energy_spectrum needs for n_energy energies with
 * `lanes` (>= 64) solves in flight (host output). */
tdse_status tdse_plan_energy_spectrum_work(tdse_plan plan, int32_t n_energy, int64_t lanes,
                                           size_t* bytes);

/* Integral of energy distributions over E >= e_lo by the trapezoid rule
 * over the grid points at or above e_lo (section "Analysing the
 * Time-Dependent Electron Energy Density": with e_lo = 0 the distribution
 * of psi(t) integrates to the time-dependent ionisation probability; over
 * the whole grid, to the norm up to the Lorentzian tails):
 *   out[b] = sum over e with E_e >= e_lo and E_{e+1} >= e_lo of
 *            (E_{e+1} - E_e) (P[b][e] + P[b][e+1]) / 2
 *   energies dev [n_energy], increasing (not checked: it is device data);
 *   spectrum dev [batch][n_energy] (e.g. from tdse_plan_energy_spectrum);
 *   out dev [batch]
 * Fails with TDSE_E_INVALID before any launch for batch < 1, n_energy < 2,
 * a non-finite e_lo other than -inf, or a NULL pointer.  Asynchronous on
 * `stream`; allocates nothing. */
tdse_status tdse_energy_integral(int32_t batch, int32_t n_energy, const double* energies,
                                 const double* spectrum, double e_lo, double* out, void* stream);

/* Gabor transform of the source term (section "Physical Examples &
 * tutorials", the microscopic analysis: a joint time-frequency picture of
 * the dipole acceleration):
 *   out[b][c][w] = |dt sum_i accel[b][i] exp(-(t_i - t_c)^2 / (2 sigma^2)) exp(-i omega_w t_i)|^2
 * with t_i = i dt, t_c = t_centres[c].  Samples farther than 9.5 sigma from
 * t_c are skipped (window below 3e-20).
 *   accel dev [batch][nt+1]; t_centres dev [n_tc] (n_tc <= 65535);
 *   omegas dev [n_w] (n_w <= 1024); out dev [batch][n_tc][n_w]
 * Asynchronous on `stream`. */
tdse_status tdse_gabor(int32_t batch, int32_t nt, double dt, const double* accel, int32_t n_tc,
                       const double* t_centres, int32_t n_w, const double* omegas, double sigma,
                       double* out, void* stream);

/* ------------------------------------------------------- harmonic yield */
/* Windowed harmonic yield of each series and its gradient.  With
 * w_i = sin^2(pi i/nt), A_k = dt sum_i w_i a_i exp(-i omega_k t_i),
 * omega_k = 2 pi k/((nt+1) dt), domega = 2 pi/((nt+1) dt) and the band
 * B = {k <= (nt+1)/2 : h_lo omega0 <= omega_k <= h_hi omega0}:
 *   yield[b]        = row_weight[b] sum_{k in B} domega |A_k|^2
 *   accel_bar[b][i] = d yield[b] / d a_b,i
 * The Fourier transform of the acceleration is the quantity the paper feeds
 * to its XUV propagation (section "XUV Propagation (Spectral Approach)");
 * the Hann window keeps the periodic-boundary caveat of the appendix
 * "Microscopic source terms" small.
 *
 * tdse_harmonic_band returns the band as bins k_lo .. k_lo+nk-1 (host).
 *   accel      dev [batch][nt+1]
 *   row_weight dev double[batch] or NULL (= 1)
 *   work       dev, 2*batch*max(nk,1) doubles of scratch owned by the caller
 *   yield      dev double[batch]; accel_bar dev [batch][nt+1] or NULL
 * Asynchronous on `stream`. */
tdse_status tdse_harmonic_band(int32_t nt, double dt, double omega0, double h_lo, double h_hi,
                               int32_t* k_lo, int32_t* nk);
tdse_status tdse_harmonic_yield(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                                double h_hi, const double* accel, const double* row_weight,
                                double* work, double* yield, double* accel_bar, void* stream);

/* The band spectrum alone: amp[b][k] = A_k of row b (as above) for the bins
 * of tdse_harmonic_band, interleaved complex, dev [batch][nk].  And its
 * adjoint: given amp_bar = dl/dRe A + i dl/dIm A of a real loss l (dev
 * complex [batch][nk]), writes accel_bar[b][i] = dl/da_i
 * = dt w_i sum_k Re(conj(amp_bar_k) exp(-i omega_k t_i)) (dev [batch][nt+1]).
 * Asynchronous on `stream`. */
tdse_status tdse_band_dft(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                          double h_hi, const double* accel, double* amp, void* stream);
tdse_status tdse_band_dft_adjoint(int32_t batch, int32_t nt, double dt, double omega0, double h_lo,
                                  double h_hi, const double* amp_bar, double* accel_bar, void* stream);

/* ----------------------------------------------------------- far field */
/* Far field of the emission of a cylindrically symmetric medium, the
 * diffraction integral of a homogeneous generating medium (section "XUV
 * Propagation (Spectral Approach)", Eq. of the far field in a homogeneous
 * medium), evaluated as a direct sum over the n_rho x n_z source points
 * (rho'_i, z'_j), source p = i * n_z + j:
 *   field[m][q] = -(exp(i k z)/(4 pi)) sum_p weights[p] / d_j
 *        exp(i (k (rho'_i^2 + rho_m^2) / (2 d_j) - k z'_j)) J0(k rho_m rho'_i / d_j) amp[p][q]
 * with k = kwave[q], d_j = z_obs - z'_j and rho_m = rho_obs[m].  mu0 is left
 * to the caller; weights[p] are the quadrature weights of rho' drho' dz'
 * times the gas density.  Lengths in any one unit, kwave in its inverse.
 * Every z'_j must lie before the observation plane (d_j > 0).
 *   rho_src dev [n_rho], z_src dev [n_z], weights dev [n_rho n_z],
 *   kwave dev [nk], rho_obs dev [n_obs]   (float64)
 *   amp     dev complex [n_rho n_z][nk]   (e.g. tdse_band_dft of the systems
 *           of an n_rho x n_z focus grid, times the density)
 *   field   dev complex [n_obs][nk]
 * tdse_far_field_adjoint takes field_bar = dl/dRe E + i dl/dIm E of a real
 * loss and writes amp_bar = dl/dRe S + i dl/dIm S, the conjugate transpose
 * of the same map.  Asynchronous on `stream`. */
tdse_status tdse_far_field(int32_t n_rho, int32_t n_z, const double* rho_src, const double* z_src,
                           const double* weights, int32_t nk, const double* kwave, const double* amp,
                           int32_t n_obs, const double* rho_obs, double z_obs, double* field,
                           void* stream);
tdse_status tdse_far_field_adjoint(int32_t n_rho, int32_t n_z, const double* rho_src,
                                   const double* z_src, const double* weights, int32_t nk,
                                   const double* kwave, const double* field_bar, int32_t n_obs,
                                   const double* rho_obs, double z_obs, double* amp_bar,
                                   void* stream);

/* ----------------------------------------------------- field resampling */
/* The input interface of the solver (section "1D-TSDE Implementation
 * (CTDSE)": the driving field's time axis is shifted to start at 0 and the
 * samples are interpolated to the propagation step dt in the Fourier
 * domain).  Row b of e_coarse holds M samples of one field at spacing
 * dt_coarse, the first taken as t = 0.  With X_k their DFT and
 * M' = M dt_coarse / dt, the zero-padded inverse transform of length M'
 * (the Nyquist bin of an even M split between +M/2 and -M/2) gives
 *   e_fine[b][i] = (1/M) [X_0 + 2 sum_{0<k<M/2} Re(X_k exp(2 pi i k i/M'))
 *                         + (M even) Re(X_{M/2}) cos(pi M i / M')],
 * i = 0..nt, which reproduces the coarse samples at i = j M'/M.  Both
 * transforms are direct sums on the device (O(M^2/2) and O(M (nt+1)/2)
 * per row): meant for coarse records of up to about 10^4 samples.
 *   batch      1 .. 65535 rows;  m: 2 .. 2^20 coarse samples per row
 *   dt_coarse, dt  > 0, with M dt_coarse / dt an integer M' (to 1e-9
 *              relative) and M' >= max(m, nt + 1)
 *   e_coarse   dev [batch][m], 8-byte aligned
 *   work       dev scratch of at least 16 batch (m/2 + 1) bytes, 16-byte
 *              aligned (the DFT of every row); contents on return undefined
 *   e_fine     dev [batch][nt+1], 8-byte aligned: ready for
 *              tdse_propagate_batch
 * Fails with TDSE_E_INVALID before any launch.  Asynchronous on `stream`;
 * allocates nothing. */
tdse_status tdse_resample_field(int32_t batch, int32_t m, double dt_coarse, double dt, int32_t nt,
                                const double* e_coarse, double* work, size_t work_bytes,
                                double* e_fine, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBTDSE_H */
