/*
 * tdse_ref.c -- plain serial CPU oracle for the microscopic step of the
 * multiscale high-harmonic-generation model of arXiv 2507.04115.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP library against an
 * independent, obviously correct implementation.  It shares no code, header,
 * table or constant with the HIP library.
 *
 * Everything is IEEE double / C99 double complex, written for readability:
 * each time step builds the Crank-Nicolson matrices from their definitions,
 * forms the right-hand side by a tridiagonal matrix-vector product and solves
 * the left-hand side with the textbook Thomas algorithm (no pivoting, no
 * precomputed factorisation, no fusion).
 *
 * Physics followed (paper sections cited by name):
 *   - Hamiltonian H = p^2/2 + V_C + x E(t), soft-core V_C = -Z/sqrt(x^2+a^2)
 *     (Sec. "Microscopic Response in XUV regime (TDSE)", Eq. Hamiltonian (a),
 *     Eq. SC potential).
 *   - Dipole acceleration <dV_C/dx + E(t)> (same section, Eq. dipole
 *     acceleration; appendix "Microscopic source terms", 1D form).
 *   - Grid [-Nx..Nx]dx, time grid from t = 0, three substeps
 *     psi^(i,1) = (M2 - i dt/2 (-D2/2 + M2 V)) psi^(i),
 *     psi^(i,2) = (M2 + i dt/2 (-D2/2 + M2 V))^-1 psi^(i,1),
 *     psi^(i+1)_j = exp(-i dt E(t_i) x_j) psi^(i,2)_j
 *     (Sec. "1D-TSDE Implementation (CTDSE)", Eqs. CN step 4, 2, 3).
 *
 * Readings where the paper is silent:
 *   - N unknowns at x_j = (j - (N-1)/2) dx, Dirichlet outside (plain
 *     truncation of the tridiagonals).
 *   - Numerov matrix M2 = I + dx^2 D2 / 12 = tridiag(1/12, 10/12, 1/12),
 *     D2 = tridiag(1, -2, 1)/dx^2.
 *   - "M2 V_C" is the matrix product M2 * diag(V).
 *   - Absorber (not in the paper): after the field substep every point is
 *     multiplied by a real mask m_j, 1 in the interior, cos(...)^power on the
 *     outer fraction of the grid at each side (a tenth of the grid each side:
 *     |x| > 0.8 x_max) and exactly 0 at the two outermost points.
 *   - Acceleration sample i uses psi^(i) and E(t_i):
 *     a_i = dx sum_j |psi_j|^2 (dV/dx)_j + E_i n_i,  n_i = dx sum_j |psi_j|^2.
 *   - Ground state: imaginary-time Crank-Nicolson (dt -> -i dtau) with
 *     renormalisation, started from exp(-x^2), stopped when successive
 *     normalised iterates differ by less than tol in the dx-weighted L2 norm.
 *   - Adjoint: exact discrete adjoint of the forward recursion, with the
 *     forward states recomputed from checkpoints.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define REF_OK 0
#define REF_EINVAL -1
#define REF_ENOMEM -2
#define REF_ENOCONV -4

static const double kPi = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Grid, potential, mask                                                     */
/* ------------------------------------------------------------------------ */

/* x_j = (j - (n-1)/2) dx;  V_j = -z / sqrt(x_j^2 + a^2);
 * dV_j = dV/dx = z x_j (x_j^2 + a^2)^(-3/2).  (Eq. SC potential.) */
int tdse_ref_grid(int n, double dx, double a, double z, double* x, double* v, double* dv)
{
    if (n < 3 || !(dx > 0.0)) return REF_EINVAL;
    for (int j = 0; j < n; ++j) {
        double xj = ((double)j - 0.5 * (double)(n - 1)) * dx;
        double s = xj * xj + a * a;
        if (x) x[j] = xj;
        if (v) v[j] = (z == 0.0) ? 0.0 : -z / sqrt(s);
        if (dv) dv[j] = (z == 0.0) ? 0.0 : z * xj / (s * sqrt(s));
    }
    return REF_OK;
}

/* Absorbing mask on the outer fraction `frac` of the grid at each side:
 * the grid spans 2 x_max, so the absorber starts at x_a = x_max - 2 frac x_max
 * (frac = 0.1: x_a = 0.8 x_max).  m = 1 for |x| <= x_a,
 * cos(pi/2 (|x|-x_a)/(x_max-x_a))^power between x_a and x_max, and 0 at
 * |x| >= x_max (the two outermost points).  frac <= 0 disables the mask (all
 * ones); frac must stay below 1/2. */
int tdse_ref_mask(int n, double dx, double frac, double power, double* m)
{
    if (n < 3 || !(dx > 0.0) || !(frac < 0.5)) return REF_EINVAL;
    double xmax = 0.5 * (double)(n - 1) * dx;
    double xa = xmax - 2.0 * frac * xmax;
    for (int j = 0; j < n; ++j) {
        double ax = fabs(((double)j - 0.5 * (double)(n - 1)) * dx);
        if (frac <= 0.0 || ax <= xa) {
            m[j] = 1.0;
        } else if (ax >= xmax) {
            m[j] = 0.0;
        } else {
            m[j] = pow(cos(0.5 * kPi * (ax - xa) / (xmax - xa)), power);
        }
    }
    return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Tridiagonal matrices of the Numerov Crank-Nicolson step                    */
/* ------------------------------------------------------------------------ */

/* A tridiagonal matrix: diag[j] = (j,j), sup[j] = (j,j+1), sub[j] = (j+1,j). */
typedef struct {
    int n;
    cplx* sub;
    cplx* diag;
    cplx* sup;
} tridiag;

static int tridiag_alloc(tridiag* t, int n)
{
    t->n = n;
    t->sub = (cplx*)calloc((size_t)n, sizeof(cplx));
    t->diag = (cplx*)calloc((size_t)n, sizeof(cplx));
    t->sup = (cplx*)calloc((size_t)n, sizeof(cplx));
    return (t->sub && t->diag && t->sup) ? REF_OK : REF_ENOMEM;
}

static void tridiag_free(tridiag* t)
{
    free(t->sub);
    free(t->diag);
    free(t->sup);
    t->sub = t->diag = t->sup = NULL;
}

/* Builds L = M2 + h A and R = M2 - h A with A = -D2/2 + M2 diag(V).
 * Real time: h = i dt / 2.  Imaginary time (dt -> -i dtau): h = dtau / 2. */
static void build_cn(int n, double dx, const double* v, cplx h, tridiag* L, tridiag* R)
{
    const double m2_diag = 10.0 / 12.0, m2_off = 1.0 / 12.0;
    const double d2_diag = -2.0 / (dx * dx), d2_off = 1.0 / (dx * dx);
    for (int j = 0; j < n; ++j) {
        /* (j,j) */
        double a_diag = -0.5 * d2_diag + m2_diag * v[j];
        L->diag[j] = m2_diag + h * a_diag;
        R->diag[j] = m2_diag - h * a_diag;
        if (j + 1 < n) {
            /* (j,j+1): column j+1 of M2 diag(V) carries V_{j+1}. */
            double a_sup = -0.5 * d2_off + m2_off * v[j + 1];
            /* (j+1,j): column j carries V_j. */
            double a_sub = -0.5 * d2_off + m2_off * v[j];
            L->sup[j] = m2_off + h * a_sup;
            R->sup[j] = m2_off - h * a_sup;
            L->sub[j] = m2_off + h * a_sub;
            R->sub[j] = m2_off - h * a_sub;
        }
    }
}

/* out = T in */
static void tridiag_matvec(const tridiag* T, const cplx* in, cplx* out)
{
    int n = T->n;
    for (int j = 0; j < n; ++j) {
        cplx s = T->diag[j] * in[j];
        if (j > 0) s += T->sub[j - 1] * in[j - 1];
        if (j + 1 < n) s += T->sup[j] * in[j + 1];
        out[j] = s;
    }
}

/* out = T^H in  (conjugate transpose: (T^H)_{jk} = conj(T_{kj})) */
static void tridiag_matvec_h(const tridiag* T, const cplx* in, cplx* out)
{
    int n = T->n;
    for (int j = 0; j < n; ++j) {
        cplx s = conj(T->diag[j]) * in[j];
        if (j > 0) s += conj(T->sup[j - 1]) * in[j - 1];
        if (j + 1 < n) s += conj(T->sub[j]) * in[j + 1];
        out[j] = s;
    }
}

/* Thomas algorithm: solves T x = rhs.  `cw` is scratch of length n. */
static void thomas(int n, const cplx* sub, const cplx* diag, const cplx* sup,
                   const cplx* rhs, cplx* x, cplx* cw)
{
    cplx den = diag[0];
    cw[0] = sup[0] / den;
    x[0] = rhs[0] / den;
    for (int j = 1; j < n; ++j) {
        den = diag[j] - sub[j - 1] * cw[j - 1];
        if (j + 1 < n) cw[j] = sup[j] / den;
        x[j] = (rhs[j] - sub[j - 1] * x[j - 1]) / den;
    }
    for (int j = n - 2; j >= 0; --j) x[j] -= cw[j] * x[j + 1];
}

/* Solves T^H x = rhs by the same algorithm on the conjugate transpose. */
static void thomas_h(const tridiag* T, const cplx* rhs, cplx* x, cplx* cw, cplx* tmp_sub,
                     cplx* tmp_diag, cplx* tmp_sup)
{
    int n = T->n;
    for (int j = 0; j < n; ++j) {
        tmp_diag[j] = conj(T->diag[j]);
        if (j + 1 < n) {
            tmp_sub[j] = conj(T->sup[j]); /* (j+1,j) of T^H = conj((j,j+1) of T) */
            tmp_sup[j] = conj(T->sub[j]); /* (j,j+1) of T^H = conj((j+1,j) of T) */
        }
    }
    thomas(n, tmp_sub, tmp_diag, tmp_sup, rhs, x, cw);
}

/* ------------------------------------------------------------------------ */
/* Observables                                                               */
/* ------------------------------------------------------------------------ */

static void observables(int n, double dx, const double* x, const double* dv, double e,
                        const cplx* psi, double* acc, double* xe, double* nrm)
{
    double s_n = 0.0, s_x = 0.0, s_v = 0.0;
    for (int j = 0; j < n; ++j) {
        double p = creal(psi[j]) * creal(psi[j]) + cimag(psi[j]) * cimag(psi[j]);
        s_n += p;
        s_x += x[j] * p;
        s_v += dv[j] * p;
    }
    if (nrm) *nrm = dx * s_n;
    if (xe) *xe = dx * s_x;
    if (acc) *acc = dx * s_v + e * dx * s_n;
}

/* ------------------------------------------------------------------------ */
/* Forward propagation                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    double dx, dt, a, z, mask_frac, mask_pow;
    double *x, *v, *dv, *m;
    tridiag L, R;
    cplx *rhs, *cw;
} ref_ctx;

static void ctx_free(ref_ctx* c)
{
    free(c->x);
    free(c->v);
    free(c->dv);
    free(c->m);
    free(c->rhs);
    free(c->cw);
    tridiag_free(&c->L);
    tridiag_free(&c->R);
}

static int ctx_init(ref_ctx* c, int n, double dx, double dt, double a, double z,
                    double mask_frac, double mask_pow)
{
    memset(c, 0, sizeof(*c));
    if (n < 3 || !(dx > 0.0) || !(dt > 0.0)) return REF_EINVAL;
    c->n = n;
    c->dx = dx;
    c->dt = dt;
    c->a = a;
    c->z = z;
    c->mask_frac = mask_frac;
    c->mask_pow = mask_pow;
    c->x = (double*)malloc(sizeof(double) * (size_t)n);
    c->v = (double*)malloc(sizeof(double) * (size_t)n);
    c->dv = (double*)malloc(sizeof(double) * (size_t)n);
    c->m = (double*)malloc(sizeof(double) * (size_t)n);
    c->rhs = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    c->cw = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!c->x || !c->v || !c->dv || !c->m || !c->rhs || !c->cw ||
        tridiag_alloc(&c->L, n) != REF_OK || tridiag_alloc(&c->R, n) != REF_OK) {
        ctx_free(c);
        return REF_ENOMEM;
    }
    tdse_ref_grid(n, dx, a, z, c->x, c->v, c->dv);
    tdse_ref_mask(n, dx, mask_frac, mask_pow, c->m);
    build_cn(n, dx, c->v, I * (0.5 * dt), &c->L, &c->R);
    return REF_OK;
}

/* One step psi^(i) -> psi^(i+1) with field sample e = E(t_i). */
static void step_forward(ref_ctx* c, double e, cplx* psi)
{
    int n = c->n;
    tridiag_matvec(&c->R, psi, c->rhs);                                      /* substep 1 */
    thomas(n, c->L.sub, c->L.diag, c->L.sup, c->rhs, psi, c->cw);           /* substep 2 */
    for (int j = 0; j < n; ++j) {
        psi[j] *= cexp(-I * (c->dt * e * c->x[j]));                          /* substep 3 */
        psi[j] *= c->m[j];                                                   /* absorber */
    }
}

/* psi0, psi_final: interleaved (re, im), n complex values.  efield: nt+1
 * samples E(t_i), t_i = i dt.  accel (required), xexp, norm: nt+1 samples;
 * xexp, norm, psi_final may be NULL. */
int tdse_ref_propagate(int n, double dx, double dt, double a, double z, double mask_frac,
                  double mask_pow, int nt, const double* efield, const double* psi0,
                  double* accel, double* xexp, double* norm, double* psi_final)
{
    if (nt < 0 || !efield || !psi0 || !accel) return REF_EINVAL;
    ref_ctx c;
    int st = ctx_init(&c, n, dx, dt, a, z, mask_frac, mask_pow);
    if (st != REF_OK) return st;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!psi) {
        ctx_free(&c);
        return REF_ENOMEM;
    }
    memcpy(psi, psi0, sizeof(cplx) * (size_t)n);
    for (int i = 0; i <= nt; ++i) {
        observables(n, dx, c.x, c.dv, efield[i], psi, &accel[i], xexp ? &xexp[i] : NULL,
                    norm ? &norm[i] : NULL);
        if (i < nt) step_forward(&c, efield[i], psi);
    }
    if (psi_final) memcpy(psi_final, psi, sizeof(cplx) * (size_t)n);
    free(psi);
    ctx_free(&c);
    return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Batched forward on host threads (used to time the oracle)                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int batch, nt;
    const int* n_per;
    const int64_t* psi_off; /* complex offsets, batch+1 */
    double dx, dt, a, z, mask_frac, mask_pow;
    const double* efield;   /* [batch][nt+1] */
    const double* psi0;
    double* accel;          /* [batch][nt+1] */
    double* xexp;
    double* norm;
    int next;
    pthread_mutex_t lock;
    int status;
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* job = (batch_job*)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int p = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (p >= job->batch) break;
        size_t row = (size_t)p * (size_t)(job->nt + 1);
        int st = tdse_ref_propagate(job->n_per[p], job->dx, job->dt, job->a, job->z, job->mask_frac,
                               job->mask_pow, job->nt, job->efield + row,
                               job->psi0 + 2 * job->psi_off[p], job->accel + row,
                               job->xexp ? job->xexp + row : NULL,
                               job->norm ? job->norm + row : NULL, NULL);
        if (st != REF_OK) {
            pthread_mutex_lock(&job->lock);
            job->status = st;
            pthread_mutex_unlock(&job->lock);
        }
    }
    return NULL;
}

int tdse_ref_propagate_batch(int batch, const int* n_per, const int64_t* psi_off, double dx,
                        double dt, double a, double z, double mask_frac, double mask_pow, int nt,
                        const double* efield, const double* psi0, double* accel, double* xexp,
                        double* norm, int nthreads)
{
    if (batch < 0 || nthreads < 1 || !n_per || !psi_off) return REF_EINVAL;
    batch_job job = {batch, nt, n_per, psi_off, dx, dt, a, z, mask_frac, mask_pow,
                     efield, psi0, accel, xexp, norm, 0, PTHREAD_MUTEX_INITIALIZER, REF_OK};
    if (nthreads > batch) nthreads = batch > 0 ? batch : 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return REF_ENOMEM;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, &job);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    return job.status;
}

/* ------------------------------------------------------------------------ */
/* Ground state by imaginary-time relaxation                                 */
/* ------------------------------------------------------------------------ */

/* H psi = M2^{-1} (-D2/2 psi) + V psi  (the Numerov Hamiltonian). */
static void apply_h(int n, double dx, const double* v, const cplx* psi, cplx* out, cplx* tmp,
                    cplx* cw, cplx* m2sub, cplx* m2diag, cplx* m2sup)
{
    for (int j = 0; j < n; ++j) {
        cplx lap = -2.0 * psi[j];
        if (j > 0) lap += psi[j - 1];
        if (j + 1 < n) lap += psi[j + 1];
        tmp[j] = -0.5 * lap / (dx * dx);
    }
    thomas(n, m2sub, m2diag, m2sup, tmp, out, cw);
    for (int j = 0; j < n; ++j) out[j] += v[j] * psi[j];
}

static double dx_norm2(int n, double dx, const cplx* psi)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += creal(psi[j] * conj(psi[j]));
    return dx * s;
}

/* psi_out: interleaved complex (imaginary parts are zero); energy_out:
 * Rayleigh quotient dx <psi, H psi>.  Returns REF_ENOCONV when max_iter
 * iterations do not bring the change of the normalised iterate below tol. */
int tdse_ref_ground_state(int n, double dx, double a, double z, double dtau, int max_iter,
                     double tol, double* psi_out, double* energy_out, int* iters_out)
{
    if (n < 3 || !(dx > 0.0) || !(dtau > 0.0) || max_iter < 1 || !psi_out) return REF_EINVAL;
    double *x = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    cplx *psi = malloc(sizeof(cplx) * n), *rhs = malloc(sizeof(cplx) * n),
         *nxt = malloc(sizeof(cplx) * n), *cw = malloc(sizeof(cplx) * n),
         *hpsi = malloc(sizeof(cplx) * n);
    cplx *m2sub = malloc(sizeof(cplx) * n), *m2diag = malloc(sizeof(cplx) * n),
         *m2sup = malloc(sizeof(cplx) * n);
    tridiag L = {0}, R = {0};
    int st = REF_OK;
    if (!x || !v || !psi || !rhs || !nxt || !cw || !hpsi || !m2sub || !m2diag || !m2sup ||
        tridiag_alloc(&L, n) != REF_OK || tridiag_alloc(&R, n) != REF_OK) {
        st = REF_ENOMEM;
        goto done;
    }
    tdse_ref_grid(n, dx, a, z, x, v, NULL);
    build_cn(n, dx, v, 0.5 * dtau, &L, &R);
    for (int j = 0; j < n; ++j) {
        m2sub[j] = 1.0 / 12.0;
        m2diag[j] = 10.0 / 12.0;
        m2sup[j] = 1.0 / 12.0;
    }
    for (int j = 0; j < n; ++j) psi[j] = exp(-x[j] * x[j]);
    double s = 1.0 / sqrt(dx_norm2(n, dx, psi));
    for (int j = 0; j < n; ++j) psi[j] *= s;

    int it = 0, converged = 0;
    while (it < max_iter) {
        tridiag_matvec(&R, psi, rhs);
        thomas(n, L.sub, L.diag, L.sup, rhs, nxt, cw);
        s = 1.0 / sqrt(dx_norm2(n, dx, nxt));
        double d = 0.0;
        for (int j = 0; j < n; ++j) {
            nxt[j] *= s;
            cplx diff = nxt[j] - psi[j];
            d += creal(diff * conj(diff));
            psi[j] = nxt[j];
        }
        ++it;
        if (sqrt(dx * d) < tol) {
            converged = 1;
            break;
        }
    }
    apply_h(n, dx, v, psi, hpsi, rhs, cw, m2sub, m2diag, m2sup);
    double e = 0.0;
    for (int j = 0; j < n; ++j) e += creal(conj(psi[j]) * hpsi[j]);
    e *= dx;
    if (energy_out) *energy_out = e;
    if (iters_out) *iters_out = it;
    memcpy(psi_out, psi, sizeof(cplx) * (size_t)n);
    if (!converged) st = REF_ENOCONV;
done:
    free(x);
    free(v);
    free(psi);
    free(rhs);
    free(nxt);
    free(cw);
    free(hpsi);
    free(m2sub);
    free(m2diag);
    free(m2sup);
    tridiag_free(&L);
    tridiag_free(&R);
    return st;
}

/* Soft-core parameter: bisection on a in [a_lo, a_hi] for E_g(a) = -ip
 * (E_g increases with a).  Stops when |E_g(a) + ip| < tol or after 100
 * halvings. */
int tdse_ref_soft_core_for_ip(double ip, int n, double dx, double dtau, double gs_tol,
                         int gs_max_iter, double tol, double a_lo, double a_hi, double* a_out,
                         double* e_out)
{
    if (!(ip > 0.0) || !(a_hi > a_lo) || !a_out) return REF_EINVAL;
    double* psi = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!psi) return REF_ENOMEM;
    double e_lo, e_hi, e_mid = 0.0, mid = a_lo;
    int st = tdse_ref_ground_state(n, dx, a_lo, 1.0, dtau, gs_max_iter, gs_tol, psi, &e_lo, NULL);
    if (st == REF_OK)
        st = tdse_ref_ground_state(n, dx, a_hi, 1.0, dtau, gs_max_iter, gs_tol, psi, &e_hi, NULL);
    if (st != REF_OK) goto done;
    if (!(e_lo < -ip && e_hi > -ip)) {
        st = REF_EINVAL;
        goto done;
    }
    st = REF_ENOCONV;
    for (int k = 0; k < 100; ++k) {
        mid = 0.5 * (a_lo + a_hi);
        int s2 = tdse_ref_ground_state(n, dx, mid, 1.0, dtau, gs_max_iter, gs_tol, psi, &e_mid, NULL);
        if (s2 != REF_OK) {
            st = s2;
            break;
        }
        if (fabs(e_mid + ip) < tol) {
            st = REF_OK;
            break;
        }
        if (e_mid < -ip)
            a_lo = mid;
        else
            a_hi = mid;
    }
    *a_out = mid;
    if (e_out) *e_out = e_mid;
done:
    free(psi);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the forward recursion                                 */
/* ------------------------------------------------------------------------ */

/* Given abar_i = dl/da_i for a loss l(a_0..a_nt), returns
 * grad_i = dl/dE_i for i = 0..nt.  Forward recursion:
 *   psi^{i+1} = D_i L^{-1} R psi^i,  D_i = diag(m_j exp(-i dt E_i x_j)),
 *   a_i = dx sum_j |psi^i_j|^2 (dV_j + E_i).
 * Costate (dl = Re sum_j conj(lam_j) dpsi_j):
 *   lam^{nt} = 2 abar_nt dx (dV + E_nt) psi^nt,
 *   lam^i = R^H L^{-H} D_i^H lam^{i+1} + 2 abar_i dx (dV + E_i) psi^i,
 *   grad_i = abar_i n_i + dt sum_j x_j Im(conj(lam^{i+1}_j) psi^{i+1}_j)  (i < nt),
 *   grad_nt = abar_nt n_nt.
 * Forward states are recomputed segment by segment from checkpoints stored
 * every `k` steps (k = 1 stores every state).  accel_out may be NULL. */
int tdse_ref_adjoint(int n, double dx, double dt, double a, double z, double mask_frac,
                double mask_pow, int nt, const double* efield, const double* psi0,
                const double* abar, int k, double* grad, double* accel_out)
{
    if (nt < 0 || k < 1 || !efield || !psi0 || !abar || !grad) return REF_EINVAL;
    ref_ctx c;
    int st = ctx_init(&c, n, dx, dt, a, z, mask_frac, mask_pow);
    if (st != REF_OK) return st;
    int nseg = nt / k + 1; /* checkpoints at i = 0, k, 2k, ... <= nt */
    cplx* ckpt = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)nseg);
    cplx* seg = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)(k + 1));
    cplx* lam = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* mu = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* nu = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* cw = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* hs = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* hd = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* hu = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)(nt + 1));
    if (!ckpt || !seg || !lam || !mu || !nu || !cw || !hs || !hd || !hu || !nrm) {
        st = REF_ENOMEM;
        goto done;
    }
    /* Forward pass: outputs, norms and checkpoints. */
    {
        cplx* psi = seg;
        memcpy(psi, psi0, sizeof(cplx) * (size_t)n);
        for (int i = 0; i <= nt; ++i) {
            if (i % k == 0) memcpy(ckpt + (size_t)(i / k) * n, psi, sizeof(cplx) * (size_t)n);
            double acc;
            observables(n, dx, c.x, c.dv, efield[i], psi, &acc, NULL, &nrm[i]);
            if (accel_out) accel_out[i] = acc;
            if (i < nt) step_forward(&c, efield[i], psi);
        }
    }
    /* Backward pass, one segment [s0, s1] at a time, last segment first. */
    int have_lam = 0;
    for (int sidx = nseg - 1; sidx >= 0; --sidx) {
        int s0 = sidx * k;
        int s1 = s0 + k < nt ? s0 + k : nt;
        /* recompute psi^{s0..s1} into seg[0..s1-s0] */
        memcpy(seg, ckpt + (size_t)sidx * n, sizeof(cplx) * (size_t)n);
        for (int i = s0; i < s1; ++i) {
            cplx* dst = seg + (size_t)(i - s0 + 1) * n;
            memcpy(dst, seg + (size_t)(i - s0) * n, sizeof(cplx) * (size_t)n);
            step_forward(&c, efield[i], dst);
        }
        if (!have_lam) {
            /* i = nt lies in this (last) segment */
            const cplx* psi_nt = seg + (size_t)(nt - s0) * n;
            for (int j = 0; j < n; ++j)
                lam[j] = 2.0 * abar[nt] * dx * (c.dv[j] + efield[nt]) * psi_nt[j];
            grad[nt] = abar[nt] * nrm[nt];
            have_lam = 1;
        }
        for (int i = s1 - 1; i >= s0; --i) {
            const cplx* psi_i = seg + (size_t)(i - s0) * n;
            const cplx* psi_ip1 = seg + (size_t)(i - s0 + 1) * n;
            double g = 0.0;
            for (int j = 0; j < n; ++j) g += c.x[j] * cimag(conj(lam[j]) * psi_ip1[j]);
            grad[i] = abar[i] * nrm[i] + dt * g;
            for (int j = 0; j < n; ++j)
                mu[j] = c.m[j] * cexp(I * (dt * efield[i] * c.x[j])) * lam[j]; /* D_i^H */
            thomas_h(&c.L, mu, nu, cw, hs, hd, hu);                            /* L^{-H} */
            tridiag_matvec_h(&c.R, nu, lam);                                    /* R^H */
            for (int j = 0; j < n; ++j)
                lam[j] += 2.0 * abar[i] * dx * (c.dv[j] + efield[i]) * psi_i[j];
        }
    }
done:
    free(ckpt);
    free(seg);
    free(lam);
    free(mu);
    free(nu);
    free(cw);
    free(hs);
    free(hd);
    free(hu);
    free(nrm);
    ctx_free(&c);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Single step (exposed for the dense-matrix pin)                             */
/* ------------------------------------------------------------------------ */

int tdse_ref_step(int n, double dx, double dt, double a, double z, double mask_frac, double mask_pow,
             double e, double* psi)
{
    ref_ctx c;
    int st = ctx_init(&c, n, dx, dt, a, z, mask_frac, mask_pow);
    if (st != REF_OK) return st;
    step_forward(&c, e, (cplx*)psi);
    ctx_free(&c);
    return REF_OK;
}
