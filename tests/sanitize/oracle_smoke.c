/* Runs every entry point of the CPU oracle (oracle/tdse_ref.c) on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 * any out-of-bounds access, use after free, leak or undefined operation in
 * the oracle aborts the run.  Exit status 0 means every call returned its
 * expected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int tdse_ref_grid(int n, double dx, double a, double z, double* x, double* v, double* dv);
int tdse_ref_mask(int n, double dx, double frac, double power, double* m);
int tdse_ref_propagate(int n, double dx, double dt, double a, double z, double mask_frac,
                  double mask_pow, int nt, const double* efield, const double* psi0,
                  double* accel, double* xexp, double* norm, double* psi_final);
int tdse_ref_propagate_batch(int batch, const int* n_per, const int64_t* psi_off, double dx,
                        double dt, double a, double z, double mask_frac, double mask_pow, int nt,
                        const double* efield, const double* psi0, double* accel, double* xexp,
                        double* norm, int nthreads);
int tdse_ref_ground_state(int n, double dx, double a, double z, double dtau, int max_iter,
                     double tol, double* psi_out, double* energy_out, int* iters_out);
int tdse_ref_soft_core_for_ip(double ip, int n, double dx, double dtau, double gs_tol,
                         int gs_max_iter, double tol, double a_lo, double a_hi, double* a_out,
                         double* e_out);
int tdse_ref_adjoint(int n, double dx, double dt, double a, double z, double mask_frac,
                double mask_pow, int nt, const double* efield, const double* psi0,
                const double* abar, int k, double* grad, double* accel_out);
int tdse_ref_step(int n, double dx, double dt, double a, double z, double mask_frac, double mask_pow,
             double e, double* psi);

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    const int n = 97, nt = 23;
    const double dx = 0.3, dt = 0.05, a = 1.1;
    double* x = malloc(sizeof(double) * n);
    double* v = malloc(sizeof(double) * n);
    double* dv = malloc(sizeof(double) * n);
    double* m = malloc(sizeof(double) * n);
    CHECK(tdse_ref_grid(n, dx, a, 1.0, x, v, dv) == 0);
    CHECK(tdse_ref_mask(n, dx, 0.1, 0.125, m) == 0);
    CHECK(m[0] == 0.0 && m[n - 1] == 0.0 && m[n / 2] == 1.0);
    CHECK(tdse_ref_mask(n, dx, 0.5, 0.125, m) != 0);   /* fraction out of range */
    CHECK(tdse_ref_grid(2, dx, a, 1.0, x, v, dv) != 0);  /* too few points */

    double* psi = malloc(sizeof(double) * 2 * n);
    double e = 0.0;
    int it = 0;
    CHECK(tdse_ref_ground_state(n, dx, a, 1.0, 1.0, 20000, 1e-12, psi, &e, &it) == 0);
    CHECK(e < 0.0 && it > 0);
    double a_fit = 0.0, e_fit = 0.0;
    CHECK(tdse_ref_soft_core_for_ip(0.5792, 64, 0.4, 1.0, 1e-12, 20000, 1e-9, 0.5, 3.0, &a_fit, &e_fit) == 0);
    CHECK(fabs(e_fit + 0.5792) < 1e-9);

    double* ef = malloc(sizeof(double) * (nt + 1));
    double* abar = malloc(sizeof(double) * (nt + 1));
    for (int i = 0; i <= nt; ++i) {
        ef[i] = 0.05 * sin(0.3 * i);
        abar[i] = cos(0.2 * i);
    }
    double* acc = malloc(sizeof(double) * (nt + 1));
    double* xe = malloc(sizeof(double) * (nt + 1));
    double* nr = malloc(sizeof(double) * (nt + 1));
    double* pf = malloc(sizeof(double) * 2 * n);
    CHECK(tdse_ref_propagate(n, dx, dt, a, 1.0, 0.1, 0.125, nt, ef, psi, acc, xe, nr, pf) == 0);
    CHECK(tdse_ref_propagate(n, dx, dt, a, 1.0, 0.1, 0.125, nt, ef, psi, acc, NULL, NULL, NULL) == 0);
    CHECK(tdse_ref_propagate(n, dx, dt, a, 1.0, 0.1, 0.125, 0, ef, psi, acc, xe, nr, pf) == 0);
    double* step_psi = malloc(sizeof(double) * 2 * n);
    for (int j = 0; j < 2 * n; ++j) step_psi[j] = psi[j];
    CHECK(tdse_ref_step(n, dx, dt, a, 1.0, 0.1, 0.125, 0.07, step_psi) == 0);

    double* grad = malloc(sizeof(double) * (nt + 1));
    for (int k = 1; k <= nt + 2; k += 5)
        CHECK(tdse_ref_adjoint(n, dx, dt, a, 1.0, 0.1, 0.125, nt, ef, psi, abar, k, grad, acc) == 0);
    CHECK(tdse_ref_adjoint(n, dx, dt, a, 1.0, 0.1, 0.125, nt, ef, psi, abar, 0, grad, acc) != 0);

    /* ragged batch on several threads, offsets with gaps */
    const int batch = 5;
    int ns[5] = {97, 33, 64, 97, 17};
    int64_t off[6];
    off[0] = 0;
    for (int b = 0; b < batch; ++b) off[b + 1] = off[b] + ns[b] + 3;
    double* buf = calloc((size_t)(2 * off[batch]), sizeof(double));
    for (int b = 0; b < batch; ++b)
        for (int j = 0; j < ns[b]; ++j) buf[2 * (off[b] + j)] = exp(-0.1 * (j - ns[b] / 2) * (j - ns[b] / 2));
    double* efb = malloc(sizeof(double) * batch * (nt + 1));
    for (int b = 0; b < batch; ++b)
        for (int i = 0; i <= nt; ++i) efb[b * (nt + 1) + i] = ef[i] * (1.0 + 0.1 * b);
    double* accb = malloc(sizeof(double) * batch * (nt + 1));
    double* xeb = malloc(sizeof(double) * batch * (nt + 1));
    double* nrb = malloc(sizeof(double) * batch * (nt + 1));
    CHECK(tdse_ref_propagate_batch(batch, ns, off, dx, dt, a, 1.0, 0.1, 0.125, nt, efb, buf, accb, xeb,
                              nrb, 3) == 0);
    CHECK(tdse_ref_propagate_batch(batch, ns, off, dx, dt, a, 1.0, 0.1, 0.125, nt, efb, buf, accb, NULL,
                              NULL, 8) == 0);
    CHECK(tdse_ref_propagate_batch(batch, ns, off, dx, dt, a, 1.0, 0.1, 0.125, nt, efb, buf, accb, xeb,
                              nrb, 0) != 0);

    free(x); free(v); free(dv); free(m); free(psi); free(ef); free(abar); free(acc); free(xe);
    free(nr); free(pf); free(step_psi); free(grad); free(buf); free(efb); free(accb); free(xeb);
    free(nrb);
    printf("oracle smoke: ok\n");
    return 0;
}
