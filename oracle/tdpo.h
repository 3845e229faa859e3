/*
 * tdpo.h -- interface of the plain FP64 CPU oracle (test infrastructure only;
 * the product library never includes or links this).  All arrays are host
 * arrays, row-major over the interior nodes, complex arrays interleaved
 * (C99 double complex).
 */
#ifndef TDPO_H
#define TDPO_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { TDPO_OK = 0, TDPO_ENOTCONV = 1, TDPO_EINVAL = -1, TDPO_ENOMEM = -2, TDPO_ECFL = -4 };

typedef struct tdpo_op tdpo_op;

/* nP == 0: automatic (smallest multiple of 4 above the CFL bound); nP > 0:
 * any n_P >= 3 above the bound (Table 1 then samples the field a phase
 * 2 pi q/n_P before the end, q = round(n_P/4), and solves a 2x2 system for
 * Im U); nP < 0: test hook, |nP| (a multiple of 4) used without the CFL
 * check (to exhibit instability).
 * dform 0: Im H = diag(omega R), integrator I_acd (Def. 2);
 * dform 1: Im H = omega sum_cells r_cell M_cell (r_cell = corner mean of R),
 *          integrator I_abd (Sec. 6, Def. 6), S_T^abd (Def. 7). */
int tdpo_op_create(int ndim, const long *n, double h, double omega, const double *c,
                   const double *R, const double *stiff, const double *mass, int nP,
                   int dform, tdpo_op **out);
void tdpo_op_destroy(tdpo_op *op);
/* vals = {omega_c, dt, alpha, beta, lam_bar} */
void tdpo_op_query(const tdpo_op *op, double *vals, int *nP);
void tdpo_cell_slowness(const tdpo_op *op, double *m);
void tdpo_apply_reH(const tdpo_op *op, const double *x, double *y);
void tdpo_apply_H(const tdpo_op *op, const double complex *x, double complex *y);
void tdpo_apply_K(const tdpo_op *op, const double *x, double *y);
void tdpo_apply_L(const tdpo_op *op, const double *x, double *y);
void tdpo_damping(const tdpo_op *op, double *l);
void tdpo_step(const tdpo_op *op, const double *u, const double *um, const double *f,
               double *up);
double tdpo_window(double s, double rho);
int tdpo_precond_apply(const tdpo_op *op, int T, double rho, const double complex *F,
                       double complex *U);
int tdpo_precond_apply_complex(const tdpo_op *op, int T, double rho,
                               const double complex *F, double complex *U);
/* variant 0: Table 1 preconditioner, 1: Definition 4 (complex-linear).
 * info = {iters, restarts, true relres, last Givens estimate, history length,
 *         preconditioner applications, 1 if a rejected cycle moved a variant-0
 *         solve to variant 1} */
int tdpo_gmres_solve(const tdpo_op *op, int restart, int max_iters, int T, double rho,
                     double tol, int fixed_iters, int x0_given, int variant,
                     const double complex *F, double complex *U, double *info,
                     double *history, int history_cap);
void tdpo_grad_m(const tdpo_op *op, const double complex *lam, const double complex *U,
                 double *grad_nodes);

#ifdef __cplusplus
}
#endif
#endif
