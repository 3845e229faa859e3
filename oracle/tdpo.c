/*
 * tdpo.c -- plain, slow FP64 CPU oracle of the time-domain preconditioned
 * Helmholtz solver (Stolk, "A time-domain preconditioner for the Helmholtz
 * equation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library: every formula
 * below is written out again from the paper.
 *
 * What it computes (each function cites the passage it follows):
 *   H        matrix-free, in the cell ("quasi finite element") form of
 *            Appendix A: Re H = sum over cells of
 *            h^-2 S_{Delta(b,g)} - omega^2 m_cell M_{Delta(b,g)},
 *            Im H = diag(omega R)                          (Sec. 1 eq. 3,
 *            Sec. 3.2, App. A, Dirichlet as in Sec. 3.1).
 *   params   omega_c, Delta t, alpha, beta from Sec. 2.2 (eqs. for A, B,
 *            omega and the CFL bound) and Prop. 1.
 *   step     the frequency-adapted central-difference integrator I_acd of
 *            Definition 2.
 *   P F      the real-field algorithm of Table 1 (Sec. 2.3), window of
 *            Sec. 2.3 (sine-square taper, parameter rho).
 *   GMRES    left-preconditioned restarted GMRES (Sec. 2.4) with modified
 *            Gram-Schmidt and complex Givens rotations.
 *   grad     dL/dm for the adjoint form: dH/dm_cell = -omega^2 M_cell.
 *
 * Readings where the paper is silent (listed with reasons in the design
 * notes): the 2-D/3-D cell tables are supplied by the caller; cell slowness
 * m = 2^-d * sum of 1/c^2 over the cell's corners with out-of-box corners
 * clamped to the nearest interior node; omega_c = omega * sqrt(max m);
 * lambda_max(A) is bounded by h^-2 sup_theta S(theta) + omega_c^2 with the
 * supremum sampled on a uniform theta grid; n_P is the smallest multiple of 4
 * strictly above pi / arcsin(omega_c / sqrt(lambda_bar)).
 *
 * Parity pins: every function here is pinned by the not-gpu tests
 * (sine-mode eigenvalues, LU, energy identity, harmonic invariance, Green's
 * function sums, window values, finite differences).
 */
#include "tdpo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct tdpo_op {
    int d;
    long n[3];
    long N;
    long nc[3];   /* cells per axis: n_a + 1 (lower corners -1 .. n_a-1) */
    long Nc;
    double h, omega;
    double S[4], M[4];
    double *mcell;  /* [Nc] cell slowness */
    double *R;      /* [N]  node damping (Im H = omega R when dform = 0) */
    int dform;      /* 0: diagonal Im H (I_acd); 1: cell damping Im H = omega sum r_a M (I_abd) */
    double *rcell;  /* [Nc] cell damping (dform 1) */
    double lam_im;  /* upper bound of lambda_max(Im H) (dform 1) */
    double omega_c, lam_bar, dt, alpha, beta;
    int nP;
};

/* ------------------------------------------------------------------ */
/* index helpers                                                       */

static void node_coords(const tdpo_op *op, long idx, long *i)
{
    for (int a = op->d - 1; a >= 0; --a) {
        i[a] = idx % op->n[a];
        idx /= op->n[a];
    }
}

/* linear index of node i, or -1 if i lies outside the interior box */
static long node_index(const tdpo_op *op, const long *i)
{
    long idx = 0;
    for (int a = 0; a < op->d; ++a) {
        if (i[a] < 0 || i[a] >= op->n[a]) return -1;
        idx = idx * op->n[a] + i[a];
    }
    return idx;
}

/* cell with lower corner alpha (each alpha_a in -1 .. n_a-1) */
static long cell_index(const tdpo_op *op, const long *alpha)
{
    long idx = 0;
    for (int a = 0; a < op->d; ++a) idx = idx * op->nc[a] + (alpha[a] + 1);
    return idx;
}

static void cell_coords(const tdpo_op *op, long idx, long *alpha)
{
    for (int a = op->d - 1; a >= 0; --a) {
        alpha[a] = idx % op->nc[a] - 1;
        idx /= op->nc[a];
    }
}

static long clamp_node(const tdpo_op *op, const long *i)
{
    long j[3];
    for (int a = 0; a < op->d; ++a) {
        j[a] = i[a] < 0 ? 0 : (i[a] >= op->n[a] ? op->n[a] - 1 : i[a]);
    }
    return node_index(op, j);
}

/* corner offset e (bit a of mask = e_a) */
static void corner_offset(int d, int mask, long *e)
{
    for (int a = 0; a < d; ++a) e[a] = (mask >> a) & 1;
}

static int delta_class(int d, int m1, int m2)
{
    int s = 0;
    for (int a = 0; a < d; ++a) s += ((m1 >> a) & 1) != ((m2 >> a) & 1);
    return s;
}

/* ------------------------------------------------------------------ */
/* setup                                                               */

/* Stiffness symbol S(theta) of the assembled constant-coefficient stencil:
 * the offset o in {-1,0,1}^d couples to 2^(d-|o|) cells, each with the class
 * |o|_1 entry of the cell table. */
static double stiffness_symbol(const tdpo_op *op, const double *theta)
{
    double s = 0.0;
    int noff = 1;
    for (int a = 0; a < op->d; ++a) noff *= 3;
    for (int k = 0; k < noff; ++k) {
        int t = k, cls = 0;
        double ph = 0.0;
        for (int a = 0; a < op->d; ++a) {
            int o = t % 3 - 1;
            t /= 3;
            cls += o != 0;
            ph += o * theta[a];
        }
        s += ldexp(op->S[cls], op->d - cls) * cos(ph);
    }
    return s;
}

/* Sec. 6.1's stability condition 4I - K - 2L > 0 for I_abd with
 * theta = omega dt, using the bounds lam_s >= lambda_max(Re H) (stiffness part)
 * and lam_im >= lambda_max(Im H):
 *   (theta^2/alpha)(lam_s/omega^2 + 1) + (theta beta/alpha)(1 + cos theta) lam_im/omega^2 < 4,
 * with omega^2 = kmax2 + (beta/theta)(1 - cos theta) lam_im (K >= 0).  The printed
 * full inequality drops the factor theta of its second term; it follows from K
 * and L of Def. 6 as written, and the section's stronger inequality keeps it. */
static int abd_stable(double theta, double kmax2, double lam_s, double lam_im, double *w2out)
{
    double sh = sin(theta / 2.0);
    double alpha = theta * theta / (4.0 * sh * sh), beta = theta / sin(theta);
    double w2 = kmax2 + beta / theta * (1.0 - cos(theta)) * lam_im;
    double lhs = theta * theta / alpha * (lam_s / w2 + 1.0) +
                 theta * beta / alpha * (1.0 + cos(theta)) * lam_im / w2;
    if (w2out) *w2out = w2;
    return lhs < 4.0;
}

int tdpo_op_create(int ndim, const long *n, double h, double omega,
                   const double *c, const double *R,
                   const double *stiff, const double *mass, int nP, int dform,
                   tdpo_op **out)
{
    *out = NULL;
    if (ndim != 2 && ndim != 3) return TDPO_EINVAL;
    if (dform != 0 && dform != 1) return TDPO_EINVAL;
    if (!(h > 0.0) || !(omega > 0.0) || !c || !stiff || !mass) return TDPO_EINVAL;
    tdpo_op *op = calloc(1, sizeof(*op));
    if (!op) return TDPO_ENOMEM;
    op->d = ndim;
    op->N = 1;
    op->Nc = 1;
    for (int a = 0; a < 3; ++a) {
        op->n[a] = a < ndim ? n[a] : 1;
        op->nc[a] = a < ndim ? n[a] + 1 : 1;
    }
    for (int a = 0; a < ndim; ++a) {
        if (n[a] < 1) { free(op); return TDPO_EINVAL; }
        op->N *= op->n[a];
        op->Nc *= op->nc[a];
    }
    op->h = h;
    op->omega = omega;
    for (int s = 0; s <= ndim; ++s) { op->S[s] = stiff[s]; op->M[s] = mass[s]; }
    op->mcell = malloc(sizeof(double) * op->Nc);
    op->R = malloc(sizeof(double) * op->N);
    if (!op->mcell || !op->R) { tdpo_op_destroy(op); return TDPO_ENOMEM; }
    for (long i = 0; i < op->N; ++i) {
        if (!(c[i] > 0.0)) { tdpo_op_destroy(op); return TDPO_EINVAL; }
        double r = R ? R[i] : 0.0;
        if (!(r >= 0.0)) { tdpo_op_destroy(op); return TDPO_EINVAL; }
        op->R[i] = r;
    }

    /* App. A: k constant per cell; here m_cell = mean over corners of 1/c^2 */
    double mmax = 0.0;
    int ncorner = 1 << ndim;
    for (long q = 0; q < op->Nc; ++q) {
        long alpha[3], corner[3], e[3];
        cell_coords(op, q, alpha);
        double s = 0.0;
        for (int k = 0; k < ncorner; ++k) {
            corner_offset(ndim, k, e);
            for (int a = 0; a < ndim; ++a) corner[a] = alpha[a] + e[a];
            double cv = c[clamp_node(op, corner)];
            s += 1.0 / (cv * cv);
        }
        op->mcell[q] = s / ncorner;
        if (op->mcell[q] > mmax) mmax = op->mcell[q];
    }

    /* Sec. 2.2: omega_c = sqrt(-lambda_min(Re H)) bounded by k_max (App. A) */
    op->omega_c = omega * sqrt(mmax);
    op->dform = dform;
    if (dform == 1) {
        /* cell damping: mean of R over the cell's corners (clamped, as for m);
         * Im H = omega sum_a r_a M_a has lambda_max <= omega max r (App. A bound
         * of the assembled mass, lambda_max <= 1) */
        op->rcell = malloc(sizeof(double) * op->Nc);
        if (!op->rcell) { tdpo_op_destroy(op); return TDPO_ENOMEM; }
        double rmax = 0.0;
        for (long q = 0; q < op->Nc; ++q) {
            long alpha[3], corner[3], e[3];
            cell_coords(op, q, alpha);
            double s = 0.0;
            for (int k = 0; k < ncorner; ++k) {
                corner_offset(ndim, k, e);
                for (int a = 0; a < ndim; ++a) corner[a] = alpha[a] + e[a];
                s += op->R[clamp_node(op, corner)];
            }
            op->rcell[q] = s / ncorner;
            if (op->rcell[q] > rmax) rmax = op->rcell[q];
        }
        op->lam_im = omega * rmax;
    }

    /* sup of the stiffness symbol sampled on a uniform grid of [0, pi]^d */
    const int G = ndim == 2 ? 201 : 101;   /* both include 0 and pi */
    double smax = 0.0;
    long total = 1;
    for (int a = 0; a < ndim; ++a) total *= G;
    for (long k = 0; k < total; ++k) {
        double th[3];
        long t = k;
        for (int a = 0; a < ndim; ++a) { th[a] = M_PI * (double)(t % G) / (G - 1); t /= G; }
        double s = stiffness_symbol(op, th);
        if (s > smax) smax = s;
    }
    if (dform == 1) {
        /* Sec. 6.1: n_P = 2 pi / theta, the smallest multiple of 4 for which the
         * stability condition holds; omega from the K >= 0 condition */
        double kmax2 = op->omega_c * op->omega_c, lam_s = smax / (h * h), w2 = 0.0;
        if (nP == 0) {
            for (nP = 4; nP <= (1 << 22); nP += 4)
                if (abd_stable(2.0 * M_PI / nP, kmax2, lam_s, op->lam_im, NULL)) break;
            if (nP > (1 << 22)) { tdpo_op_destroy(op); return TDPO_ECFL; }
        } else if (nP < 0) {
            nP = -nP;
            if (nP % 4) { tdpo_op_destroy(op); return TDPO_EINVAL; }
        } else if (nP < 3 || !abd_stable(2.0 * M_PI / nP, kmax2, lam_s, op->lam_im, NULL)) {
            tdpo_op_destroy(op);
            return TDPO_ECFL;
        }
        double theta = 2.0 * M_PI / nP;
        abd_stable(theta, kmax2, lam_s, op->lam_im, &w2);
        op->nP = nP;
        op->omega_c = sqrt(w2);
        op->dt = theta / op->omega_c;
        double sh = sin(theta / 2.0);
        op->alpha = theta * theta / (4.0 * sh * sh);
        op->beta = theta / sin(theta);
        op->lam_bar = lam_s + w2;
        *out = op;
        return TDPO_OK;
    }
    op->lam_bar = smax / (h * h) + op->omega_c * op->omega_c;

    /* CFL bound of Sec. 2.2: Delta t < (2/omega) arcsin(omega/sqrt(lambda_max(A))),
     * i.e. n_P = 2 pi/(omega Delta t) > pi / arcsin(omega/sqrt(lambda_max(A))) */
    double nmin = M_PI / asin(op->omega_c / sqrt(op->lam_bar));
    if (nP == 0) {
        nP = 4 * ((int)floor(nmin / 4.0) + 1);
    } else if (nP < 0) {
        nP = -nP;   /* test hook: accept any n_P (multiple of 4) without the CFL check */
        if (nP % 4) { tdpo_op_destroy(op); return TDPO_EINVAL; }
    } else if (nP < 3 || !((double)nP > nmin)) {
        tdpo_op_destroy(op);
        return TDPO_ECFL;
    }
    op->nP = nP;
    op->dt = 2.0 * M_PI / (op->omega_c * nP);

    /* Prop. 1 */
    double wdt = op->omega_c * op->dt;
    double sh = sin(wdt / 2.0);
    op->alpha = wdt * wdt / (4.0 * sh * sh);
    op->beta = wdt / sin(wdt);
    *out = op;
    return TDPO_OK;
}

void tdpo_op_destroy(tdpo_op *op)
{
    if (!op) return;
    free(op->mcell);
    free(op->R);
    free(op->rcell);
    free(op);
}

void tdpo_op_query(const tdpo_op *op, double *vals, int *nP)
{
    vals[0] = op->omega_c;
    vals[1] = op->dt;
    vals[2] = op->alpha;
    vals[3] = op->beta;
    vals[4] = op->lam_bar;
    *nP = op->nP;
}

void tdpo_cell_slowness(const tdpo_op *op, double *m)
{
    memcpy(m, op->mcell, sizeof(double) * op->Nc);
}

/* ------------------------------------------------------------------ */
/* operators                                                           */

/* (Re H x)_b = sum over cells a containing b, over corners g of a:
 *              (h^-2 S_{Delta(b,g)} - omega^2 m_a M_{Delta(b,g)}) x_g,
 * with x_g = 0 for g outside the interior (Dirichlet).  Real vector x. */
static double reH_row(const tdpo_op *op, const double *x, long b)
{
    long ib[3], alpha[3], e[3], g[3];
    node_coords(op, b, ib);
    int d = op->d, nk = 1 << d;
    double hm2 = 1.0 / (op->h * op->h), w2 = op->omega * op->omega;
    double y = 0.0;
    for (int kb = 0; kb < nk; ++kb) {           /* b is corner kb of cell a */
        corner_offset(d, kb, e);
        for (int a = 0; a < d; ++a) alpha[a] = ib[a] - e[a];
        double mc = op->mcell[cell_index(op, alpha)];
        for (int kg = 0; kg < nk; ++kg) {
            corner_offset(d, kg, e);
            for (int a = 0; a < d; ++a) g[a] = alpha[a] + e[a];
            long gi = node_index(op, g);
            if (gi < 0) continue;
            int s = delta_class(d, kb, kg);
            y += (hm2 * op->S[s] - w2 * mc * op->M[s]) * x[gi];
        }
    }
    return y;
}

/* (Im H x)_b for the cell damping (dform 1): omega sum over cells a containing
 * b, over corners g of a, of r_a M_{Delta(b,g)} x_g (Sec. 6: non-diagonal B);
 * omega R_b x_b for the diagonal damping. */
static double imH_row(const tdpo_op *op, const double *x, long b)
{
    if (op->dform == 0) return op->omega * op->R[b] * x[b];
    long ib[3], alpha[3], e[3], g[3];
    node_coords(op, b, ib);
    int d = op->d, nk = 1 << d;
    double y = 0.0;
    for (int kb = 0; kb < nk; ++kb) {
        corner_offset(d, kb, e);
        for (int a = 0; a < d; ++a) alpha[a] = ib[a] - e[a];
        double rc = op->rcell[cell_index(op, alpha)];
        for (int kg = 0; kg < nk; ++kg) {
            corner_offset(d, kg, e);
            for (int a = 0; a < d; ++a) g[a] = alpha[a] + e[a];
            long gi = node_index(op, g);
            if (gi < 0) continue;
            y += rc * op->M[delta_class(d, kb, kg)] * x[gi];
        }
    }
    return op->omega * y;
}

void tdpo_apply_reH(const tdpo_op *op, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (long b = 0; b < op->N; ++b) y[b] = reH_row(op, x, b);
}

/* H x = Re H x + i omega R x  (complex x stored as interleaved re/im pairs) */
void tdpo_apply_H(const tdpo_op *op, const double complex *x, double complex *y)
{
    double *xr = malloc(sizeof(double) * op->N), *xi = malloc(sizeof(double) * op->N);
    for (long b = 0; b < op->N; ++b) { xr[b] = creal(x[b]); xi[b] = cimag(x[b]); }
#pragma omp parallel for schedule(static)
    for (long b = 0; b < op->N; ++b) {
        double yr = reH_row(op, xr, b) - imH_row(op, xi, b);
        double yi = reH_row(op, xi, b) + imH_row(op, xr, b);
        y[b] = yr + I * yi;
    }
    free(xr);
    free(xi);
}

/* K x = (dt^2/alpha) A x, A = Re H + omega_c^2 I                 (Def. 2)
 * dform 1: K x = (dt^2/alpha) A x - (dt beta (1 - cos(omega dt))/alpha) B x,
 *          B = Im H / omega                                      (Def. 6) */
void tdpo_apply_K(const tdpo_op *op, const double *x, double *y)
{
    double s = op->dt * op->dt / op->alpha, wc2 = op->omega_c * op->omega_c;
    double kb = op->dt * op->beta * (1.0 - cos(op->omega_c * op->dt)) / op->alpha / op->omega_c;
#pragma omp parallel for schedule(static)
    for (long b = 0; b < op->N; ++b) {
        y[b] = s * (reH_row(op, x, b) + wc2 * x[b]);
        if (op->dform == 1) y[b] -= kb * imH_row(op, x, b);
    }
}

/* L x = (beta dt/alpha) B x, B = Im H / omega_c           (Defs. 2 and 6) */
void tdpo_apply_L(const tdpo_op *op, const double *x, double *y)
{
    double lb = op->beta * op->dt / op->alpha / op->omega_c;
#pragma omp parallel for schedule(static)
    for (long b = 0; b < op->N; ++b) y[b] = lb * imH_row(op, x, b);
}

/* diagonal of L = (beta dt/alpha) B, B = omega_c^-1 Im H = omega R / omega_c */
void tdpo_damping(const tdpo_op *op, double *l)
{
    double s = op->beta * op->dt / op->alpha;
    for (long b = 0; b < op->N; ++b) l[b] = s * op->omega * op->R[b] / op->omega_c;
}

/* One step of I_acd (Def. 2):
 * u+ = (I + L/2)^-1 ((2 - K) u - (I - L/2) u- + g),  g = (dt^2/alpha) f */
void tdpo_step(const tdpo_op *op, const double *u, const double *um, const double *f,
               double *up)
{
    double s = op->dt * op->dt / op->alpha, wc2 = op->omega_c * op->omega_c;
    if (op->dform == 1) {
        /* I_abd (Def. 6): u+ = (2 - K - L) u - (I - L) u- + g */
        double kb = op->dt * op->beta * (1.0 - cos(op->omega_c * op->dt)) / op->alpha / op->omega_c;
        double lb = op->beta * op->dt / op->alpha / op->omega_c;
#pragma omp parallel for schedule(static)
        for (long b = 0; b < op->N; ++b) {
            double iu = imH_row(op, u, b);
            double Ku = s * (reH_row(op, u, b) + wc2 * u[b]) - kb * iu;
            double Lu = lb * iu, Lum = lb * imH_row(op, um, b);
            up[b] = 2.0 * u[b] - Ku - Lu - (um[b] - Lum) + s * (f ? f[b] : 0.0);
        }
        return;
    }
    double ls = op->beta * op->dt / op->alpha;
#pragma omp parallel for schedule(static)
    for (long b = 0; b < op->N; ++b) {
        double Ku = s * (reH_row(op, u, b) + wc2 * u[b]);
        double l = ls * op->omega * op->R[b] / op->omega_c;
        double rhs = 2.0 * u[b] - Ku - (1.0 - 0.5 * l) * um[b] + s * (f ? f[b] : 0.0);
        up[b] = rhs / (1.0 + 0.5 * l);
    }
}

/* Sec. 2.3: sine-square taper, chi = 1 on |s| <= 1-rho, 0 for |s| >= 1 */
double tdpo_window(double s, double rho)
{
    double a = fabs(s);
    if (a >= 1.0) return 0.0;
    if (a <= 1.0 - rho) return 1.0;
    double v = sin(M_PI * (1.0 - a) / (2.0 * rho));
    return v * v;
}

/* Table 1: U = S_T F with real fields.  rho <= 0 means "ramp over one
 * period" (Sec. 5.1), i.e. rho = 1/T. */
int tdpo_precond_apply(const tdpo_op *op, int T, double rho, const double complex *F,
                       double complex *U)
{
    if (T < 1 || op->dform != 0) return TDPO_EINVAL;   /* Table 1 runs I_acd */
    if (rho <= 0.0) rho = 1.0 / T;
    if (rho > 1.0) return TDPO_EINVAL;
    long N = op->N;
    int nP = op->nP;
    /* the second sample lies q steps (phase phi = 2 pi q / n_P) before the end:
     * u_{N_s - q} = cos(phi) Re U + sin(phi) Im U, so Im U comes from a 2x2 solve
     * with Re U = u_{N_s}; for 4 | n_P, q = n_P/4 and Im U = u_{N_s - q} (Table 1) */
    int q = nP % 4 == 0 ? nP / 4 : (nP + 2) / 4;
    long Ns = (long)T * nP, jsnap = Ns - q;
    double *um = calloc(N, sizeof(double)), *u = calloc(N, sizeof(double));
    double *up = malloc(sizeof(double) * N), *f = malloc(sizeof(double) * N);
    double *snap = malloc(sizeof(double) * N);
    if (!um || !u || !up || !f || !snap) {
        free(um); free(u); free(up); free(f); free(snap);
        return TDPO_ENOMEM;
    }
    for (long j = 0; j < Ns; ++j) {
        double chi = tdpo_window(1.0 - (double)j / (double)Ns, rho);
        double cs = cos(2.0 * M_PI * j / nP), sn = sin(2.0 * M_PI * j / nP);
        for (long b = 0; b < N; ++b) f[b] = chi * (cs * creal(F[b]) - sn * cimag(F[b]));
        tdpo_step(op, u, um, f, up);
        double *t = um; um = u; u = up; up = t;     /* now u = u_{j+1} */
        if (j + 1 == jsnap) memcpy(snap, u, sizeof(double) * N);
    }
    if (nP % 4 == 0) {
        for (long b = 0; b < N; ++b) U[b] = u[b] + I * snap[b];
    } else {
        double phi = 2.0 * M_PI * q / nP, c = cos(phi), s = sin(phi);
        for (long b = 0; b < N; ++b) U[b] = u[b] + I * ((snap[b] - c * u[b]) / s);
    }
    free(um); free(u); free(up); free(f); free(snap);
    return TDPO_OK;
}

/* Definition 4 as stated (complex-linear S_T): the integrator driven by the
 * complex forcing f_n = chi(1 - n dt/T~) e^{i omega n dt} F, T~ = 2 pi T/omega,
 * from zero fields; S_T F = e^{-i 2 pi T} u_{N_s} = u_{N_s} for integer T.
 * The recurrence is real, so the real and imaginary parts of u are two real
 * recurrences driven by the real and imaginary parts of f_n.  With the cell
 * damping the integrator is I_abd and this is S_T^abd of Def. 7. */
int tdpo_precond_apply_complex(const tdpo_op *op, int T, double rho, const double complex *F,
                               double complex *U)
{
    if (T < 1) return TDPO_EINVAL;
    if (rho <= 0.0) rho = 1.0 / T;
    if (rho > 1.0) return TDPO_EINVAL;
    long N = op->N;
    int nP = op->nP;
    long Ns = (long)T * nP;
    double *buf = calloc(8 * (size_t)N, sizeof(double));
    if (!buf) return TDPO_ENOMEM;
    double *ur = buf, *urm = buf + N, *urp = buf + 2 * N, *fr = buf + 3 * N;
    double *ui = buf + 4 * N, *uim = buf + 5 * N, *uip = buf + 6 * N, *fi = buf + 7 * N;
    for (long j = 0; j < Ns; ++j) {
        double chi = tdpo_window(1.0 - (double)j / (double)Ns, rho);
        double complex ph = cexp(I * 2.0 * M_PI * j / nP);
        for (long b = 0; b < N; ++b) {
            double complex fv = chi * ph * F[b];
            fr[b] = creal(fv);
            fi[b] = cimag(fv);
        }
        tdpo_step(op, ur, urm, fr, urp);
        tdpo_step(op, ui, uim, fi, uip);
        double *t = urm; urm = ur; ur = urp; urp = t;
        t = uim; uim = ui; ui = uip; uip = t;
    }
    for (long b = 0; b < N; ++b) U[b] = ur[b] + I * ui[b];
    free(buf);
    return TDPO_OK;
}

/* with the cell damping (dform 1) S_T is S_T^abd (Def. 7), complex-linear */
static int precond_variant(const tdpo_op *op, int variant, int T, double rho,
                           const double complex *F, double complex *U)
{
    return (variant || op->dform == 1) ? tdpo_precond_apply_complex(op, T, rho, F, U)
                   : tdpo_precond_apply(op, T, rho, F, U);
}

/* ------------------------------------------------------------------ */
/* GMRES (Sec. 2.4: left preconditioning, P H U = P F)                 */

static double complex zdot(long N, const double complex *a, const double complex *b)
{
    double complex s = 0.0;
    for (long i = 0; i < N; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double znrm(long N, const double complex *a)
{
    return sqrt(creal(zdot(N, a, a)));
}

/* Restarted GMRES on P H U = P F (modified Gram-Schmidt, complex Givens).
 * fixed_iters > 0: exactly that many iterations, restarts every `restart`.
 * Otherwise (tolerance mode) the true residual ||F - H x||/||F|| of the
 * current iterate x = x0 + V y is evaluated after every iteration; the solve
 * stops as soon as it is <= tol, and the cycle restarts early when the true
 * residual stalls while the Givens estimate still falls (the Table 1
 * preconditioner is only real-linear, so the Arnoldi relation holds only
 * approximately): relt > 2 * rel_start * est_cycle and relt > 0.7 * rel_prev. */
int tdpo_gmres_solve(const tdpo_op *op, int restart, int max_iters, int T, double rho,
                     double tol, int fixed_iters, int x0_given, int variant,
                     const double complex *F, double complex *U, double *info,
                     double *history, int history_cap)
{
    long N = op->N;
    int m = restart;
    if (m < 1 || T < 1 || max_iters < 1 || !(tol > 0.0)) return TDPO_EINVAL;
    int tolmode = fixed_iters <= 0;
    int limit = tolmode ? max_iters : fixed_iters;
    if (op->dform == 1) variant = 1;   /* S_T^abd is complex-linear (Def. 7) */
    double complex *V = malloc(sizeof(double complex) * N * (m + 1));
    double complex *w = malloc(sizeof(double complex) * N);
    double complex *r = malloc(sizeof(double complex) * N);
    double complex *xt = malloc(sizeof(double complex) * N);
    double complex *xbest = malloc(sizeof(double complex) * N);
    double complex *Hm = calloc((size_t)(m + 1) * m, sizeof(double complex));
    double complex *gv = malloc(sizeof(double complex) * (m + 1));
    double complex *sn = malloc(sizeof(double complex) * m);
    double *cs = malloc(sizeof(double) * m);
    double complex *y = malloc(sizeof(double complex) * m);
    if (!V || !w || !r || !xt || !xbest || !Hm || !gv || !sn || !cs || !y) {
        free(V); free(w); free(r); free(xt); free(xbest); free(Hm); free(gv); free(sn); free(cs);
        free(y);
        return TDPO_ENOMEM;
    }
#define HM(i, j) Hm[(size_t)(j) * (m + 1) + (i)]
    if (!x0_given) memset(U, 0, sizeof(double complex) * N);
    double bnorm = znrm(N, F);
    int its = 0, restarts = 0, nhist = 0, status = TDPO_ENOTCONV, switched = 0;
    long napply = 0;
    double pnorm0 = -1.0, est = 1.0, rel = 1.0;
    if (bnorm == 0.0) {
        memset(U, 0, sizeof(double complex) * N);
        status = TDPO_OK;
        rel = 0.0;
        est = 0.0;
        goto done;
    }
    for (;;) {
        /* r = F - H x,  z = P r */
        tdpo_apply_H(op, U, r);
        for (long i = 0; i < N; ++i) r[i] = F[i] - r[i];
        rel = znrm(N, r) / bnorm;
        if (tolmode && rel <= tol) { status = TDPO_OK; break; }
        if (its >= limit) break;
        precond_variant(op, variant, T, rho, r, V);
        ++napply;
        double beta0 = znrm(N, V);
        if (pnorm0 < 0.0) pnorm0 = beta0;
        if (beta0 == 0.0) break;
        for (long i = 0; i < N; ++i) V[i] /= beta0;
        for (int k = 0; k <= m; ++k) gv[k] = 0.0;
        gv[0] = beta0;
        double rel_start = rel, rel_prev = rel, best_rel = rel, rel_last = rel;
        int k_used = 0, converged = 0, best_k = 0;
        for (int i = 0; i < m && its < limit; ++i) {
            double complex *vi = V + (size_t)i * N, *vn = V + (size_t)(i + 1) * N;
            tdpo_apply_H(op, vi, r);
            precond_variant(op, variant, T, rho, r, w);
            ++napply;
            ++its;
            for (int k = 0; k <= i; ++k) {                 /* modified Gram-Schmidt */
                double complex *vk = V + (size_t)k * N;
                double complex hk = zdot(N, vk, w);
                HM(k, i) = hk;
                for (long q = 0; q < N; ++q) w[q] -= hk * vk[q];
            }
            double hn = znrm(N, w);
            HM(i + 1, i) = hn;
            for (int k = 0; k < i; ++k) {                  /* previous rotations */
                double complex a = HM(k, i), b = HM(k + 1, i);
                HM(k, i) = cs[k] * a + sn[k] * b;
                HM(k + 1, i) = -conj(sn[k]) * a + cs[k] * b;
            }
            double complex a = HM(i, i);
            double b = hn, rr = hypot(cabs(a), b);
            if (cabs(a) == 0.0) {
                cs[i] = 0.0;
                sn[i] = 1.0;
                HM(i, i) = b;
            } else {
                double complex ph = a / cabs(a);
                cs[i] = cabs(a) / rr;
                sn[i] = ph * b / rr;
                HM(i, i) = ph * rr;
            }
            HM(i + 1, i) = 0.0;
            gv[i + 1] = -conj(sn[i]) * gv[i];
            gv[i] = cs[i] * gv[i];
            est = cabs(gv[i + 1]) / pnorm0;
            double est_cycle = cabs(gv[i + 1]) / beta0;
            if (history && nhist < history_cap) history[nhist++] = est;
            k_used = i + 1;
            if (tolmode) {
                /* current iterate and its true residual */
                for (int k = k_used - 1; k >= 0; --k) {
                    double complex s = gv[k];
                    for (int j = k + 1; j < k_used; ++j) s -= HM(k, j) * y[j];
                    y[k] = s / HM(k, k);
                }
                memcpy(xt, U, sizeof(double complex) * N);
                for (int k = 0; k < k_used; ++k) {
                    double complex *vk = V + (size_t)k * N;
                    for (long q = 0; q < N; ++q) xt[q] += y[k] * vk[q];
                }
                tdpo_apply_H(op, xt, r);
                for (long q = 0; q < N; ++q) r[q] = F[q] - r[q];
                double relt = znrm(N, r) / bnorm;
                rel_last = relt;
                if (relt < best_rel) {                     /* best iterate of the cycle */
                    best_rel = relt;
                    best_k = k_used;
                    memcpy(xbest, xt, sizeof(double complex) * N);
                }
                if (relt <= tol) { converged = 1; break; }
                if (hn == 0.0) break;
                if (!(relt <= 1e6 * rel_start)) break;     /* runaway or not finite */
                if (relt > 2.0 * rel_start * est_cycle && relt > 0.7 * rel_prev) break;
                rel_prev = relt;
            } else if (hn == 0.0) {
                break;                                     /* happy breakdown */
            }
            for (long q = 0; q < N; ++q) vn[q] = w[q] / hn;
        }
        ++restarts;
        if (tolmode) {
            /* keep the cycle's iterate of least true residual; a Table 1 cycle
               that did not lower it is rejected and Definition 4 takes over */
            if (best_k == 0 && k_used > 0 && variant != 0) {
                /* Definition 4 is complex-linear: GMRES's own last iterate stands */
                best_k = k_used;
                best_rel = rel_last;
                memcpy(xbest, xt, sizeof(double complex) * N);
            }
            if (best_k > 0) memcpy(U, xbest, sizeof(double complex) * N);
            rel = best_rel;
            if (best_k == 0 && k_used > 0) {
                variant = 1;
                switched = 1;
            }
        } else {
            for (int k = k_used - 1; k >= 0; --k) {        /* back substitution R y = g */
                double complex s = gv[k];
                for (int j = k + 1; j < k_used; ++j) s -= HM(k, j) * y[j];
                y[k] = s / HM(k, k);
            }
            for (int k = 0; k < k_used; ++k) {
                double complex *vk = V + (size_t)k * N;
                for (long q = 0; q < N; ++q) U[q] += y[k] * vk[q];
            }
        }
        if (converged) { status = TDPO_OK; break; }
        if (!tolmode && its >= limit) {
            tdpo_apply_H(op, U, r);
            for (long i = 0; i < N; ++i) r[i] = F[i] - r[i];
            rel = znrm(N, r) / bnorm;
            status = TDPO_OK;
            break;
        }
        if (its >= limit) break;
    }
done:
    if (info) {
        info[0] = its;
        info[1] = restarts;
        info[2] = rel;
        info[3] = est;
        info[4] = nhist;
        info[5] = (double)napply;
        info[6] = switched;
    }
#undef HM
    free(V); free(w); free(r); free(xt); free(xbest); free(Hm); free(gv); free(sn); free(cs);
    free(y);
    return status;
}

/* ------------------------------------------------------------------ */
/* gradient: dL/dm_cell = omega^2 Re sum_{b,g in C(a)} M_{Delta(b,g)} conj(lam_b) U_g,
 * then the adjoint of m_cell = 2^-d sum over (clamped) corners of m_node.   */

void tdpo_grad_m(const tdpo_op *op, const double complex *lam, const double complex *U,
                 double *grad_nodes)
{
    int d = op->d, nk = 1 << d;
    double w2 = op->omega * op->omega;
    memset(grad_nodes, 0, sizeof(double) * op->N);
    for (long q = 0; q < op->Nc; ++q) {
        long alpha[3], e[3], b[3], g[3];
        cell_coords(op, q, alpha);
        double complex s = 0.0;
        for (int kb = 0; kb < nk; ++kb) {
            corner_offset(d, kb, e);
            for (int a = 0; a < d; ++a) b[a] = alpha[a] + e[a];
            long bi = node_index(op, b);
            if (bi < 0) continue;
            for (int kg = 0; kg < nk; ++kg) {
                corner_offset(d, kg, e);
                for (int a = 0; a < d; ++a) g[a] = alpha[a] + e[a];
                long gi = node_index(op, g);
                if (gi < 0) continue;
                s += op->M[delta_class(d, kb, kg)] * conj(lam[bi]) * U[gi];
            }
        }
        double gc = w2 * creal(s);
        for (int k = 0; k < nk; ++k) {
            corner_offset(d, k, e);
            for (int a = 0; a < d; ++a) b[a] = alpha[a] + e[a];
            grad_nodes[clamp_node(op, b)] += gc / nk;
        }
    }
}
