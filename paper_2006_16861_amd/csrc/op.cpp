// Host side of libtdp: operator setup (Sec. 2.2, Prop. 1, App. A), the
// preconditioner driver (Table 1), left-preconditioned restarted GMRES
// (Sec. 2.4) and the m-gradient, behind the C ABI of include/tdp.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tdp_internal.h"

namespace tdp {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

#define TDP_FAIL(code, ...)        \
    do {                           \
        ::tdp::set_error(__VA_ARGS__); \
        return (code);             \
    } while (0)

// Captured step loops kept per op (keyed by T, rho, variant and tuning); the
// cache is emptied when it would grow beyond this.
static const size_t kMaxGraphs = 16;

// Classical fourth-order compact scheme in the cell form (entries by the
// number of axes on which two corners of a cell differ).
static const double kStiff2[3] = {5.0 / 6.0, -1.0 / 3.0, -1.0 / 6.0};
static const double kMass2[3] = {1.0 / 6.0, 1.0 / 24.0, 0.0};
static const double kStiff3[4] = {0.5, -1.0 / 12.0, -1.0 / 12.0, 0.0};
static const double kMass3[4] = {1.0 / 16.0, 1.0 / 48.0, 0.0, 0.0};

// Elementary symmetric polynomial e_k of the d values s (each +-1).
static double esym(int d, const int *s, int k)
{
    double tot = 0.0;
    for (int mask = 0; mask < (1 << d); ++mask) {
        if (__builtin_popcount(mask) != k) continue;
        double p = 1.0;
        for (int a = 0; a < d; ++a)
            if (mask >> a & 1) p *= s[a];
        tot += p;
    }
    return tot;
}

// For a cell table T (entries by class k) the element matrix over the 2^d
// corners is diagonalised by the Walsh vectors prod_a s_a^{corner_a},
// s in {-1,1}^d, with eigenvalue sum_k T_k e_k(s).  The same sum times 2^d is
// the symbol of the assembled stencil at theta in {0, pi}^d (cos theta = s);
// the symbol is multi-affine in the cos theta_a, so its maximum over all
// theta is attained at one of these vertices.
static void table_spectrum(int d, const double *T, double *lo, double *hi)
{
    *lo = INFINITY;
    *hi = -INFINITY;
    for (int v = 0; v < (1 << d); ++v) {
        int s[3];
        for (int a = 0; a < d; ++a) s[a] = (v >> a & 1) ? -1 : 1;
        double e = 0.0;
        for (int k = 0; k <= d; ++k) e += T[k] * esym(d, s, k);
        *lo = std::fmin(*lo, e);
        *hi = std::fmax(*hi, e);
    }
}

// Sec. 6.1: stability of I_abd at theta = omega dt with the bounds lam_s >=
// lambda_max of the stiffness part of Re H and lam_im >= lambda_max(Im H):
// omega^2 = kmax2 + (beta/theta)(1 - cos theta) lam_im makes K >= 0, and
// 4I - K - 2L > 0 holds when
//   (theta^2/alpha)(lam_s/omega^2 + 1) + (theta beta/alpha)(1 + cos theta) lam_im/omega^2 < 4
// (the factor theta of the second term follows from K and L of Def. 6).
static bool abd_stable(double theta, double kmax2, double lam_s, double lam_im, double *w2out)
{
    const double sh = std::sin(0.5 * theta);
    const double alpha = theta * theta / (4.0 * sh * sh), beta = theta / std::sin(theta);
    const double w2 = kmax2 + beta / theta * (1.0 - std::cos(theta)) * lam_im;
    const double lhs = theta * theta / alpha * (lam_s / w2 + 1.0) +
                       theta * beta / alpha * (1.0 + std::cos(theta)) * lam_im / w2;
    if (w2out) *w2out = w2;
    return lhs < 4.0;
}

}  // namespace tdp

using namespace tdp;

extern "C" const char *tdp_last_error(void) { return g_last_error.c_str(); }

static int free_op(tdp_op *op)
{
    if (!op) return TDP_OK;
    if (op->ev) (void)hipEventDestroy(op->ev);
    for (hipEvent_t e : op->tev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(op->Fstage);
    (void)hipFree(op->Ustage);
    (void)hipFree(op->gcell);
    for (auto &kv : op->graphs) (void)hipGraphExecDestroy(kv.second);
    void *bufs[] = {op->m, op->rw, op->dn, op->m32, op->dn32, op->rc32, op->u0, op->u1, op->u2, op->v0, op->v1,
                    op->u3, op->u4, op->u5, op->rc, op->Fst, op->scratch, op->V, op->wv, op->tv, op->rv,
                    op->xv, op->red, op->dcoef};
    for (void *b : bufs) (void)hipFree(b);
    (void)hipFree(op->res_shadow);
    (void)hipFree(op->res_flags);
    for (auto &kv : op->dtables) (void)hipFree(kv.second);
    if (op->res_host) (void)hipHostFree(op->res_host);
    if (op->hres) (void)hipHostFree(op->hres);
    if (op->own_stream && op->stream) (void)hipStreamDestroy(op->stream);
    delete op;
    return TDP_OK;
}

extern "C" int tdp_op_destroy(tdp_op *op)
{
    clear_error();
    if (op) (void)hipStreamSynchronize(op->stream);
    return free_op(op);
}

static int create_impl(const tdp_op_desc *d, tdp_op *op)
{
    if (d->ndim != 2 && d->ndim != 3) TDP_FAIL(TDP_EINVAL, "ndim must be 2 or 3 (got %d)", d->ndim);
    if (!(d->h > 0.0)) TDP_FAIL(TDP_EINVAL, "h must be > 0");
    if (!(d->omega > 0.0)) TDP_FAIL(TDP_EINVAL, "omega must be > 0");
    if (!d->c) TDP_FAIL(TDP_EINVAL, "c must not be NULL");
    if (d->prec != TDP_F64 && d->prec != TDP_F32) TDP_FAIL(TDP_EINVAL, "prec must be TDP_F64 or TDP_F32");
    if (d->damping != TDP_DAMP_NODE && d->damping != TDP_DAMP_CELL)
        TDP_FAIL(TDP_EINVAL, "damping must be TDP_DAMP_NODE or TDP_DAMP_CELL");
    op->dform = d->damping;
    op->ndim = d->ndim;
    op->N = 1;
    op->Nc = 1;
    for (int a = 0; a < d->ndim; ++a) {
        if (d->n[a] < 1 || d->n[a] > (1 << 20))
            TDP_FAIL(TDP_EINVAL, "n[%d] = %lld out of range [1, 2^20]", a, (long long)d->n[a]);
        op->n[a] = (int)d->n[a];
        op->N *= d->n[a];
        op->Nc *= d->n[a] + 1;
    }
    if (op->N > (int64_t)1 << 36) TDP_FAIL(TDP_EINVAL, "grid too large");
    // launch grids of the node (and cell) per thread kernels: blocks of 4 rows
    // along axis ndim-2 and one (cell) plane of axis 0 in 3-D per grid row,
    // at most 65535 blocks along grid y and z
    {
        const int64_t ylen = d->n[d->ndim - 2] + 1;
        if ((ylen + 3) / 4 > 65535)
            TDP_FAIL(TDP_EINVAL, "n[%d] = %lld exceeds 262139", d->ndim - 2,
                     (long long)d->n[d->ndim - 2]);
        if (d->ndim == 3 && d->n[0] + 1 > 65535)
            TDP_FAIL(TDP_EINVAL, "n[0] = %lld exceeds 65534 in 3-D", (long long)d->n[0]);
    }
    op->h = d->h;
    op->omega = d->omega;
    op->prec = d->prec;
    const int D = d->ndim;
    const double *S = d->stiff ? d->stiff : (D == 2 ? kStiff2 : kStiff3);
    const double *M = d->mass ? d->mass : (D == 2 ? kMass2 : kMass3);
    for (int k = 0; k <= D; ++k) {
        op->S[k] = S[k];
        op->M[k] = M[k];
        if (!std::isfinite(S[k]) || !std::isfinite(M[k])) TDP_FAIL(TDP_EINVAL, "non-finite cell table");
    }
    // App. A conditions: element stiffness PSD, element mass PSD with
    // largest eigenvalue <= 2^-d (so Re H >= -k_max^2).
    double slo, shi, mlo, mhi;
    table_spectrum(D, op->S, &slo, &shi);
    table_spectrum(D, op->M, &mlo, &mhi);
    const double tol = 1e-12;
    if (slo < -tol * std::fmax(1.0, shi)) TDP_FAIL(TDP_EINVAL, "stiffness cell table is not PSD");
    if (mlo < -tol || mhi > std::ldexp(1.0, -D) * (1 + tol))
        TDP_FAIL(TDP_EINVAL, "mass cell table must be PSD with eigenvalues <= 2^-d");
    if (!(shi > 0.0)) TDP_FAIL(TDP_EINVAL, "stiffness cell table is zero");
    op->sc = 1;
    op->mc = 0;
    for (int k = 1; k <= D; ++k)
        if (op->S[k] != 0.0) op->sc = k + 1;
    for (int k = 0; k <= D; ++k)
        if (op->M[k] != 0.0) op->mc = k + 1;

    TDP_CHECK_HIP(hipGetDevice(&op->device));
    TDP_CHECK(noalloc_setup_device(op->device));
    TDP_CHECK_HIP(hipDeviceGetAttribute(&op->ncu, hipDeviceAttributeMultiprocessorCount, op->device));
    op->user_stream = (hipStream_t)d->stream;
    if (op->user_stream) {
        op->stream = op->user_stream;
    } else {
        TDP_CHECK_HIP(hipStreamCreateWithFlags(&op->stream, hipStreamNonBlocking));
        op->own_stream = true;
        TDP_CHECK_HIP(hipEventCreateWithFlags(&op->ev, hipEventDisableTiming));
    }
    StreamJoin join(op->user_stream, op->stream, op->ev);
    hipStream_t s = op->stream;

    const size_t nb = sizeof(double) * op->N;
    if (hipMalloc(&op->m, sizeof(double) * op->Nc) != hipSuccess ||
        hipMalloc(&op->rw, nb) != hipSuccess || hipMalloc(&op->dn, nb) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "device allocation of operator arrays failed");
    op->scratch_bytes = sizeof(double) * 2048;
    if (hipMalloc(&op->scratch, op->scratch_bytes) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "device allocation failed");

    // validate c > 0 and R >= 0 on the host (one pass, setup only)
    {
        std::vector<double> hc(op->N);
        TDP_CHECK_HIP(hipMemcpyAsync(hc.data(), d->c, nb, hipMemcpyDeviceToHost, s));
        std::vector<double> hr;
        if (d->R) {
            hr.resize(op->N);
            TDP_CHECK_HIP(hipMemcpyAsync(hr.data(), d->R, nb, hipMemcpyDeviceToHost, s));
        }
        TDP_CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < op->N; ++i) {
            if (!(hc[i] > 0.0) || !std::isfinite(hc[i]))
                TDP_FAIL(TDP_EINVAL, "c must be finite and > 0 (node %lld)", (long long)i);
            if (d->R && (!(hr[i] >= 0.0) || !std::isfinite(hr[i])))
                TDP_FAIL(TDP_EINVAL, "R must be finite and >= 0 (node %lld)", (long long)i);
        }
    }

    // cell slowness and its maximum (App. A: k constant per cell)
    TDP_CHECK_HIP(launch_cell_slowness(D, op->n, d->c, op->m, s));
    const int nblk = 256;
    TDP_CHECK_HIP(launch_max_reduce(op->m, op->Nc, op->scratch, nblk, op->scratch + nblk, s));
    double mmax = 0.0;
    TDP_CHECK_HIP(hipMemcpyAsync(&mmax, op->scratch + nblk, sizeof(double), hipMemcpyDeviceToHost, s));
    TDP_CHECK_HIP(hipStreamSynchronize(s));

    // Sec. 2.2: omega_c bounds sqrt(-lambda_min(Re H)); the CFL bound uses
    // lambda_max(A) <= h^-2 max S(theta) + omega_c^2.
    op->omega_c = op->omega * std::sqrt(mmax);
    const double lam_s = std::ldexp(shi, D) / (op->h * op->h);
    int nP = d->steps_per_period;
    if (op->dform == TDP_DAMP_CELL) {
        // cell damping r_cell (corner mean of R); lambda_max(Im H) <= omega max r_cell
        if (hipMalloc(&op->rc, sizeof(double) * op->Nc) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "device allocation of the cell damping failed");
        if (d->R) {
            TDP_CHECK_HIP(launch_cell_mean(D, op->n, d->R, op->rc, s));
        } else {
            TDP_CHECK_HIP(launch_fill_zero(op->rc, sizeof(double) * op->Nc, s));
        }
        TDP_CHECK_HIP(launch_max_reduce(op->rc, op->Nc, op->scratch, nblk, op->scratch + nblk, s));
        double rmax = 0.0;
        TDP_CHECK_HIP(hipMemcpyAsync(&rmax, op->scratch + nblk, sizeof(double), hipMemcpyDeviceToHost, s));
        TDP_CHECK_HIP(hipStreamSynchronize(s));
        op->lam_im = op->omega * rmax;
        // Sec. 6.1: theta = omega dt = 2 pi / n_P with n_P the smallest multiple of 4
        // (steps_per_period = -1: the smallest integer >= 3) satisfying the
        // stability condition; omega from the K >= 0 condition
        const double kmax2 = op->omega_c * op->omega_c;
        if (nP == 0 || nP == -1) {
            const int step = nP == 0 ? 4 : 1;
            for (nP = nP == 0 ? 4 : 3; nP <= (1 << 22); nP += step)
                if (abd_stable(2.0 * M_PI / nP, kmax2, lam_s, op->lam_im, nullptr)) break;
            if (nP > (1 << 22)) TDP_FAIL(TDP_ECFL, "no stable step for the cell damping");
        } else if (nP < 3 || !abd_stable(2.0 * M_PI / nP, kmax2, lam_s, op->lam_im, nullptr)) {
            TDP_FAIL(TDP_ECFL, "steps_per_period %d violates the I_abd stability condition", nP);
        }
        double w2 = 0.0;
        abd_stable(2.0 * M_PI / nP, kmax2, lam_s, op->lam_im, &w2);
        op->omega_c = std::sqrt(w2);
    } else {
        const double lb = lam_s + op->omega_c * op->omega_c;
        const double nmin = M_PI / std::asin(op->omega_c / std::sqrt(lb));
        if (nP == 0) {
            nP = 4 * ((int)std::floor(nmin / 4.0) + 1);
        } else if (nP == -1) {
            nP = std::max(3, (int)std::floor(nmin) + 1);
        } else if (nP < 3 || !((double)nP > nmin)) {
            TDP_FAIL(TDP_ECFL, "steps_per_period %d must be at least 3 and above the CFL bound %.6f",
                     nP, nmin);
        }
    }
    op->lam_bar = lam_s + op->omega_c * op->omega_c;
    op->nP = nP;
    op->dt = 2.0 * M_PI / (op->omega_c * nP);
    const double th = 2.0 * M_PI / nP;   // omega_c * dt
    const double sh = std::sin(0.5 * th);
    op->alpha = th * th / (4.0 * sh * sh);   // Prop. 1
    op->beta = th / std::sin(th);
    op->g = op->dt * op->dt / op->alpha;
    op->cS = op->g / (op->h * op->h);
    op->cM = op->g * op->omega * op->omega;
    op->cw = op->g * op->omega_c * op->omega_c;
    const double lscale = op->beta * op->dt / op->alpha * op->omega / op->omega_c;

    // stencil constants: (2 - K) u for the step, Re H x for the H-apply
    op->st_step.c0 = 2.0 - op->cw - op->cS * std::ldexp(op->S[0], D);
    op->st_H.c0 = std::ldexp(op->S[0], D) / (op->h * op->h);
    op->st_step.s[0] = op->st_H.s[0] = 0.0;
    for (int k = 1; k < 4; ++k) {
        const double sk = k <= D ? std::ldexp(op->S[k], D - k) : 0.0;
        op->st_step.s[k] = -op->cS * sk;
        op->st_H.s[k] = sk / (op->h * op->h);
    }
    for (int k = 0; k < 4; ++k) {
        const double mk = k <= D ? op->M[k] : 0.0;
        op->st_step.m[k] = op->cM * mk;
        op->st_H.m[k] = -op->omega * op->omega * mk;
    }
    // Im H (cell damping) and (beta dt / (alpha omega_c)) Im H as mass-class
    // stencils over r_cell (Sec. 6: L = (beta dt/alpha) B, B = Im H / omega_c)
    op->cos_th = std::cos(th);
    const double lb = op->beta * op->dt / op->alpha / op->omega_c;
    for (int k = 0; k < 4; ++k) {
        const double mk = k <= D ? op->M[k] : 0.0;
        op->st_I.m[k] = op->omega * mk;
        op->st_B.m[k] = lb * op->omega * mk;
    }
    op->st_step32.c0 = (float)op->st_step.c0;
    op->st_B32.c0 = (float)op->st_B.c0;
    for (int k = 0; k < 4; ++k) {
        op->st_step32.s[k] = (float)op->st_step.s[k];
        op->st_step32.m[k] = (float)op->st_step.m[k];
        op->st_B32.s[k] = (float)op->st_B.s[k];
        op->st_B32.m[k] = (float)op->st_B.m[k];
    }

    TDP_CHECK_HIP(launch_node_factors(d->R, op->N, op->omega, lscale, op->rw, op->dn, s));

    const size_t fb = (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    if (hipMalloc(&op->u0, fb) != hipSuccess || hipMalloc(&op->u1, fb) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "device allocation of recurrence fields failed");
    if (op->prec == TDP_F32) {
        if (hipMalloc(&op->m32, sizeof(float) * op->Nc) != hipSuccess ||
            hipMalloc(&op->dn32, sizeof(float) * op->N) != hipSuccess ||
            hipMalloc(&op->Fst, sizeof(float) * 2 * op->N) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "device allocation of FP32 arrays failed");
        TDP_CHECK_HIP(launch_cvt_f64_to_f32(op->m, op->m32, op->Nc, s));
        TDP_CHECK_HIP(launch_cvt_f64_to_f32(op->dn, op->dn32, op->N, s));
        if (op->dform == TDP_DAMP_CELL) {
            if (hipMalloc(&op->rc32, sizeof(float) * op->Nc) != hipSuccess)
                TDP_FAIL(TDP_ENOMEM, "device allocation of FP32 arrays failed");
            TDP_CHECK_HIP(launch_cvt_f64_to_f32(op->rc, op->rc32, op->Nc, s));
        }
    }
    if (hipMalloc(&op->Fstage, 16 * op->N) != hipSuccess || hipMalloc(&op->Ustage, 16 * op->N) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "device allocation of staging buffers failed");
    TDP_CHECK_HIP(hipStreamSynchronize(s));
    return TDP_OK;
}

extern "C" int tdp_op_create(const tdp_op_desc *d, tdp_op **out)
{
    clear_error();
    if (!d || !out) TDP_FAIL(TDP_EINVAL, "NULL argument");
    *out = nullptr;
    tdp_op *op = new tdp_op();
    int rc = create_impl(d, op);
    if (rc != TDP_OK) {
        std::string msg = g_last_error;
        if (op->stream) (void)hipStreamSynchronize(op->stream);
        free_op(op);
        g_last_error = msg;
        return rc;
    }
    *out = op;
    return TDP_OK;
}

extern "C" int tdp_op_query(const tdp_op *op, tdp_op_info *o)
{
    clear_error();
    if (!op || !o) TDP_FAIL(TDP_EINVAL, "NULL argument");
    o->omega_c = op->omega_c;
    o->dt = op->dt;
    o->alpha = op->alpha;
    o->beta = op->beta;
    o->lam_bar = op->lam_bar;
    o->n_P = op->nP;
    o->ndim = op->ndim;
    o->N = op->N;
    o->lam_im = op->lam_im;
    o->res_aborts = op->res_aborts;
    return TDP_OK;
}

extern "C" int tdp_op_set_tuning(tdp_op *op, const tdp_tuning *t)
{
    clear_error();
    if (!op || !t) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (t->kernel < 0 || t->kernel > 5) TDP_FAIL(TDP_EINVAL, "kernel must be in [0, 5]");
    if (t->kernel == 3 || t->kernel == 4) {
        if (t->tb_depth < 0 || t->tb_depth > (1 << 20)) TDP_FAIL(TDP_EINVAL, "bad chunk length");
        if (t->tile < 0 || t->tile > 2) TDP_FAIL(TDP_EINVAL, "tile must be 0, 1 or 2 for kernels 3 and 4");
    } else {
        if (t->tb_depth < 0 || t->tb_depth > TDP_TB_KMAX) TDP_FAIL(TDP_EINVAL, "tb_depth must be in [0, 16]");
        if (t->tile < 0 || t->tile > 15) TDP_FAIL(TDP_EINVAL, "tile must be in [0, 15]");
        if ((t->kernel == 0 || t->kernel == 2) && tb2d_f32_only(t->tile) && op->prec == TDP_F64)
            TDP_FAIL(TDP_EINVAL, "tiles 2, 8, 12 and 13 are FP32 only");
    }
    op->tune = *t;
    return TDP_OK;
}

extern "C" int tdp_op_force_resident_abort(tdp_op *op, int on)
{
    clear_error();
    if (!op) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (on != 0 && on != 1) TDP_FAIL(TDP_EINVAL, "on must be 0 or 1");
    op->res_force_abort = on != 0;
    for (auto &kv : op->graphs) (void)hipGraphExecDestroy(kv.second);   // graphs hold the old waits
    op->graphs.clear();
    return TDP_OK;
}

extern "C" int tdp_op_get_tuning(const tdp_op *op, tdp_tuning *t)
{
    clear_error();
    if (!op || !t) TDP_FAIL(TDP_EINVAL, "NULL argument");
    *t = op->tune;
    return TDP_OK;
}

// ---------------------------------------------------------------------------
int apply_H_impl(const tdp_op *op, const void *x, const void *F, void *y)
{
    TDP_CHECK_HIP(launch_apply_H(op->ndim, op->n, op->sc, op->mc, op->m, op->rw,
                                 op->dform == TDP_DAMP_CELL ? op->rc : nullptr, op->st_H, op->st_I,
                                 x, F, y, op->stream));
    return TDP_OK;
}

extern "C" int tdp_apply_H(const tdp_op *op, const void *x, void *y)
{
    clear_error();
    if (!op || !x || !y) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (x == y) TDP_FAIL(TDP_EINVAL, "x and y must not alias");
    if (misaligned16(x) || misaligned16(y)) TDP_FAIL(TDP_EINVAL, "complex arrays must be 16-byte aligned");
    StreamJoin join(op->user_stream, op->stream, op->ev);
    return apply_H_impl(op, x, nullptr, y);
}

// Sec. 2.3 window: 1 on |s| <= 1-rho, sin^2(pi (1-|s|) / (2 rho)) on the taper.
static double window(double s, double rho)
{
    const double a = std::fabs(s);
    if (a >= 1.0) return 0.0;
    if (a <= 1.0 - rho) return 1.0;
    const double v = std::sin(M_PI * (1.0 - a) / (2.0 * rho));
    return v * v;
}

// Forcing scalars for steps j = 0..N_s-1, already scaled by g = dt^2/alpha
// (Def. 2), chi_j = chi(1 - j/N_s), phi_j = 2 pi j/n_P:
//   Table 1 (real field):   fa_j = g chi_j cos phi_j,  fb_j = -g chi_j sin phi_j,
//                           forcing fa Re F + fb Im F = g Re(chi_j e^{i phi_j} F);
//   Definition 4 (complex): fa_j = g chi_j cos phi_j,  fb_j = g chi_j sin phi_j,
//                           forcing (fa + i fb) F = g chi_j e^{i phi_j} F.
void forcing_pair(const tdp_op *op, int64_t Ns, double rho, int variant, int64_t j, double *fa,
                  double *fb)
{
    const double chi = window(1.0 - (double)j / (double)Ns, rho);
    const double ph = 2.0 * M_PI * (double)j / op->nP;
    if (variant == 2) {          // imaginary part of Definition 4's forcing
        *fa = op->g * chi * std::sin(ph);
        *fb = op->g * chi * std::cos(ph);
    } else {
        *fa = op->g * chi * std::cos(ph);
        *fb = (variant ? 1.0 : -1.0) * op->g * chi * std::sin(ph);
    }
}

const std::vector<double> &forcing_table(tdp_op *op, int T, double rho, int variant)
{
    auto key = std::make_tuple(T, rho, variant);
    auto it = op->tables.find(key);
    if (it != op->tables.end()) return it->second;
    const int64_t Ns = (int64_t)T * op->nP;
    std::vector<double> t(2 * Ns);
    for (int64_t j = 0; j < Ns; ++j) forcing_pair(op, Ns, rho, variant, j, &t[2 * j], &t[2 * j + 1]);
    return op->tables.emplace(key, std::move(t)).first->second;
}

// Forcing scalars of one loop: read from the cached table, or (for the
// allocation-free entry point) evaluated step by step with the same formula.
struct ForcingSrc {
    const double *tab = nullptr;
    const tdp_op *op = nullptr;
    int64_t Ns = 0;
    double rho = 0;
    int variant = 0;
    double a(int64_t j) const { return tab ? tab[2 * j] : pair(j).first; }
    double b(int64_t j) const { return tab ? tab[2 * j + 1] : pair(j).second; }
    std::pair<double, double> pair(int64_t j) const
    {
        double fa, fb;
        forcing_pair(op, Ns, rho, variant, j, &fa, &fb);
        return {fa, fb};
    }
};
static ForcingSrc forcing_src(tdp_op *op, int T, double rho, int variant, const LoopBufs &lb)
{
    ForcingSrc f;
    f.op = op;
    f.Ns = (int64_t)T * op->nP;
    f.rho = rho;
    f.variant = variant;
    if (!lb.table_free) f.tab = forcing_table(op, T, rho, variant).data();
    return f;
}

// Table 1's second sample: u_{N_s - q} with q = n_P/4 (a quarter period) when
// 4 divides n_P, else q = round(n_P/4), whose phase 2 pi q/n_P stays within
// 45 degrees of a quarter period, and Im U follows from a 2x2 solve (Sec. 2.3).
int64_t snap_lag(int nP)
{
    return nP % 4 == 0 ? nP / 4 : (nP + 2) / 4;
}

static int ensure_complex_fields(tdp_op *op)
{
    const size_t fb = 2 * (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    if (!op->u2 && (hipMalloc(&op->u2, fb) != hipSuccess || hipMalloc(&op->u3, fb) != hipSuccess))
        TDP_FAIL(TDP_ENOMEM, "device allocation of complex recurrence fields failed");
    if (op->dform == TDP_DAMP_CELL && !op->u4 &&
        (hipMalloc(&op->u4, fb) != hipSuccess || hipMalloc(&op->u5, fb) != hipSuccess))
        TDP_FAIL(TDP_ENOMEM, "device allocation of complex recurrence fields failed");
    return TDP_OK;
}

// Which sweep kernel, depth and tile the loop uses: 1 one step per launch, 2
// the blocked 2-D kernel (k steps per launch), 3 / 4 the streamed 3-D kernels
// (depth = planes per chunk).  kernel 0 chooses all three: the blocked 2-D
// sweep on the 32 x 64 tile (FP64) or the 128 x 64 tile (FP32) at depth 8,
// the streamed 3-D sweep on 8 x 64 columns, with the chunk below.
// Kernel 5, the resident-tile 2-D sweep (exchange depth = depth), applies to
// Table 1 fields with node damping and tables without corner mass terms, on grids whose tiles fit the compute units (one workgroup each);
// elsewhere, and for the allocation-free entry point (resident = false), the
// plan falls back to the blocked sweep.
static bool res_applies(const tdp_op *op, int k)
{
    const int nt = res_tiles(op->n[0], op->n[1], k, op->prec == TDP_F64, nullptr, nullptr);
    return op->ndim == 2 && op->dform == TDP_DAMP_NODE && op->mc <= 2 && nt > 0 && nt <= op->ncu;
}

static void sweep_plan(const tdp_op *op, int variant, int *kernel, int *depth, int *tile,
                       bool resident = true)
{
    int kern = op->tune.kernel, k = op->tune.tb_depth, t = op->tune.tile;
    (void)variant;    // Definition 4 runs the same kernels as two real passes
    const bool f64 = op->prec == TDP_F64;
    if (kern == 5) {
        if (k == 0) k = 4;
        if (resident && res_applies(op, k)) {
            *kernel = 5;
            *depth = k;
            *tile = 0;
            return;
        }
        kern = k = t = 0;
    }
    if (kern == 0) {
        if (op->ndim == 2) {
            kern = 2;
            k = 8;
            t = f64 ? 5 : 8;
        } else if (op->sc <= 3 && op->mc <= 2) {
            // 3-D compact tables: two steps per launch, FP64 on 66 x 15
            // blocks, FP32 on 66 x 31 blocks (66 x 15 below about 3 * 2^20
            // nodes).  Measured per step against the one-step sweep: FP64
            // 17.9 / 23.4 us at 128^3, 73 / 81 at 192^3, 132 / 146 at 256^3;
            // FP32 14.3 / 17.5 at 128^3, 41 / 49 at 192^3, 77 / 84 at 224^3,
            // but 82 / 79 at 256^3 (the autotuner decides there)
            kern = 4;
            k = 8;
            t = f64 || op->N < (3 << 20) ? 1 : 2;
        } else {
            kern = 3;
            k = t = 0;
        }
        if (op->dform == TDP_DAMP_CELL) t = f64 ? 7 : 4;
    }
    // I_abd: the blocked 2-D kernel on the tiles that hold its per-node state
    // (mass tables without corner entries), else one step per launch
    if (op->dform == TDP_DAMP_CELL &&
        !(kern == 2 && op->ndim == 2 && op->mc <= 2 && abd_tile_ok(t, f64)))
        kern = 1;
    if (kern == 2 && op->ndim != 2) kern = 1;
    // the weights-without-d tiles hold one corner weight: tables with corner
    // mass terms take the 32 x 64 tile instead
    if (kern == 2 && (t == 14 || t == 15) && op->mc > 2) t = 5;
    if ((kern == 3 || kern == 4) && op->ndim != 3) kern = 1;
    if (kern == 2) {
        if (k == 0) k = 4;
        const int rows = tb2d_tile_rows(t, op->prec == TDP_F64);
        if (4 * k > rows || 4 * k > tb2d_tile_cols(t)) k = rows / 8;   // keep at least half the tile exact
    } else if (kern == 3 || kern == 4) {
        if (t > 2) t = 1;
        if (k == 0 && kern == 4) {
            // fewest planes per workgroup run: the run count per column block
            // is chosen to fill whole rounds of the resident workgroups, so
            // this only bounds how finely a small grid is split
            k = 8;
        } else if (k == 0) {
            // default chunk length: halve from 32 (down to 8) until the launch
            // has about 8192 waves, so that small grids still fill the chip
            // (128^3: 8 planes, 2x faster than 32; 256^3: 16)
            const int rows = t == 0 ? 8 : 16;
            const int waves = t == 2 ? 8 : 4;
            const int64_t txy = (int64_t)((op->n[2] + 63) / 64) * ((op->n[1] + rows - 1) / rows);
            k = 32;
            while (k > 8 && txy * ((op->n[0] + k - 1) / k) * waves < 8192) k /= 2;
        }
    } else {
        k = 1;
    }
    *kernel = kern;
    *depth = k;
    *tile = t;
}

static int ensure_tb_fields(tdp_op *op)
{
    if (op->v0) return TDP_OK;
    const size_t fb = (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    if (hipMalloc(&op->v0, fb) != hipSuccess || hipMalloc(&op->v1, fb) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "device allocation of blocked-sweep fields failed");
    return TDP_OK;
}

// Blocked loop: launches of k steps, ping-ponging between the field pairs
// (u0, u1) and (v0, v1).
// Real-field loops (Table 1's recurrence with the forcing table `tabv`): the
// final field goes to out_final and, when out_snap is given, the sample
// u_{N_s - q} to out_snap (stride-2 doubles inside a complex128 array).
static int issue_steps_tb(tdp_op *op, const LoopBufs &lb, int T, double rho, int depth, int tile,
                          const void *Fin, int tabv, double *out_final, double *out_snap)
{
    hipStream_t s = op->stream;
    const ForcingSrc tab = forcing_src(op, T, rho, tabv, lb);
    const int64_t Ns = (int64_t)T * op->nP, jsnap = out_snap ? Ns - snap_lag(op->nP) : -1;
    const size_t fb = (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    void *cur = lb.u0, *prev = lb.u1, *ncur = lb.v0, *nprev = lb.v1;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    TBArgs a;
    a.ny = op->n[0];
    a.nx = op->n[1];
    a.sc = op->sc;
    a.mc = op->mc;
    a.shape = tile;
    a.m = op->prec == TDP_F64 ? (const void *)op->m : (const void *)op->m32;
    a.dn = op->prec == TDP_F64 ? (const void *)op->dn : (const void *)op->dn32;
    a.F = Fin;
    for (int64_t j0 = 0; j0 < Ns; j0 += depth) {
        const int k = (int)std::min<int64_t>(depth, Ns - j0);
        a.u_in = cur;
        a.up_in = prev;
        a.u_out = ncur;
        a.up_out = nprev;
        a.cf.k = k;
        for (int q = 0; q < k; ++q) {
            a.cf.fa[q] = tab.a(j0 + q);
            a.cf.fb[q] = tab.b(j0 + q);
        }
        // step q (1-based) of this launch produces u_{j0+q}
        a.cf.out_step[0] = (jsnap > j0 && jsnap <= j0 + k) ? (int)(jsnap - j0) : 0;
        a.cf.out[0] = out_snap;
        a.cf.out_step[1] = (Ns > j0 && Ns <= j0 + k) ? (int)(Ns - j0) : 0;
        a.cf.out[1] = out_final;
        if (op->prec == TDP_F64)
            TDP_CHECK_HIP(launch_sweep2d_tb_f64(a, op->st_step, s));
        else
            TDP_CHECK_HIP(launch_sweep2d_tb_f32(a, op->st_step32, s));
        std::swap(cur, ncur);
        std::swap(prev, nprev);
    }
    return TDP_OK;
}

// Blocked I_abd loop on the complex field of S_T^abd: both real parts per
// launch (the real part driven by the Table 1 form of the forcing table, the
// imaginary part by (-fb, fa)), ping-ponging between the complex field pairs
// (u2, u3) and (u4, u5); the final field goes to U (complex128).
static int issue_steps_abd2(tdp_op *op, const LoopBufs &lb, int T, double rho, int depth,
                            int tile, const void *Fin, double *U)
{
    hipStream_t s = op->stream;
    const ForcingSrc tab = forcing_src(op, T, rho, 0, lb);
    const int64_t Ns = (int64_t)T * op->nP;
    const bool f64 = op->prec == TDP_F64;
    const size_t fb = 2 * (f64 ? sizeof(double) : sizeof(float)) * op->N;
    void *cur = op->u2, *prev = op->u3, *ncur = op->u4, *nprev = op->u5;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    TBArgs a;
    a.ny = op->n[0];
    a.nx = op->n[1];
    a.sc = op->sc;
    a.mc = op->mc;
    a.shape = tile;
    a.m = f64 ? (const void *)op->m : (const void *)op->m32;
    a.rc = f64 ? (const void *)op->rc : (const void *)op->rc32;
    a.cth = op->cos_th;
    a.F = Fin;
    for (int64_t j0 = 0; j0 < Ns; j0 += depth) {
        const int k = (int)std::min<int64_t>(depth, Ns - j0);
        a.u_in = cur;
        a.up_in = prev;
        a.u_out = ncur;
        a.up_out = nprev;
        a.cf.k = k;
        for (int q = 0; q < k; ++q) {
            a.cf.fa[q] = tab.a(j0 + q);
            a.cf.fb[q] = tab.b(j0 + q);
        }
        a.cf.out_step[0] = 0;
        a.cf.out[0] = nullptr;
        a.cf.out_step[1] = (Ns > j0 && Ns <= j0 + k) ? (int)(Ns - j0) : 0;
        a.cf.out[1] = U;
        if (f64)
            TDP_CHECK_HIP(launch_sweep2d_abd2_tb_f64(a, op->st_step, op->st_B, s));
        else
            TDP_CHECK_HIP(launch_sweep2d_abd2_tb_f32(a, op->st_step32, op->st_B32, s));
        std::swap(cur, ncur);
        std::swap(prev, nprev);
    }
    return TDP_OK;
}

// Resident-tile loop (kernel 5): launches of up to TDP_RES_MAXSTEPS steps,
// each preceded by a fill of the tile flags and the abort word, ping-ponging
// between the field pairs (u0, u1) and (v0, v1).
static int issue_steps_res(tdp_op *op, const LoopBufs &lb, int T, double rho, int k,
                           const void *Fin, int tabv, double *out_final, double *out_snap)
{
    hipStream_t s = op->stream;
    const int64_t Ns = (int64_t)T * op->nP, jsnap = out_snap ? Ns - snap_lag(op->nP) : -1;
    auto it = op->dtables.find(std::make_tuple(T, rho, tabv));
    if (it == op->dtables.end()) TDP_FAIL(TDP_EINVAL, "resident sweep: forcing table not staged");
    ResArgs a;
    a.ny = op->n[0];
    a.nx = op->n[1];
    a.sc = op->sc;
    a.k = k;
    const bool f64 = op->prec == TDP_F64;
    const int nt = res_tiles(a.ny, a.nx, k, f64, &a.tiles_x, &a.tiles_y);
    if (nt <= 0 || nt > op->res_ntiles) TDP_FAIL(TDP_EINVAL, "resident sweep: tile grid not set up");
    a.m = f64 ? (const void *)op->m : (const void *)op->m32;
    a.dn = f64 ? (const void *)op->dn : (const void *)op->dn32;
    a.F = Fin;
    a.shadow = op->res_shadow;
    a.flags = op->res_flags;
    a.poll_limit = op->res_force_abort ? 16 : (1 << 20);
    a.wait_bias = op->res_force_abort ? (1 << 30) : 0;
    const size_t fb = (f64 ? sizeof(double) : sizeof(float)) * op->N;
    const size_t flag_bytes = sizeof(int) * ((size_t)nt * TDP_RES_FLAG_STRIDE + TDP_RES_FLAG_STRIDE);
    void *cur = lb.u0, *prev = lb.u1, *ncur = lb.v0, *nprev = lb.v1;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    for (int64_t j0 = 0; j0 < Ns; j0 += TDP_RES_MAXSTEPS) {
        const int n = (int)std::min<int64_t>(TDP_RES_MAXSTEPS, Ns - j0);
        a.nsteps = n;
        a.u_in = cur;
        a.up_in = prev;
        a.u_out = ncur;
        a.up_out = nprev;
        a.tab = it->second + 2 * j0;
        a.out_step[0] = (jsnap > j0 && jsnap <= j0 + n) ? (int)(jsnap - j0) : 0;
        a.out[0] = out_snap;
        a.out_step[1] = (Ns > j0 && Ns <= j0 + n) ? (int)(Ns - j0) : 0;
        a.out[1] = out_final;
        TDP_CHECK_HIP(launch_fill_zero(op->res_flags, flag_bytes, s));
        if (f64)
            TDP_CHECK_HIP(launch_sweep2d_res_f64(a, op->st_step, s));
        else
            TDP_CHECK_HIP(launch_sweep2d_res_f32(a, op->st_step32, s));
        std::swap(cur, ncur);
        std::swap(prev, nprev);
    }
    return TDP_OK;
}

// Buffers of the resident sweep, allocated before any capture: exchange
// buffer (two parities of every tile's two-level band), tile flags with the abort word, its pinned mirror, and device
// copies of the forcing tables the loop reads.
static int ensure_res(tdp_op *op, int T, double rho, int variant)
{
    if (!op->res_shadow) {
        const size_t n = 2 * (size_t)op->ncu * std::max(res_band_bytes(true), res_band_bytes(false));
        if (hipMalloc(&op->res_shadow, n) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "device allocation of the exchange buffer failed");
    }
    if (!op->res_flags) {
        const size_t n = (size_t)op->ncu * TDP_RES_FLAG_STRIDE + TDP_RES_FLAG_STRIDE;
        if (hipMalloc(&op->res_flags, sizeof(int) * n) != hipSuccess ||
            hipHostMalloc(&op->res_host, sizeof(int)) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "allocation of the tile flags failed");
        op->res_ntiles = op->ncu;
    }
    const int tabvs[2] = {0, 2};
    for (int q = 0; q < (variant ? 2 : 1); ++q) {
        const auto key = std::make_tuple(T, rho, tabvs[q]);
        if (op->dtables.count(key)) continue;
        const std::vector<double> &h = forcing_table(op, T, rho, tabvs[q]);
        double *d = nullptr;
        if (hipMalloc(&d, sizeof(double) * h.size()) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "device allocation of a forcing table failed");
        if (hipMemcpy(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            TDP_FAIL(TDP_EHIP, "copy of a forcing table failed");
        }
        op->dtables.emplace(key, d);
    }
    return TDP_OK;
}

// After a resident loop: the abort word is raised when a tile waited in vain
// for a neighbour, which happens when not every tile was resident at once
// (other work holding compute units).  Returns 1 then, else TDP_OK or a HIP
// error.
static int res_check(tdp_op *op, int ntiles)
{
    hipStream_t s = op->stream;
    TDP_CHECK_HIP(hipMemcpyAsync(op->res_host, op->res_flags + (size_t)ntiles * TDP_RES_FLAG_STRIDE,
                                 sizeof(int), hipMemcpyDeviceToHost, s));
    TDP_CHECK_HIP(hipStreamSynchronize(s));
    return *op->res_host ? 1 : TDP_OK;
}

// Streamed 3-D loop with two steps per launch, ping-ponging between the field
// pairs (u0, u1) and (v0, v1); an odd last step runs the one-step kernel in place.
static int issue_steps_3d2(tdp_op *op, const LoopBufs &lb, int T, double rho, int zc, int shape,
                           const void *Fin, int tabv, double *out_final, double *out_snap)
{
    hipStream_t s = op->stream;
    const ForcingSrc tab = forcing_src(op, T, rho, tabv, lb);
    const int64_t Ns = (int64_t)T * op->nP, jsnap = out_snap ? Ns - snap_lag(op->nP) : -1;
    const bool f64 = op->prec == TDP_F64;
    const size_t fb = (f64 ? sizeof(double) : sizeof(float)) * op->N;
    void *cur = lb.u0, *prev = lb.u1, *ncur = lb.v0, *nprev = lb.v1;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    auto out_for = [&](int64_t j1) -> double * {      // destination of u_{j1}, if any
        return j1 == jsnap ? out_snap : (j1 == Ns ? out_final : nullptr);
    };
    Stream2Args a;
    for (int k = 0; k < 3; ++k) a.n[k] = op->n[k];
    a.sc = op->sc;
    a.mc = op->mc;
    a.zc = zc;
    a.ncu = op->ncu;
    a.m = f64 ? (const void *)op->m : (const void *)op->m32;
    a.dn = f64 ? (const void *)op->dn : (const void *)op->dn32;
    a.F = Fin;
    int64_t j = 0;
    for (; j + 2 <= Ns; j += 2) {
        a.u = cur;
        a.up = prev;
        a.u2out = ncur;
        a.u1out = nprev;
        a.fa[0] = tab.a(j);
        a.fb[0] = tab.b(j);
        a.fa[1] = tab.a(j + 1);
        a.fb[1] = tab.b(j + 1);
        a.out1 = out_for(j + 1);
        a.out2 = out_for(j + 2);
        if (f64)
            TDP_CHECK_HIP(launch_sweep3d_stream2_f64(a, op->st_step, shape, s));
        else
            TDP_CHECK_HIP(launch_sweep3d_stream2_f32(a, op->st_step32, shape, s));
        std::swap(cur, ncur);
        std::swap(prev, nprev);
    }
    if (j < Ns) {
        SweepArgs b;
        b.ndim = op->ndim;
        for (int k = 0; k < 3; ++k) b.n[k] = op->n[k];
        b.sc = op->sc;
        b.mc = op->mc;
        b.u = cur;
        b.up = prev;
        b.m = a.m;
        b.dn = a.dn;
        b.F = Fin;
        b.out = out_for(j + 1);
        if (f64)
            TDP_CHECK_HIP(launch_sweep3d_stream_f64(b, op->st_step, tab.a(j), tab.b(j), shape, zc, s));
        else
            TDP_CHECK_HIP(launch_sweep3d_stream_f32(b, op->st_step32, (float)tab.a(j),
                                                    (float)tab.b(j), shape, zc, s));
    }
    return TDP_OK;
}

// One step per launch on a real field (kernel 1, or kernel 3 in 3-D),
// u0/u1 swapped in place.
static int issue_steps_real1(tdp_op *op, const LoopBufs &lb, int T, double rho, int kern,
                             int depth, int shape3, const void *Fin, int tabv, double *out_final,
                             double *out_snap)
{
    hipStream_t s = op->stream;
    const ForcingSrc tab = forcing_src(op, T, rho, tabv, lb);
    const int64_t Ns = (int64_t)T * op->nP, jsnap = out_snap ? Ns - snap_lag(op->nP) : -1;
    const size_t fb = (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    void *cur = lb.u0, *prev = lb.u1;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    SweepArgs a;
    a.ndim = op->ndim;
    for (int k = 0; k < 3; ++k) a.n[k] = op->n[k];
    a.sc = op->sc;
    a.mc = op->mc;
    a.F = Fin;
    a.m = op->prec == TDP_F64 ? (const void *)op->m : (const void *)op->m32;
    a.dn = op->prec == TDP_F64 ? (const void *)op->dn : (const void *)op->dn32;
    for (int64_t j = 0; j < Ns; ++j) {
        a.u = cur;
        a.up = prev;
        const double fa = tab.a(j), fbv = tab.b(j);
        a.out = (j + 1 == jsnap) ? out_snap : (j + 1 == Ns ? out_final : nullptr);
        if (kern == 3) {
            if (op->prec == TDP_F64)
                TDP_CHECK_HIP(launch_sweep3d_stream_f64(a, op->st_step, fa, fbv, shape3, depth, s));
            else
                TDP_CHECK_HIP(launch_sweep3d_stream_f32(a, op->st_step32, (float)fa, (float)fbv,
                                                        shape3, depth, s));
        } else if (op->prec == TDP_F64) {
            TDP_CHECK_HIP(launch_sweep_f64(a, op->st_step, fa, fbv, s));
        } else {
            TDP_CHECK_HIP(launch_sweep_f32(a, op->st_step32, (float)fa, (float)fbv, s));
        }
        std::swap(cur, prev);
    }
    return TDP_OK;
}

// Issue the recurrence loop reading F (complex128, or float2 staged for FP32)
// and writing U (complex128).  variant 0: Table 1 (real field; u_{N_s} to
// Re U and the sample u_{N_s - q} to Im U, see snap_lag).  variant 1:
// Definition 4.  Its recurrence has real coefficients, so the real and
// imaginary parts of the complex field are two real recurrences driven by the
// real and imaginary parts of the forcing: with the blocked or streamed
// kernels they run as two real passes (tables 0 and 2), with kernel 1 as one
// complex pass.  The cell damping runs I_abd, whose recurrence has real
// coefficients too: the blocked 2-D kernel advances both parts per launch
// (sharing the coefficients and F), kernel 1 the complex field.
static int issue_steps_loop(tdp_op *op, const LoopBufs &lb, int T, double rho, int variant,
                            const void *Fin, void *U)
{
    int kern, depth, tile;
    sweep_plan(op, variant, &kern, &depth, &tile, !lb.table_free);
    double *Ud = (double *)U;
    auto real_pass = [&](int tabv, double *fin, double *snap) -> int {
        if (kern == 5) return issue_steps_res(op, lb, T, rho, depth, Fin, tabv, fin, snap);
        if (kern == 2) return issue_steps_tb(op, lb, T, rho, depth, tile, Fin, tabv, fin, snap);
        if (kern == 4) return issue_steps_3d2(op, lb, T, rho, depth, tile, Fin, tabv, fin, snap);
        return issue_steps_real1(op, lb, T, rho, kern, depth, tile, Fin, tabv, fin, snap);
    };
    if (op->dform == TDP_DAMP_CELL && kern == 2)
        return issue_steps_abd2(op, lb, T, rho, depth, tile, Fin, Ud);
    if (variant == 0) return real_pass(0, Ud, Ud + 1);
    if (op->dform == TDP_DAMP_NODE && kern != 1) {
        TDP_CHECK(real_pass(0, Ud, nullptr));
        return real_pass(2, Ud + 1, nullptr);
    }
    hipStream_t s = op->stream;
    const std::vector<double> &tab = forcing_table(op, T, rho, variant);
    const int64_t Ns = (int64_t)T * op->nP;
    const size_t fb = 2 * (op->prec == TDP_F64 ? sizeof(double) : sizeof(float)) * op->N;
    void *cur = op->u2, *prev = op->u3, *nxt = op->u4;
    TDP_CHECK_HIP(launch_fill_zero(cur, fb, s));
    TDP_CHECK_HIP(launch_fill_zero(prev, fb, s));
    SweepArgs a;
    a.ndim = op->ndim;
    for (int k = 0; k < 3; ++k) a.n[k] = op->n[k];
    a.sc = op->sc;
    a.mc = op->mc;
    a.F = Fin;
    a.m = op->prec == TDP_F64 ? (const void *)op->m : (const void *)op->m32;
    a.dn = op->prec == TDP_F64 ? (const void *)op->dn : (const void *)op->dn32;
    for (int64_t j = 0; j < Ns; ++j) {
        a.u = cur;
        a.up = prev;
        const double fa = tab[2 * j], fbv = tab[2 * j + 1];
        a.out = (j + 1 == Ns) ? Ud : nullptr;
        if (op->dform == TDP_DAMP_CELL) {
            // I_abd reads u_{n-1} at the neighbours: three fields rotate
            if (op->prec == TDP_F64)
                TDP_CHECK_HIP(launch_sweep_abd_f64(a, nxt, op->rc, op->st_step, op->st_B,
                                                   op->cos_th, fa, fbv, s));
            else
                TDP_CHECK_HIP(launch_sweep_abd_f32(a, nxt, op->rc32, op->st_step32, op->st_B32,
                                                   (float)op->cos_th, (float)fa, (float)fbv, s));
            void *t = prev;
            prev = cur;
            cur = nxt;
            nxt = t;
            continue;
        }
        if (op->prec == TDP_F64)
            TDP_CHECK_HIP(launch_sweep_c_f64(a, op->st_step, fa, fbv, s));
        else
            TDP_CHECK_HIP(launch_sweep_c_f32(a, op->st_step32, (float)fa, (float)fbv, s));
        std::swap(cur, prev);
    }
    return TDP_OK;
}

static int issue_steps(tdp_op *op, const LoopBufs &lb, int T, double rho, int variant,
                       const void *Fin, void *U)
{
    TDP_CHECK(issue_steps_loop(op, lb, T, rho, variant, Fin, U));
    if (variant == 0 && op->nP % 4 != 0) {
        const double phi = 2.0 * M_PI * (double)snap_lag(op->nP) / op->nP;
        TDP_CHECK_HIP(launch_phase_extract(U, op->N, std::cos(phi), std::sin(phi), op->stream));
    }
    return TDP_OK;
}

static int res_finish(tdp_op *op, int ntiles, int T, double rho, int variant, const void *F,
                      void *U, bool direct, int *pending);

// direct: F and U are buffers owned by the op (GMRES work vectors), so the
// loop may be captured on them; otherwise a captured loop works on the
// staging buffers, with copies of F in and U out around the replay.
// pending (GMRES): when the resident sweep ran, its abort word is copied to
// op->res_host without waiting, and *pending receives its tile count (else
// 0); the caller reads op->res_host at its next synchronisation and, if
// the word is raised, calls res_redo for this application.
static int precond_impl(tdp_op *op, int T, double rho, int variant, const void *F, void *U,
                        bool direct = false, int *pending = nullptr)
{
    if (pending) *pending = 0;
    if (T < 1) TDP_FAIL(TDP_EINVAL, "periods_T must be >= 1");
    if (rho <= 0.0) rho = 1.0 / T;
    if (rho > 1.0) TDP_FAIL(TDP_EINVAL, "rho must be <= 1");
    if (variant != 0 && variant != 1) TDP_FAIL(TDP_EINVAL, "variant must be 0 or 1");
    if (op->dform == TDP_DAMP_CELL && variant == 0)
        TDP_FAIL(TDP_EINVAL, "Table 1 runs I_acd: with the cell damping use the complex form (S_T^abd)");
    const int64_t Ns = (int64_t)T * op->nP;
    if (Ns > TDP_MAX_STEPS)
        TDP_FAIL(TDP_EINVAL, "N_s = periods_T n_P = %lld exceeds 2^24", (long long)Ns);
    if (variant) TDP_CHECK(ensure_complex_fields(op));
    int64_t launches;
    int res_nt = 0;      // tiles of the resident sweep, when it runs
    {   // allocate before any stream capture: no allocation may happen inside it
        int kern, depth, tile;
        sweep_plan(op, variant, &kern, &depth, &tile);
        if (kern == 2 || kern == 4 || kern == 5) TDP_CHECK(ensure_tb_fields(op));
        if (kern == 4) sweep3d_stream2_prepare(op->prec == TDP_F64, tile);
        if (kern == 5) {
            TDP_CHECK(ensure_res(op, T, rho, variant));
            res_nt = res_tiles(op->n[0], op->n[1], depth, op->prec == TDP_F64, nullptr, nullptr);
        }
        launches = kern == 2 ? (Ns + depth - 1) / depth
                 : kern == 4 ? (Ns + 1) / 2
                 : kern == 5 ? 2 * ((Ns + TDP_RES_MAXSTEPS - 1) / TDP_RES_MAXSTEPS)
                             : Ns;
        // two real passes (one launch for both with the blocked I_abd kernel)
        if (variant == 1 && kern != 1 && !(op->dform == TDP_DAMP_CELL && kern == 2)) launches *= 2;
    }
    const LoopBufs lb{op->u0, op->u1, op->v0, op->v1, false};
    hipStream_t s = op->stream;
    // a graph holds one kernel node per launch: very long loops are issued
    // directly instead of being captured
    if (!op->tune.use_graph || launches > TDP_MAX_GRAPH_LAUNCHES) {
        const void *Fin = F;
        if (op->prec == TDP_F32) {
            TDP_CHECK_HIP(launch_cvt_c128_to_c64(F, op->Fst, op->N, s));
            Fin = op->Fst;
        }
        TDP_CHECK(issue_steps(op, lb, T, rho, variant, Fin, U));
        return res_nt ? res_finish(op, res_nt, T, rho, variant, F, U, direct, pending) : TDP_OK;
    }
    // captured loop: on F and U themselves (direct), else reading op->Fstage
    // (F64) / op->Fst (F32) and writing op->Ustage
    auto key = std::make_tuple(T, rho, variant, op->tune.kernel, op->tune.tb_depth, op->tune.tile,
                               direct ? F : nullptr, direct ? (const void *)U : nullptr);
    auto it = op->graphs.find(key);
    if (it == op->graphs.end()) {
        hipGraph_t g;
        TDP_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = TDP_OK;
        if (direct) {
            if (op->prec == TDP_F32) {
                const hipError_t e = launch_cvt_c128_to_c64(F, op->Fst, op->N, s);
                if (e != hipSuccess) {
                    set_error("launch_cvt_c128_to_c64 failed: %s", hipGetErrorString(e));
                    rc = TDP_EHIP;
                }
            }
            if (rc == TDP_OK)
                rc = issue_steps(op, lb, T, rho, variant, op->prec == TDP_F64 ? F : op->Fst, U);
        } else {
            rc = issue_steps(op, lb, T, rho, variant, op->prec == TDP_F64 ? op->Fstage : op->Fst,
                             op->Ustage);
        }
        hipError_t ce = hipStreamEndCapture(s, &g);
        if (rc != TDP_OK) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            return rc;
        }
        TDP_CHECK_HIP(ce);
        hipGraphExec_t ge;
        hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        TDP_CHECK_HIP(ie);
        // each graph holds N_s launch nodes: keep at most kMaxGraphs per op
        if (op->graphs.size() >= kMaxGraphs) {
            TDP_CHECK_HIP(hipStreamSynchronize(s));
            for (auto &kv : op->graphs) (void)hipGraphExecDestroy(kv.second);
            op->graphs.clear();
        }
        it = op->graphs.emplace(key, ge).first;
    }
    if (direct) {
        TDP_CHECK_HIP(hipGraphLaunch(it->second, s));
        return res_nt ? res_finish(op, res_nt, T, rho, variant, F, U, direct, pending) : TDP_OK;
    }
    if (op->prec == TDP_F64)
        TDP_CHECK_HIP(hipMemcpyAsync(op->Fstage, F, 16 * op->N, hipMemcpyDeviceToDevice, s));
    else
        TDP_CHECK_HIP(launch_cvt_c128_to_c64(F, op->Fst, op->N, s));
    TDP_CHECK_HIP(hipGraphLaunch(it->second, s));
    TDP_CHECK_HIP(hipMemcpyAsync(U, op->Ustage, 16 * op->N, hipMemcpyDeviceToDevice, s));
    return res_nt ? res_finish(op, res_nt, T, rho, variant, F, U, direct, pending) : TDP_OK;
}

// A resident loop that ended early is redone with the blocked sweep, and the
// op stops using the resident kernel (its tuning goes back to auto).
static int res_redo(tdp_op *op, int T, double rho, int variant, const void *F, void *U,
                    bool direct)
{
    ++op->res_aborts;
    op->tune.kernel = 0;
    op->tune.tb_depth = 0;
    op->tune.tile = 0;
    return precond_impl(op, T, rho, variant, F, U, direct);
}

static int res_finish(tdp_op *op, int ntiles, int T, double rho, int variant, const void *F,
                      void *U, bool direct, int *pending)
{
    if (pending) {          // the caller reads the word at its next synchronisation
        TDP_CHECK_HIP(hipMemcpyAsync(op->res_host, op->res_flags + (size_t)ntiles * TDP_RES_FLAG_STRIDE,
                                     sizeof(int), hipMemcpyDeviceToHost, op->stream));
        *pending = ntiles;
        return TDP_OK;
    }
    const int rc = res_check(op, ntiles);
    if (rc != 1) return rc;
    return res_redo(op, T, rho, variant, F, U, direct);
}

int precond_noalloc_impl(tdp_op *op, int T, double rho, const void *F, void *U,
                         const LoopBufs &bufs, void *f32_stage)
{
    if (T < 1) TDP_FAIL(TDP_EINVAL, "periods_T must be >= 1");
    if (rho <= 0.0) rho = 1.0 / T;
    if (rho > 1.0) TDP_FAIL(TDP_EINVAL, "rho must be <= 1");
    if (op->dform == TDP_DAMP_CELL)
        TDP_FAIL(TDP_EINVAL, "Table 1 runs I_acd: with the cell damping use the complex form (S_T^abd)");
    const int64_t Ns = (int64_t)T * op->nP;
    if (Ns > TDP_MAX_STEPS)
        TDP_FAIL(TDP_EINVAL, "N_s = periods_T n_P = %lld exceeds 2^24", (long long)Ns);
    const void *Fin = F;
    if (op->prec == TDP_F32) {
        TDP_CHECK_HIP(launch_cvt_c128_to_c64(F, f32_stage, op->N, op->stream));
        Fin = f32_stage;
    }
    LoopBufs lb = bufs;
    lb.table_free = true;
    return issue_steps(op, lb, T, rho, 0, Fin, U);
}

static int precond_entry(const tdp_op *cop, int T, double rho, int variant, const void *F, void *U)
{
    clear_error();
    if (!cop || !F || !U) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (F == U) TDP_FAIL(TDP_EINVAL, "F and U must not alias");
    if (misaligned16(F) || misaligned16(U)) TDP_FAIL(TDP_EINVAL, "complex arrays must be 16-byte aligned");
    tdp_op *op = const_cast<tdp_op *>(cop);
    StreamJoin join(op->user_stream, op->stream, op->ev);
    return precond_impl(op, T, rho, variant, F, U);
}

extern "C" int tdp_precond_apply(const tdp_op *op, int T, double rho, const void *F, void *U)
{
    return precond_entry(op, T, rho, 0, F, U);
}

extern "C" int tdp_precond_apply_complex(const tdp_op *op, int T, double rho, const void *F,
                                         void *U)
{
    return precond_entry(op, T, rho, 1, F, U);
}

// Autotuner: times every sweep variant that applies to this op (one step per
// launch; blocked tiles x depths in 2-D) on `periods_T` periods of the loop,
// with HIP events on the op's stream, keeps the fastest.
extern "C" int tdp_op_autotune(tdp_op *op, int periods_T, double rho, int variant,
                               tdp_tuning *best, double *table, int cap)
{
    clear_error();
    if (!op) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (periods_T < 1) TDP_FAIL(TDP_EINVAL, "periods_T must be >= 1");
    if (variant != 0 && variant != 1) TDP_FAIL(TDP_EINVAL, "variant must be 0 or 1");
    if (op->dform == TDP_DAMP_CELL) variant = 1;      // S_T^abd: the complex form
    StreamJoin join(op->user_stream, op->stream, op->ev);
    hipStream_t s = op->stream;
    std::vector<tdp_tuning> cand;
    cand.push_back({1, 0, 1, 0});
    if (op->ndim == 2 && op->dform == TDP_DAMP_NODE) {
        const int depths[] = {2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16};
        for (int tile = 0; tile <= 15; ++tile) {
            if (tb2d_f32_only(tile) && op->prec == TDP_F64) continue;
            if ((tile == 14 || tile == 15) && op->mc > 2) continue;
            const int rows = tb2d_tile_rows(tile, op->prec == TDP_F64);
            for (int k : depths)
                if (4 * k <= rows && 4 * k <= tb2d_tile_cols(tile)) cand.push_back({2, k, 1, tile});
        }
    }
    for (int k : {2, 4, 6, 8})
        if (res_applies(op, k)) cand.push_back({5, k, 1, 0});
    if (op->ndim == 2 && op->dform == TDP_DAMP_CELL && op->mc <= 2) {
        for (int tile = 4; tile <= 7; ++tile) {
            if (!abd_tile_ok(tile, op->prec == TDP_F64)) continue;
            const int rows = tb2d_tile_rows(tile, op->prec == TDP_F64);
            for (int k : {2, 3, 4, 6, 8})
                if (4 * k <= rows) cand.push_back({2, k, 1, tile});
        }
    }
    if (op->ndim == 3 && op->dform == TDP_DAMP_NODE) {
        for (int shape = 0; shape < 3; ++shape)
            for (int zc : {4, 8, 16, 32, 64}) cand.push_back({3, zc, 1, shape});
        // two-step kernel: the depth is only the fewest planes per workgroup
        // run (it matters on small grids); FP64 runs shape 2 as shape 1
        for (int shape = 0; shape < 3; ++shape) {
            if (shape == 2 && op->prec == TDP_F64) continue;
            for (int zc : {8, 32}) cand.push_back({4, zc, 1, shape});
        }
    }
    const tdp_tuning saved = op->tune;
    void *tin = nullptr, *tout = nullptr;
    if (hipMalloc(&tin, 16 * op->N) != hipSuccess || hipMalloc(&tout, 16 * op->N) != hipSuccess) {
        (void)hipFree(tin);
        TDP_FAIL(TDP_ENOMEM, "autotune buffers");
    }
    TDP_CHECK_HIP(launch_fill_zero(tin, 16 * op->N, s));
    hipEvent_t e0, e1;
    TDP_CHECK_HIP(hipEventCreate(&e0));
    TDP_CHECK_HIP(hipEventCreate(&e1));
    // every candidate is run once (graph capture, first touch), then timed in
    // two interleaved passes; a candidate's time is its faster pass, so clock
    // ramps and ordering do not favour the candidates timed later
    const int reps = 2, passes = 2;
    const double steps = (double)periods_T * op->nP * reps;
    std::vector<double> per_step(cand.size(), INFINITY);
    int rc = TDP_OK;
    for (size_t i = 0; i < cand.size() && rc == TDP_OK; ++i) {
        op->tune = cand[i];
        rc = precond_impl(op, periods_T, rho, variant, tin, tout);
    }
    for (int pass = 0; pass < passes && rc == TDP_OK; ++pass) {
        for (size_t i = 0; i < cand.size(); ++i) {
            op->tune = cand[i];
            if (hipEventRecord(e0, s) != hipSuccess) { rc = TDP_EHIP; break; }
            for (int r = 0; r < reps && rc == TDP_OK; ++r)
                rc = precond_impl(op, periods_T, rho, variant, tin, tout);
            if (rc != TDP_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = TDP_EHIP;
                break;
            }
            per_step[i] = std::min(per_step[i], ms / steps);
        }
    }
    double best_ms = INFINITY;
    tdp_tuning bt = saved;
    int i = 0;
    for (; rc == TDP_OK && i < (int)cand.size(); ++i) {
        const tdp_tuning &c = cand[i];
        const double per = per_step[i];
        if (table && i < cap) {
            table[4 * i] = c.kernel;
            table[4 * i + 1] = c.tb_depth;
            table[4 * i + 2] = c.tile;
            table[4 * i + 3] = per * 1e3;   // microseconds per step
        }
        if (per < best_ms) {
            best_ms = per;
            bt = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(tin);
    (void)hipFree(tout);
    for (auto &kv : op->graphs) (void)hipGraphExecDestroy(kv.second);
    op->graphs.clear();
    if (rc != TDP_OK) {
        op->tune = saved;
        return rc;
    }
    op->tune = bt;
    if (best) *best = bt;
    return i;
}

// ---------------------------------------------------------------------------
// GMRES
static int ensure_krylov(tdp_op *op, int m)
{
    if (op->V && op->V_cols >= m + 1) return TDP_OK;
    (void)hipStreamSynchronize(op->stream);
    (void)hipFree(op->V);
    op->V = nullptr;
    if (hipMalloc(&op->V, (size_t)16 * op->N * (m + 1)) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "Krylov basis allocation (%d x %lld complex) failed", m + 1,
                 (long long)op->N);
    op->V_cols = m + 1;
    if (!op->wv) {
        if (hipMalloc(&op->wv, 16 * op->N) != hipSuccess || hipMalloc(&op->tv, 16 * op->N) != hipSuccess ||
            hipMalloc(&op->rv, 16 * op->N) != hipSuccess || hipMalloc(&op->xv, 16 * op->N) != hipSuccess)
            TDP_FAIL(TDP_ENOMEM, "GMRES work vector allocation failed");
    }
    const int nblk = blas_nblocks(op->N);
    const size_t rb = sizeof(double) * 2 * (size_t)nblk * (m + 2);
    if (rb > op->red_bytes) {
        (void)hipFree(op->red);
        if (hipMalloc(&op->red, rb) != hipSuccess) TDP_FAIL(TDP_ENOMEM, "allocation failed");
        op->red_bytes = rb;
    }
    (void)hipFree(op->dcoef);
    (void)hipHostFree(op->hres);
    op->dcoef = nullptr;
    op->hres = nullptr;
    const size_t cb = sizeof(double) * (8 * (size_t)(m + 2));
    if (hipMalloc(&op->dcoef, cb) != hipSuccess || hipHostMalloc(&op->hres, cb) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "allocation failed");
    return TDP_OK;
}

// ||x||^2 of a complex vector, result in dres[0] (device) -> host
static int norm2_host(tdp_op *op, const void *x, double *out)
{
    const int nblk = blas_nblocks(op->N);
    TDP_CHECK_HIP(launch_mdot(x, op->N, 1, x, op->N, op->red, nblk, op->dcoef, op->stream));
    TDP_CHECK_HIP(hipMemcpyAsync(op->hres, op->dcoef, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                 op->stream));
    TDP_CHECK_HIP(hipStreamSynchronize(op->stream));
    *out = op->hres[0];
    return TDP_OK;
}

typedef std::complex<double> cplx;

// Restarted GMRES on P H U = P F, the same iteration as the CPU oracle but
// with classical Gram-Schmidt applied twice (fused multi-dot / multi-axpy
// kernels).  Tolerance mode evaluates the true residual of the current iterate
// after every iteration (a multi-axpy, one H-apply and a norm: under 1% of a
// preconditioner application), stops as soon as it is <= tol, and restarts
// the cycle early when the true residual stalls while the Givens estimate
// keeps falling (the Table 1 preconditioner is only real-linear).  Each cycle
// keeps its iterate of least true residual; a Table 1 cycle that does not
// lower the true residual is rejected and the solve continues with the
// complex-linear variant 1, whose cycles always keep their last iterate when
// none lowered the true residual.
static int gmres_impl(tdp_op *op, const tdp_gmres_cfg *cfg, const void *F, void *U,
                      tdp_gmres_info *info)
{
    auto t0 = std::chrono::steady_clock::now();
    const int m = cfg->restart;
    if (m < 1 || m > 512) TDP_FAIL(TDP_EINVAL, "restart must be in [1, 512]");
    if (cfg->max_iters < 1) TDP_FAIL(TDP_EINVAL, "max_iters must be >= 1");
    if (cfg->periods_T < 1) TDP_FAIL(TDP_EINVAL, "periods_T must be >= 1");
    if (!(cfg->tol > 0.0)) TDP_FAIL(TDP_EINVAL, "tol must be > 0");
    if (cfg->rho > 1.0) TDP_FAIL(TDP_EINVAL, "rho must be <= 1");
    if (cfg->variant != 0 && cfg->variant != 1) TDP_FAIL(TDP_EINVAL, "variant must be 0 or 1");
    TDP_CHECK(ensure_krylov(op, m));
    for (hipEvent_t &e : op->tev)
        if (!e) TDP_CHECK_HIP(hipEventCreate(&e));
    hipStream_t s = op->stream;
    const int64_t N = op->N;
    const int T = cfg->periods_T;
    // TDP_LOG=1 in the environment: one stderr line per cycle
    static const bool log_cycles = [] {
        const char *v = std::getenv("TDP_LOG");
        return v && v[0] == '1';
    }();
    // phase timing: GPU time of the preconditioner applications (0), the
    // H-applies (1) and the Gram-Schmidt kernels (2), from event pairs on the
    // op's stream read after its next synchronisation (each phase is recorded
    // at most once between two synchronisations)
    double ms_phase[3] = {0.0, 0.0, 0.0};
    bool pending[3] = {false, false, false};
    auto mark = [&](int ph, int end) -> int {
        TDP_CHECK_HIP(hipEventRecord(op->tev[2 * ph + end], s));
        if (end) pending[ph] = true;
        return TDP_OK;
    };
    auto collect_time = [&]() {
        for (int ph = 0; ph < 3; ++ph) {
            if (!pending[ph]) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, op->tev[2 * ph], op->tev[2 * ph + 1]) == hipSuccess)
                ms_phase[ph] += ms;
            pending[ph] = false;
        }
    };
    // the resident sweep's abort word is read at the synchronisation that
    // follows (no wait of its own); a raised word redoes the application
    // and the work that used it
    int res_pending = 0;
    auto precond_timed = [&](const void *x, void *y, int var) -> int {
        TDP_CHECK(mark(0, 0));
        TDP_CHECK(precond_impl(op, T, cfg->rho, var, x, y, true, &res_pending));
        return mark(0, 1);
    };
    auto res_aborted = [&]() -> bool { return res_pending && *op->res_host; };
    auto apply_H_timed = [&](const void *x, const void *Fr, void *y) -> int {
        TDP_CHECK(mark(1, 0));
        TDP_CHECK(apply_H_impl(op, x, Fr, y));
        return mark(1, 1);
    };
    const bool tolmode = cfg->fixed_iters <= 0;
    const int limit = tolmode ? cfg->max_iters : cfg->fixed_iters;
    const int nblk = blas_nblocks(N);
    char *V = (char *)op->V;
    auto col = [&](int k) -> void * { return V + (size_t)16 * N * k; };
    double *d1 = op->dcoef;                 // CGS pass 1 coefficients [2(m+1)]
    double *d2 = op->dcoef + 2 * (m + 1);   // pass 2
    double *dn2 = op->dcoef + 4 * (m + 1);  // ||w||^2
    double *dy = op->dcoef + 4 * (m + 1) + 2;

    double b2;
    TDP_CHECK(norm2_host(op, F, &b2));
    const double bnorm = std::sqrt(b2);
    if (!std::isfinite(bnorm)) TDP_FAIL(TDP_EINVAL, "F holds NaN or Inf");   // nothing written
    if (!cfg->x0_given) TDP_CHECK_HIP(launch_fill_zero(U, 16 * N, s));
    int its = 0, restarts = 0, nhist = 0, status = TDP_ENOTCONV;
    int variant = op->dform == TDP_DAMP_CELL ? 1 : cfg->variant, switched = 0;
    int64_t napply = 0;
    double pnorm0 = -1.0, est = 1.0, rel = 1.0;
    std::vector<cplx> Hm((size_t)(m + 1) * m), gv(m + 1), sn(m), y(m), ybest(m);
    std::vector<double> cs(m);
    auto HM = [&](int i, int j) -> cplx & { return Hm[(size_t)j * (m + 1) + i]; };
    auto solve_y = [&](int k_used) {
        for (int k = k_used - 1; k >= 0; --k) {
            cplx sum = gv[k];
            for (int j = k + 1; j < k_used; ++j) sum -= HM(k, j) * y[j];
            y[k] = sum / HM(k, k);
        }
    };
    // x_out = x_in + V y  (y from the host), x_out may equal x_in
    auto update = [&](void *x_out, const void *x_in, int k_used) -> int {
        for (int k = 0; k < k_used; ++k) {
            op->hres[2 * k] = y[k].real();
            op->hres[2 * k + 1] = y[k].imag();
        }
        TDP_CHECK_HIP(hipMemcpyAsync(dy, op->hres, sizeof(double) * 2 * k_used,
                                     hipMemcpyHostToDevice, s));
        if (x_out != x_in)
            TDP_CHECK_HIP(hipMemcpyAsync(x_out, x_in, 16 * N, hipMemcpyDeviceToDevice, s));
        TDP_CHECK_HIP(launch_maxpy(x_out, op->V, N, k_used, dy, 1.0, N, s));
        return TDP_OK;
    };
    if (bnorm == 0.0) {
        TDP_CHECK_HIP(launch_fill_zero(U, 16 * N, s));
        status = TDP_OK;
        rel = 0.0;
        est = 0.0;
    }
    while (status != TDP_OK) {
        double r2;
        TDP_CHECK(apply_H_timed(U, F, op->rv));   // r = F - H U
        TDP_CHECK(norm2_host(op, op->rv, &r2));
        collect_time();
        rel = std::sqrt(r2) / bnorm;
        if (!std::isfinite(rel) && its == 0 && restarts == 0)   // U is still the caller's x0
            TDP_FAIL(TDP_EINVAL, "non-finite residual: the initial U holds NaN or Inf");
        if (tolmode && rel <= cfg->tol) {
            status = TDP_OK;
            break;
        }
        if (its >= limit) break;
        TDP_CHECK(precond_timed(op->rv, col(0), variant));
        ++napply;
        double z2;
        TDP_CHECK(norm2_host(op, col(0), &z2));
        if (res_aborted()) {
            res_pending = 0;
            TDP_CHECK(res_redo(op, T, cfg->rho, variant, op->rv, col(0), true));
            TDP_CHECK(norm2_host(op, col(0), &z2));
        }
        collect_time();
        const double beta0 = std::sqrt(z2);
        if (pnorm0 < 0.0) pnorm0 = beta0;
        if (beta0 == 0.0) break;
        // norm2_host left ||col0||^2 in dcoef[0]
        TDP_CHECK_HIP(launch_scale_by_invnorm(col(0), col(0), op->dcoef, N, s));
        for (int k = 0; k <= m; ++k) gv[k] = 0.0;
        gv[0] = beta0;
        double rel_start = rel, rel_prev = rel, best_rel = rel, rel_last = rel;
        int k_used = 0, best_k = 0;       // best_k: the cycle's candidate with the
        bool converged = false;           // smallest true residual (0: the start)
        for (int i = 0; i < m && its < limit; ++i) {
            TDP_CHECK(apply_H_timed(col(i), nullptr, op->tv));
            TDP_CHECK(precond_timed(op->tv, op->wv, variant));
            ++napply;
            ++its;
            // classical Gram-Schmidt, two passes (w = P H v_i is only read
            // and rewritten in place, v_{i+1} only written: both are redone
            // from P H v_i if the application is)
            auto cgs2 = [&]() -> int {
                TDP_CHECK(mark(2, 0));
                TDP_CHECK_HIP(launch_mdot(op->V, N, i + 1, op->wv, N, op->red, nblk, d1, s));
                TDP_CHECK_HIP(launch_maxpy(op->wv, op->V, N, i + 1, d1, -1.0, N, s));
                TDP_CHECK_HIP(launch_mdot(op->V, N, i + 1, op->wv, N, op->red, nblk, d2, s));
                TDP_CHECK_HIP(launch_maxpy(op->wv, op->V, N, i + 1, d2, -1.0, N, s));
                TDP_CHECK_HIP(launch_mdot(op->wv, N, 1, op->wv, N, op->red, nblk, dn2, s));
                TDP_CHECK_HIP(launch_scale_by_invnorm(col(i + 1), op->wv, dn2, N, s));
                TDP_CHECK(mark(2, 1));
                TDP_CHECK_HIP(hipMemcpyAsync(op->hres, op->dcoef, sizeof(double) * (4 * (m + 1) + 2),
                                             hipMemcpyDeviceToHost, s));
                TDP_CHECK_HIP(hipStreamSynchronize(s));
                return TDP_OK;
            };
            TDP_CHECK(cgs2());
            if (res_aborted()) {
                res_pending = 0;
                TDP_CHECK(res_redo(op, T, cfg->rho, variant, op->tv, op->wv, true));
                TDP_CHECK(cgs2());
            }
            collect_time();
            const double *h1 = op->hres, *h2 = op->hres + 2 * (m + 1);
            for (int k = 0; k <= i; ++k)
                HM(k, i) = cplx(h1[2 * k] + h2[2 * k], h1[2 * k + 1] + h2[2 * k + 1]);
            const double hn = std::sqrt(op->hres[4 * (m + 1)]);
            HM(i + 1, i) = hn;
            for (int k = 0; k < i; ++k) {
                const cplx a = HM(k, i), b = HM(k + 1, i);
                HM(k, i) = cs[k] * a + sn[k] * b;
                HM(k + 1, i) = -std::conj(sn[k]) * a + cs[k] * b;
            }
            const cplx a = HM(i, i);
            const double rr = std::hypot(std::abs(a), hn);
            if (std::abs(a) == 0.0) {
                cs[i] = 0.0;
                sn[i] = 1.0;
                HM(i, i) = hn;
            } else {
                const cplx ph = a / std::abs(a);
                cs[i] = std::abs(a) / rr;
                sn[i] = ph * hn / rr;
                HM(i, i) = ph * rr;
            }
            HM(i + 1, i) = 0.0;
            gv[i + 1] = -std::conj(sn[i]) * gv[i];
            gv[i] = cs[i] * gv[i];
            est = std::abs(gv[i + 1]) / pnorm0;
            const double est_cycle = std::abs(gv[i + 1]) / beta0;
            if (info && info->history && nhist < info->history_cap) info->history[nhist] = est;
            ++nhist;
            k_used = i + 1;
            if (tolmode) {
                solve_y(k_used);
                TDP_CHECK(update(op->xv, U, k_used));
                TDP_CHECK(apply_H_timed(op->xv, F, op->rv));
                TDP_CHECK(norm2_host(op, op->rv, &r2));
                collect_time();
                const double relt = std::sqrt(r2) / bnorm;
                rel_last = relt;
                if (relt < best_rel) {
                    best_rel = relt;
                    best_k = k_used;
                    std::copy(y.begin(), y.begin() + k_used, ybest.begin());
                }
                if (relt <= cfg->tol) {
                    converged = true;
                    break;
                }
                if (hn == 0.0) break;
                if (!(relt <= 1e6 * rel_start)) break;      // runaway or non-finite
                if (relt > 2.0 * rel_start * est_cycle && relt > 0.7 * rel_prev) break;
                rel_prev = relt;
            } else if (hn == 0.0) {
                break;
            }
        }
        ++restarts;
        if (tolmode) {
            // keep the best iterate of the cycle; a cycle that did not lower the
            // true residual is rejected (x unchanged)
            if (best_k == 0 && k_used > 0 && variant != 0) {
                // complex-linear P: the Arnoldi relation is exact, so the cycle's
                // last iterate (least preconditioned residual) is kept regardless
                best_k = k_used;
                best_rel = rel_last;
            }
            if (best_k > 0 && best_k == k_used) {
                TDP_CHECK_HIP(hipMemcpyAsync(U, op->xv, 16 * N, hipMemcpyDeviceToDevice, s));
            } else if (best_k > 0) {
                std::copy(ybest.begin(), ybest.begin() + best_k, y.begin());
                TDP_CHECK(update(U, U, best_k));
            }
            rel = best_rel;
            if (log_cycles)
                std::fprintf(stderr,
                             "tdp gmres: cycle %d its %d variant %d kept %d/%d true relres %.3e "
                             "(start %.3e) est %.3e%s\n",
                             restarts, its, variant, best_k, k_used, best_rel, rel_start, est,
                             best_k == 0 && k_used > 0 ? " rejected" : "");
            if (best_k == 0 && k_used > 0) {      // Table 1 cycle rejected:
                variant = 1;                      // continue with Definition 4
                switched = 1;
            }
        } else if (k_used > 0) {
            solve_y(k_used);
            TDP_CHECK(update(U, U, k_used));
        }
        if (converged) {
            status = TDP_OK;
            break;
        }
        if (!tolmode && its >= limit) {
            TDP_CHECK(apply_H_timed(U, F, op->rv));
            TDP_CHECK(norm2_host(op, op->rv, &r2));
            collect_time();
            rel = std::sqrt(r2) / bnorm;
            status = TDP_OK;
            break;
        }
        if (its >= limit) break;
    }
    TDP_CHECK_HIP(hipStreamSynchronize(s));
    collect_time();
    if (log_cycles)
        std::fprintf(stderr, "tdp gmres: %s after %d iterations, %d cycles, true relres %.3e, "
                             "%.1f ms (preconditioner %.1f ms)\n",
                     status == TDP_OK ? "done" : "not converged", its, restarts, rel,
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(),
                     ms_phase[0]);
    if (info) {
        info->iters = its;
        info->restarts = restarts;
        info->relres_true = rel;
        info->relres_prec = est;
        info->steps = napply * (int64_t)T * op->nP;
        info->history_len = nhist < info->history_cap ? nhist : info->history_cap;
        info->switched = switched;
        info->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->ms_precond = ms_phase[0];
        info->ms_H = ms_phase[1];
        info->ms_arnoldi = ms_phase[2];
    }
    return status;
}

extern "C" int tdp_gmres_solve(const tdp_op *cop, const tdp_gmres_cfg *cfg, const void *F,
                               void *U, tdp_gmres_info *info)
{
    clear_error();
    if (!cop || !cfg || !F || !U) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (F == U) TDP_FAIL(TDP_EINVAL, "F and U must not alias");
    if (misaligned16(F) || misaligned16(U)) TDP_FAIL(TDP_EINVAL, "complex arrays must be 16-byte aligned");
    tdp_op *op = const_cast<tdp_op *>(cop);
    StreamJoin join(op->user_stream, op->stream, op->ev);
    return gmres_impl(op, cfg, F, U, info);
}

// ---------------------------------------------------------------------------
extern "C" int tdp_grad_m(const tdp_op *cop, const void *lam, const void *U, double *grad)
{
    clear_error();
    if (!cop || !lam || !U || !grad) TDP_FAIL(TDP_EINVAL, "NULL argument");
    if (misaligned16(lam) || misaligned16(U)) TDP_FAIL(TDP_EINVAL, "complex arrays must be 16-byte aligned");
    tdp_op *op = const_cast<tdp_op *>(cop);
    if (!op->gcell && hipMalloc(&op->gcell, sizeof(double) * op->Nc) != hipSuccess)
        TDP_FAIL(TDP_ENOMEM, "allocation failed");
    StreamJoin join(op->user_stream, op->stream, op->ev);
    TDP_CHECK_HIP(launch_grad_cells(op->ndim, op->n, op->omega * op->omega, op->M, lam, U,
                                    op->gcell, op->stream));
    TDP_CHECK_HIP(launch_grad_nodes(op->ndim, op->n, op->gcell, grad, op->stream));
    return TDP_OK;
}
