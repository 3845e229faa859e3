// Batched form: many right-hand sides on one medium and many independent 2-D
// problems of uneven sizes advanced together.  Every k-step launch of the
// batched blocked sweeps covers all live fields (each with its own medium,
// stencil constants, forcing table, step count and output): the live
// right-hand sides of a medium go in slabs of several per workgroup through
// the shared-medium tile (the medium is loaded and folded once per slab),
// single fields through the per-field tile.  The whole step schedule of one
// preconditioner application is captured in one hipGraph,
// and restarted GMRES (Sec. 2.4) runs for every field in lockstep: one
// batched preconditioner application per round, with each field following
// exactly the decision sequence of a single solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "tdp_internal.h"

using namespace tdp;
typedef std::complex<double> cplx;

// H-apply of field's operator on the batch stream (y = H x, or F - H x)
static int apply_H_on(const tdp_op *op, const void *x, const void *F, void *y, hipStream_t s)
{
    TDP_CHECK_HIP(launch_apply_H(op->ndim, op->n, op->sc, op->mc, op->m, op->rw, nullptr, op->st_H,
                                 op->st_I, x, F, y, s));
    return TDP_OK;
}

#define TDP_BFAIL(code, ...)           \
    do {                               \
        ::tdp::set_error(__VA_ARGS__); \
        return (code);                 \
    } while (0)

struct tdp_batch {
    std::vector<tdp_op *> ops;
    struct Field {
        int op;
        int64_t N;
        void *a0 = nullptr, *a1 = nullptr, *b0 = nullptr, *b1 = nullptr;   // fields (prec)
        void *Fst = nullptr;     // FP32 staged right-hand side
        void *pin = nullptr, *pout = nullptr;   // preconditioner input / output (c128)
        void *V = nullptr, *rv = nullptr, *xv = nullptr;
        double *red = nullptr, *dco = nullptr;
        int Vcols = 0;
    };
    std::vector<Field> f;
    bool f64 = true, general = false;
    hipStream_t s = nullptr;
    int K = 8, shape = 1;
    int mshape = 0;               // shared-medium tile (-1: every field on its own tile)
    // device copies of per-op forcing tables, keyed by (op, T, rho)
    std::map<std::tuple<int, int, double>, double *> dtab;
    void *dfields = nullptr;      // BFieldT<T>[] for the current (T, rho) set
    std::vector<int> tkey;        // the T of each op the descriptor array was built for
    double rho_key = -1;
    // captured applications keyed by (active mask, T set, rho, K, shape)
    std::map<std::string, std::pair<hipGraphExec_t, int *>> graphs;
    double *hbuf = nullptr;       // pinned host scratch
    size_t hbuf_n = 0;
    // batched Gram-Schmidt: per-field descriptors (pinned host copy and
    // device copy) and the device array the coefficients are gathered into
    GsField *gs_host = nullptr, *gs_dev = nullptr;
    double *gstage = nullptr;
    size_t gs_n = 0, gstage_n = 0;
    // the other batched GMRES steps (update, H-apply, residual norm):
    // descriptors (pinned host, device) and the |r|^2 of every field (two
    // doubles per field, device and pinned host)
    TrField *tr_host = nullptr, *tr_dev = nullptr;
    double *tr_out = nullptr, *tr_outh = nullptr;
    size_t tr_n = 0;
};

static void free_batch(tdp_batch *b)
{
    if (!b) return;
    for (auto &kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.first);
        (void)hipFree(kv.second.second);
    }
    for (auto &kv : b->dtab) (void)hipFree(kv.second);
    for (auto &fl : b->f) {
        void *p[] = {fl.a0, fl.a1, fl.b0, fl.b1, fl.Fst, fl.pin, fl.pout, fl.V, fl.rv, fl.xv,
                     fl.red, fl.dco};
        for (void *q : p) (void)hipFree(q);
    }
    (void)hipFree(b->dfields);
    if (b->hbuf) (void)hipHostFree(b->hbuf);
    if (b->gs_host) (void)hipHostFree(b->gs_host);
    (void)hipFree(b->gs_dev);
    (void)hipFree(b->gstage);
    if (b->tr_host) (void)hipHostFree(b->tr_host);
    if (b->tr_outh) (void)hipHostFree(b->tr_outh);
    (void)hipFree(b->tr_dev);
    (void)hipFree(b->tr_out);
    delete b;
}

extern "C" int tdp_batch_destroy(tdp_batch *b)
{
    if (b && b->s) (void)hipStreamSynchronize(b->s);
    free_batch(b);
    return TDP_OK;
}

extern "C" int tdp_batch_create(tdp_op *const *ops, int nops, const int *nrhs, tdp_batch **out)
{
    if (!ops || nops < 1 || !nrhs || !out) TDP_BFAIL(TDP_EINVAL, "bad batch arguments");
    *out = nullptr;
    tdp_batch *b = new tdp_batch();
    for (int i = 0; i < nops; ++i) {
        tdp_op *op = ops[i];
        if (!op) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "NULL op %d", i); }
        if (op->ndim != 2) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "batched form is 2-D only (op %d)", i); }
        if (op->prec != ops[0]->prec) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "all ops must share one precision"); }
        if (op->dform != TDP_DAMP_NODE) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "the batched form runs Table 1 (diagonal damping only)"); }
        if (op->user_stream != ops[0]->user_stream) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "all ops must share one stream"); }
        (void)hipStreamSynchronize(op->stream);
        const bool gen = !(op->sc <= 3 && op->mc <= 2);
        if (i > 0 && gen != b->general) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "all ops must share one stencil class pattern"); }
        b->general = gen;
        if (nrhs[i] < 1) { free_batch(b); TDP_BFAIL(TDP_EINVAL, "nrhs[%d] < 1", i); }
        b->ops.push_back(op);
    }
    b->f64 = ops[0]->prec == TDP_F64;
    b->s = ops[0]->stream;
    b->shape = b->f64 ? 4 : 8;    // FP32: the 128 x 64 tile
    b->K = 8;
    const size_t es = b->f64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < nops; ++i) {
        for (int r = 0; r < nrhs[i]; ++r) {
            tdp_batch::Field fl;
            fl.op = i;
            fl.N = ops[i]->N;
            const size_t fb = es * fl.N;
            bool ok = hipMalloc(&fl.a0, fb) == hipSuccess && hipMalloc(&fl.a1, fb) == hipSuccess &&
                      hipMalloc(&fl.b0, fb) == hipSuccess && hipMalloc(&fl.b1, fb) == hipSuccess &&
                      hipMalloc(&fl.pin, 16 * fl.N) == hipSuccess &&
                      hipMalloc(&fl.pout, 16 * fl.N) == hipSuccess;
            if (ok && !b->f64) ok = hipMalloc(&fl.Fst, 8 * fl.N) == hipSuccess;
            if (!ok) {
                b->f.push_back(fl);
                free_batch(b);
                TDP_BFAIL(TDP_ENOMEM, "batch field allocation failed");
            }
            b->f.push_back(fl);
        }
    }
    *out = b;
    return TDP_OK;
}

extern "C" int tdp_batch_set_tuning(tdp_batch *b, int depth, int tile, int medium_tile)
{
    if (!b) TDP_BFAIL(TDP_EINVAL, "NULL batch");
    if (depth < 1 || depth > 15) TDP_BFAIL(TDP_EINVAL, "depth must be in [1, 15]");
    if (tile < 0 || tile > 8 || ((tile == 2 || tile == 8) && b->f64)) TDP_BFAIL(TDP_EINVAL, "bad tile");
    const int rows = tb2d_tile_rows(tile, b->f64);
    if (4 * depth > rows) TDP_BFAIL(TDP_EINVAL, "depth too large for the tile");
    if (medium_tile < -1 || (medium_tile >= 0 && mrhs_nr(medium_tile, b->f64) == 0))
        TDP_BFAIL(TDP_EINVAL, "bad shared-medium tile");
    if (medium_tile >= 0 && 4 * depth > mrhs_rows(medium_tile, b->f64))
        TDP_BFAIL(TDP_EINVAL, "depth too large for the shared-medium tile");
    b->K = depth;
    b->shape = tile;
    b->mshape = medium_tile;
    return TDP_OK;
}

// descriptor array BFieldT<T>[] for the given per-op periods
template <typename T>
static int build_fields(tdp_batch *b, const int *T_op, double rho)
{
    std::vector<BFieldT<T>> h(b->f.size());
    for (size_t q = 0; q < b->f.size(); ++q) {
        const auto &fl = b->f[q];
        tdp_op *op = b->ops[fl.op];
        const double rho_op = rho <= 0.0 ? 1.0 / T_op[fl.op] : rho;   // rho <= 0: one period
        auto key = std::make_tuple(fl.op, T_op[fl.op], rho_op);
        if (!b->dtab.count(key)) {
            const std::vector<double> &tab = forcing_table(op, T_op[fl.op], rho_op, 0);
            double *d = nullptr;
            if (hipMalloc(&d, sizeof(double) * tab.size()) != hipSuccess)
                TDP_BFAIL(TDP_ENOMEM, "forcing table allocation failed");
            TDP_CHECK_HIP(hipMemcpyAsync(d, tab.data(), sizeof(double) * tab.size(),
                                         hipMemcpyHostToDevice, b->s));
            TDP_CHECK_HIP(hipStreamSynchronize(b->s));
            b->dtab[key] = d;
        }
        BFieldT<T> &x = h[q];
        x.ny = op->n[0];
        x.nx = op->n[1];
        x.Ns = T_op[fl.op] * op->nP;
        x.jsnap = x.Ns - snap_lag(op->nP);
        x.m = (const T *)(b->f64 ? (const void *)op->m : (const void *)op->m32);
        x.dn = (const T *)(b->f64 ? (const void *)op->dn : (const void *)op->dn32);
        x.F = b->f64 ? fl.pin : fl.Fst;
        x.Fin = fl.pin;
        x.a0 = (T *)fl.a0;
        x.a1 = (T *)fl.a1;
        x.b0 = (T *)fl.b0;
        x.b1 = (T *)fl.b1;
        x.tab = b->dtab[key];
        x.U = (double *)fl.pout;
        if constexpr (sizeof(T) == 8) x.st = op->st_step;
        else x.st = op->st_step32;
    }
    if (!b->dfields && hipMalloc(&b->dfields, sizeof(BFieldT<double>) * b->f.size()) != hipSuccess)
        TDP_BFAIL(TDP_ENOMEM, "descriptor allocation failed");
    TDP_CHECK_HIP(hipMemcpyAsync(b->dfields, h.data(), sizeof(BFieldT<T>) * h.size(),
                                 hipMemcpyHostToDevice, b->s));
    TDP_CHECK_HIP(hipStreamSynchronize(b->s));
    return TDP_OK;
}

static const size_t kMaxBatchGraphs = 32;

// periods per op: >= 1, and N_s = T n_P within TDP_MAX_STEPS
static int check_periods(const tdp_batch *b, const int *periods_T)
{
    for (size_t i = 0; i < b->ops.size(); ++i) {
        if (periods_T[i] < 1) TDP_BFAIL(TDP_EINVAL, "periods_T[%zu] < 1", i);
        if ((int64_t)periods_T[i] * b->ops[i]->nP > TDP_MAX_STEPS)
            TDP_BFAIL(TDP_EINVAL, "periods_T[%zu] n_P exceeds 2^24 steps", i);
    }
    return TDP_OK;
}

// One batched preconditioner application (Table 1) for the fields with
// active[q] != 0: reads each field's pin, writes its pout.
static int batch_precond(tdp_batch *b, const int *T_op, double rho, const std::vector<char> &active)
{
    hipStream_t s = b->s;
    std::vector<int> Tv(T_op, T_op + b->ops.size());
    if (Tv != b->tkey || rho != b->rho_key) {
        // cached applications may still be running on the stream: wait before
        // their graphs and schedules are released
        if (!b->graphs.empty()) TDP_CHECK_HIP(hipStreamSynchronize(s));
        for (auto &kv : b->graphs) {
            (void)hipGraphExecDestroy(kv.second.first);
            (void)hipFree(kv.second.second);
        }
        b->graphs.clear();
        int rc = b->f64 ? build_fields<double>(b, T_op, rho) : build_fields<float>(b, T_op, rho);
        if (rc != TDP_OK) return rc;
        b->tkey = Tv;
        b->rho_key = rho;
    }
    std::string key(active.begin(), active.end());
    key += "|" + std::to_string(b->K) + "|" + std::to_string(b->shape) + "|" +
           std::to_string(b->mshape);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        // schedule: launch L advances every active field with N_s > L*K
        std::vector<int> act;
        int maxNs = 0;
        for (size_t q = 0; q < b->f.size(); ++q)
            if (active[q]) {
                act.push_back((int)q);
                const tdp_op *op = b->ops[b->f[q].op];
                maxNs = std::max(maxNs, T_op[b->f[q].op] * op->nP);
            }
        const int nl = (maxNs + b->K - 1) / b->K;
        if (nl > TDP_MAX_GRAPH_LAUNCHES)     // the application is one captured graph
            TDP_BFAIL(TDP_EINVAL, "%d launches per batched application exceed 2^17 (lower periods_T)", nl);
        // per launch: the single fields (list + tile prefix) and the slabs of
        // right-hand sides sharing a medium (NR field indices each + prefix)
        struct Sched { int lo, po, n, tiles, so, sp, ns, stiles; };
        const int NR = b->mshape >= 0 ? mrhs_nr(b->mshape, b->f64) : 0;
        std::vector<int> host;
        std::vector<Sched> launches;
        for (int L = 0; L < nl; ++L) {
            std::map<int, std::vector<int>> byop;     // live fields of each medium
            for (int q : act) {
                const tdp_op *op = b->ops[b->f[q].op];
                if (T_op[b->f[q].op] * op->nP > L * b->K) byop[b->f[q].op].push_back(q);
            }
            std::vector<int> list, pre{0}, slabs, spre{0};
            for (const auto &kv : byop) {
                const tdp_op *op = b->ops[kv.first];
                const std::vector<int> &qs = kv.second;
                if (NR >= 2 && qs.size() >= 2) {
                    const int et = mrhs_rows(b->mshape, b->f64);
                    const int OX = 64 - 2 * b->K, OY = et - 2 * b->K;
                    const int tiles = ((op->n[1] + OX - 1) / OX) * ((op->n[0] + OY - 1) / OY);
                    for (size_t a = 0; a < qs.size(); a += NR) {
                        for (int r = 0; r < NR; ++r)
                            slabs.push_back(a + r < qs.size() ? qs[a + r] : -1);
                        spre.push_back(spre.back() + tiles);
                    }
                } else {
                    for (int q : qs) {
                        list.push_back(q);
                        pre.push_back(pre.back() + tb2d_tiles(b->shape, b->K, op->n[0], op->n[1]));
                    }
                }
            }
            Sched sc;
            sc.lo = (int)host.size();
            host.insert(host.end(), list.begin(), list.end());
            sc.po = (int)host.size();
            host.insert(host.end(), pre.begin(), pre.end());
            sc.n = (int)list.size();
            sc.tiles = pre.back();
            sc.so = (int)host.size();
            host.insert(host.end(), slabs.begin(), slabs.end());
            sc.sp = (int)host.size();
            host.insert(host.end(), spre.begin(), spre.end());
            sc.ns = (int)spre.size() - 1;
            sc.stiles = spre.back();
            launches.push_back(sc);
        }
        // the active fields, for the stage-in launch
        const int ao = (int)host.size();
        host.insert(host.end(), act.begin(), act.end());
        int64_t n_max = 0;
        for (int q : act) n_max = std::max(n_max, b->f[q].N);
        int *dsched = nullptr;
        if (hipMalloc(&dsched, sizeof(int) * std::max<size_t>(1, host.size())) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "schedule allocation failed");
        TDP_CHECK_HIP(hipMemcpyAsync(dsched, host.data(), sizeof(int) * host.size(),
                                     hipMemcpyHostToDevice, s));
        TDP_CHECK_HIP(hipStreamSynchronize(s));
        hipGraph_t g;
        TDP_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_batch_stage_in(b->dfields, dsched + ao, (int)act.size(), n_max,
                                              b->f64, s);
        for (int L = 0; L < nl && le == hipSuccess; ++L) {
            const Sched &sc = launches[L];
            if (sc.n > 0) {
                TBBatchLaunch bl;
                bl.fields = b->dfields;
                bl.list = dsched + sc.lo;
                bl.prefix = dsched + sc.po;
                bl.nlist = sc.n;
                bl.ntiles = sc.tiles;
                bl.j0 = L * b->K;
                bl.K = b->K;
                bl.parity = L & 1;
                bl.shape = b->shape;
                bl.general = b->general;
                le = launch_sweep2d_tb_batch(bl, b->f64, s);
            }
            if (sc.ns > 0 && le == hipSuccess) {
                TBMrhsLaunch ml;
                ml.fields = b->dfields;
                ml.slabs = dsched + sc.so;
                ml.prefix = dsched + sc.sp;
                ml.nslab = sc.ns;
                ml.ntiles = sc.stiles;
                ml.j0 = L * b->K;
                ml.K = b->K;
                ml.parity = L & 1;
                ml.shape = b->mshape;
                ml.general = b->general;
                le = launch_sweep2d_tb_mrhs(ml, b->f64, s);
            }
        }
        // Table 1 with 4 not dividing n_P: Im U from the two samples (2x2 solve)
        for (int q : act) {
            const tdp_op *op = b->ops[b->f[q].op];
            if (le != hipSuccess || op->nP % 4 == 0) continue;
            const double phi = 2.0 * M_PI * (double)snap_lag(op->nP) / op->nP;
            le = launch_phase_extract(b->f[q].pout, b->f[q].N, std::cos(phi), std::sin(phi), s);
        }
        hipError_t ce = hipStreamEndCapture(s, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (ce == hipSuccess) (void)hipGraphDestroy(g);
            (void)hipFree(dsched);
            TDP_CHECK_HIP(le);
            TDP_CHECK_HIP(ce);
        }
        hipGraphExec_t ge;
        hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) (void)hipFree(dsched);
        TDP_CHECK_HIP(ie);
        // one graph per active set: as fields converge the sets change, so the
        // cache is emptied when it would grow beyond kMaxBatchGraphs
        if (b->graphs.size() >= kMaxBatchGraphs) {
            const hipError_t se = hipStreamSynchronize(s);
            for (auto &kv : b->graphs) {
                (void)hipGraphExecDestroy(kv.second.first);
                (void)hipFree(kv.second.second);
            }
            b->graphs.clear();
            if (se != hipSuccess) {
                (void)hipGraphExecDestroy(ge);
                (void)hipFree(dsched);
                TDP_CHECK_HIP(se);
            }
        }
        it = b->graphs.emplace(key, std::make_pair(ge, dsched)).first;
    }
    TDP_CHECK_HIP(hipGraphLaunch(it->second.first, s));
    return TDP_OK;
}

extern "C" int tdp_batch_precond(tdp_batch *b, const int *periods_T, double rho,
                                 const void *const *F, void *const *U)
{
    if (!b || !periods_T || !F || !U) TDP_BFAIL(TDP_EINVAL, "NULL argument");
    if (rho > 1.0) TDP_BFAIL(TDP_EINVAL, "rho must be <= 1");
    TDP_CHECK(check_periods(b, periods_T));
    StreamJoin join(b->ops[0]->user_stream, b->s, b->ops[0]->ev);
    std::vector<char> active(b->f.size(), 1);
    for (size_t q = 0; q < b->f.size(); ++q) {
        if (!F[q] || !U[q] || F[q] == U[q] || misaligned16(F[q]) || misaligned16(U[q]))
            TDP_BFAIL(TDP_EINVAL, "bad F/U pointer for field %zu (NULL, aliased or not 16-byte aligned)", q);
        TDP_CHECK_HIP(hipMemcpyAsync(b->f[q].pin, F[q], 16 * b->f[q].N, hipMemcpyDeviceToDevice, b->s));
    }
    TDP_CHECK(batch_precond(b, periods_T, rho, active));
    for (size_t q = 0; q < b->f.size(); ++q)
        TDP_CHECK_HIP(hipMemcpyAsync(U[q], b->f[q].pout, 16 * b->f[q].N, hipMemcpyDeviceToDevice, b->s));
    return TDP_OK;
}

// Autotuner of the batched sweep: times one batched application (periods_T
// per op) for every depth x per-field tile shape with every field on its own
// tile, then for every shared-medium tile with that depth's best per-field
// tile; keeps the fastest.
extern "C" int tdp_batch_autotune(tdp_batch *b, const int *periods_T, double rho, double *table,
                                  int cap)
{
    if (!b || !periods_T) TDP_BFAIL(TDP_EINVAL, "NULL argument");
    if (rho > 1.0) TDP_BFAIL(TDP_EINVAL, "rho must be <= 1");
    TDP_CHECK(check_periods(b, periods_T));
    StreamJoin join(b->ops[0]->user_stream, b->s, b->ops[0]->ev);
    std::vector<char> active(b->f.size(), 1);
    for (auto &fl : b->f) TDP_CHECK_HIP(launch_fill_zero(fl.pin, 16 * fl.N, b->s));
    const int K0 = b->K, S0 = b->shape, M0 = b->mshape;
    double best = INFINITY;
    int bk = K0, bs = S0, bm = M0, n = 0;
    hipEvent_t e0, e1;
    TDP_CHECK_HIP(hipEventCreate(&e0));
    TDP_CHECK_HIP(hipEventCreate(&e1));
    int rc = TDP_OK;
    // one candidate: capture + warm, then two timed applications
    auto trial = [&](int K, int shape, int mshape, double *out_ms) -> int {
        b->K = K;
        b->shape = shape;
        b->mshape = mshape;
        int r = batch_precond(b, periods_T, rho, active);
        if (r != TDP_OK) return r;
        float ms = 0.f;
        if (hipEventRecord(e0, b->s) != hipSuccess) return TDP_EHIP;
        for (int i = 0; i < 2 && r == TDP_OK; ++i) r = batch_precond(b, periods_T, rho, active);
        if (r != TDP_OK) return r;
        if (hipEventRecord(e1, b->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return TDP_EHIP;
        *out_ms = ms / 2;
        if (table && n < cap) {
            table[4 * n] = K;
            table[4 * n + 1] = shape;
            table[4 * n + 2] = mshape;
            table[4 * n + 3] = ms / 2;
        }
        ++n;
        if (*out_ms < best) {
            best = *out_ms;
            bk = K;
            bs = shape;
            bm = mshape;
        }
        return TDP_OK;
    };
    // stage 1: every depth x single-field tile with each field on its own
    // tile; stage 2: every shared-medium tile with that depth's best
    // single-field tile (which then runs the fields that have no partner)
    for (int K : {4, 6, 8}) {
        double kbest = INFINITY;
        int kshape = -1;
        for (int shape = 0; shape < 9 && rc == TDP_OK; ++shape) {
            if ((shape == 2 || shape == 8) && b->f64) continue;
            if (4 * K > tb2d_tile_rows(shape, b->f64)) continue;
            double ms = INFINITY;
            rc = trial(K, shape, -1, &ms);
            if (rc == TDP_OK && ms < kbest) {
                kbest = ms;
                kshape = shape;
            }
        }
        for (int mt = 0; mt < 3 && rc == TDP_OK && kshape >= 0; ++mt) {
            if (4 * K > mrhs_rows(mt, b->f64)) continue;
            double ms = INFINITY;
            rc = trial(K, kshape, mt, &ms);
        }
        if (rc != TDP_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const hipError_t se = hipStreamSynchronize(b->s);   // no timed graph may still run
    if (se != hipSuccess && rc == TDP_OK) {
        ::tdp::set_error("HIP error: %s", hipGetErrorString(se));
        rc = TDP_EHIP;
    }
    for (auto &kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.first);
        (void)hipFree(kv.second.second);
    }
    b->graphs.clear();
    if (rc != TDP_OK) {
        b->K = K0;
        b->shape = S0;
        b->mshape = M0;
        return rc;
    }
    b->K = bk;
    b->shape = bs;
    b->mshape = bm;
    return n;
}

// ---------------------------------------------------------------------------
// Lockstep GMRES.  Per field, the same iteration as the single solve
// (tdp_gmres_solve): r = F - H x; z = P r; Arnoldi with CGS2; complex Givens;
// in tolerance mode the true residual of the current iterate after every
// iteration, stop at <= tol, restart early on a stall.
namespace {
enum Phase { NEED_RES, AWAIT_P0, NEED_HV, AWAIT_P, DONE };
struct FS {
    Phase ph = NEED_RES;
    int its = 0, restarts = 0, nhist = 0, status = TDP_ENOTCONV, i = 0, k_used = 0;
    int64_t napply = 0;
    double bnorm = 0, pnorm0 = -1, est = 1, rel = 1, rel_start = 1, rel_prev = 1, beta0 = 0;
    double best_rel = 1;
    int best_k = 0;             // the cycle's candidate with the smallest true residual
    std::vector<cplx> Hm, gv, sn, y, ybest;
    std::vector<double> cs;
};
}  // namespace

static int ensure_field_krylov(tdp_batch *b, int m)
{
    for (auto &fl : b->f) {
        if (fl.V && fl.Vcols >= m + 1) continue;
        (void)hipStreamSynchronize(b->s);
        (void)hipFree(fl.V);
        fl.V = nullptr;
        if (hipMalloc(&fl.V, (size_t)16 * fl.N * (m + 1)) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "batch Krylov basis allocation failed");
        fl.Vcols = m + 1;
        if (!fl.rv && (hipMalloc(&fl.rv, 16 * fl.N) != hipSuccess || hipMalloc(&fl.xv, 16 * fl.N) != hipSuccess))
            TDP_BFAIL(TDP_ENOMEM, "batch work vector allocation failed");
        (void)hipFree(fl.red);
        (void)hipFree(fl.dco);
        fl.red = fl.dco = nullptr;
        const int nblk = blas_nblocks(fl.N);
        if (hipMalloc(&fl.red, sizeof(double) * 2 * (size_t)nblk * (m + 2)) != hipSuccess ||
            hipMalloc(&fl.dco, sizeof(double) * 8 * (size_t)(m + 2)) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "batch reduction allocation failed");
    }
    const size_t need = b->f.size() * 8 * (size_t)(m + 2);
    if (need > b->hbuf_n) {
        if (b->hbuf) (void)hipHostFree(b->hbuf);
        b->hbuf = nullptr;
        if (hipHostMalloc(&b->hbuf, sizeof(double) * need) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "pinned host allocation failed");
        b->hbuf_n = need;
    }
    if (need > b->gstage_n) {
        (void)hipStreamSynchronize(b->s);
        (void)hipFree(b->gstage);
        b->gstage = nullptr;
        if (hipMalloc(&b->gstage, sizeof(double) * need) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "batch staging allocation failed");
        b->gstage_n = need;
    }
    if (b->f.size() > b->gs_n) {
        (void)hipStreamSynchronize(b->s);
        if (b->gs_host) (void)hipHostFree(b->gs_host);
        (void)hipFree(b->gs_dev);
        b->gs_host = nullptr;
        b->gs_dev = nullptr;
        if (hipHostMalloc(&b->gs_host, sizeof(GsField) * b->f.size()) != hipSuccess ||
            hipMalloc(&b->gs_dev, sizeof(GsField) * b->f.size()) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "batch descriptor allocation failed");
        b->gs_n = b->f.size();
    }
    if (b->f.size() > b->tr_n) {
        (void)hipStreamSynchronize(b->s);
        if (b->tr_host) (void)hipHostFree(b->tr_host);
        if (b->tr_outh) (void)hipHostFree(b->tr_outh);
        (void)hipFree(b->tr_dev);
        (void)hipFree(b->tr_out);
        b->tr_host = nullptr;
        b->tr_outh = nullptr;
        b->tr_dev = nullptr;
        b->tr_out = nullptr;
        const size_t n = b->f.size();
        if (hipHostMalloc(&b->tr_host, sizeof(TrField) * n) != hipSuccess ||
            hipHostMalloc(&b->tr_outh, sizeof(double) * 2 * n) != hipSuccess ||
            hipMalloc(&b->tr_dev, sizeof(TrField) * n) != hipSuccess ||
            hipMalloc(&b->tr_out, sizeof(double) * 2 * n) != hipSuccess)
            TDP_BFAIL(TDP_ENOMEM, "batch descriptor allocation failed");
        b->tr_n = n;
    }
    return TDP_OK;
}

extern "C" int tdp_batch_solve(tdp_batch *b, const tdp_gmres_cfg *cfg, const int *periods_T,
                               const void *const *F, void *const *U, tdp_gmres_info *infos)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!b || !cfg || !periods_T || !F || !U) TDP_BFAIL(TDP_EINVAL, "NULL argument");
    const int m = cfg->restart;
    if (m < 1 || m > 512) TDP_BFAIL(TDP_EINVAL, "restart must be in [1, 512]");
    if (cfg->max_iters < 1 || !(cfg->tol > 0.0) || cfg->rho > 1.0)
        TDP_BFAIL(TDP_EINVAL, "bad GMRES configuration");
    if (cfg->variant != 0) TDP_BFAIL(TDP_EINVAL, "the batched form uses the Table 1 preconditioner");
    TDP_CHECK(check_periods(b, periods_T));
    const size_t nf = b->f.size();
    for (size_t q = 0; q < nf; ++q)
        if (!F[q] || !U[q] || F[q] == U[q] || misaligned16(F[q]) || misaligned16(U[q]))
            TDP_BFAIL(TDP_EINVAL, "bad F/U pointer for field %zu (NULL, aliased or not 16-byte aligned)", q);
    TDP_CHECK(ensure_field_krylov(b, m));
    StreamJoin join(b->ops[0]->user_stream, b->s, b->ops[0]->ev);
    hipStream_t s = b->s;
    const bool tolmode = cfg->fixed_iters <= 0;
    const int limit = tolmode ? cfg->max_iters : cfg->fixed_iters;
    std::vector<FS> st(nf);
    double *hb = b->hbuf;
    const size_t hs = 8 * (size_t)(m + 2);   // host slots per field
    auto col = [&](size_t q, int k) -> void * { return (char *)b->f[q].V + (size_t)16 * b->f[q].N * k; };
    auto norm2_async = [&](size_t q, const void *x, double *dst_dev) -> int {
        const auto &fl = b->f[q];
        TDP_CHECK_HIP(launch_mdot(x, fl.N, 1, x, fl.N, fl.red, blas_nblocks(fl.N), dst_dev, s));
        return TDP_OK;
    };
    // bnorm of every field
    for (size_t q = 0; q < nf; ++q) {
        auto &S = st[q];
        S.Hm.assign((size_t)(m + 1) * m, 0.0);
        S.gv.assign(m + 1, 0.0);
        S.sn.assign(m, 0.0);
        S.y.assign(m, 0.0);
        S.ybest.assign(m, 0.0);
        S.cs.assign(m, 0.0);
        TDP_CHECK(norm2_async(q, F[q], b->f[q].dco));
        TDP_CHECK_HIP(hipMemcpyAsync(hb + q * hs, b->f[q].dco, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    TDP_CHECK_HIP(hipStreamSynchronize(s));
    for (size_t q = 0; q < nf; ++q)     // refused before any output is written
        if (!std::isfinite(std::sqrt(hb[q * hs]))) TDP_BFAIL(TDP_EINVAL, "F[%zu] holds NaN or Inf", q);
    for (size_t q = 0; q < nf; ++q) {
        if (!cfg->x0_given) TDP_CHECK_HIP(launch_fill_zero(U[q], 16 * b->f[q].N, s));
        st[q].bnorm = std::sqrt(hb[q * hs]);
        if (st[q].bnorm == 0.0) {
            TDP_CHECK_HIP(launch_fill_zero(U[q], 16 * b->f[q].N, s));
            st[q].ph = DONE;
            st[q].status = TDP_OK;
            st[q].rel = st[q].est = 0.0;
        }
    }
    auto HMq = [&](FS &S, int i, int j) -> cplx & { return S.Hm[(size_t)j * (m + 1) + i]; };
    auto solve_y = [&](FS &S) {
        for (int k = S.k_used - 1; k >= 0; --k) {
            cplx sum = S.gv[k];
            for (int j = k + 1; j < S.k_used; ++j) sum -= HMq(S, k, j) * S.y[j];
            S.y[k] = sum / HMq(S, k, k);
        }
    };
    // x_out = x_in + V y  for field q (y staged through the host buffer)
    auto update = [&](size_t q, void *x_out, const void *x_in) -> int {
        FS &S = st[q];
        auto &fl = b->f[q];
        double *hy = hb + q * hs + 4 * (m + 1) + 2;
        for (int k = 0; k < S.k_used; ++k) {
            hy[2 * k] = S.y[k].real();
            hy[2 * k + 1] = S.y[k].imag();
        }
        double *dy = fl.dco + 4 * (m + 1) + 2;
        TDP_CHECK_HIP(hipMemcpyAsync(dy, hy, sizeof(double) * 2 * S.k_used, hipMemcpyHostToDevice, s));
        if (x_out != x_in)
            TDP_CHECK_HIP(hipMemcpyAsync(x_out, x_in, 16 * fl.N, hipMemcpyDeviceToDevice, s));
        TDP_CHECK_HIP(launch_maxpy(x_out, fl.V, fl.N, S.k_used, dy, 1.0, fl.N, s));
        return TDP_OK;
    };
    // batched per-field steps: descriptors collected by tr_add, issued as one
    // launch sequence by tr_launch (r = F - H xh or H xh, optionally after
    // x_out = x_in + V y and followed by |r|^2 into b->tr_out at 2q)
    int ntr = 0, tr_nblk = 0, tr_ny = 0, tr_nx = 0;
    int64_t tr_nmax = 0;
    auto tr_add = [&](size_t q, const void *xh, const void *Fq, void *r, bool norm, int k,
                      void *x_out, const void *x_in, const double *ydev) {
        const auto &fl = b->f[q];
        const tdp_op *op = b->ops[fl.op];
        TrField &g = b->tr_host[ntr++];
        g.V = (const double2 *)fl.V;
        g.x_in = (const double2 *)x_in;
        g.x_out = (double2 *)x_out;
        g.y = ydev;
        g.xh = (const double2 *)xh;
        g.F = (const double2 *)Fq;
        g.r = (double2 *)r;
        g.m = op->m;
        g.rw = op->rw;
        g.red = fl.red;
        g.out = norm ? b->tr_out + 2 * q : nullptr;
        g.st = op->st_H;
        g.N = fl.N;
        g.k = k;
        g.nblk = blas_nblocks(fl.N);
        g.ny = op->n[0];
        g.nx = op->n[1];
        tr_nblk = std::max(tr_nblk, g.nblk);
        tr_ny = std::max(tr_ny, g.ny);
        tr_nx = std::max(tr_nx, g.nx);
        tr_nmax = std::max(tr_nmax, g.N);
    };
    auto tr_launch = [&](bool upd, bool norm) -> int {
        if (ntr == 0) return TDP_OK;
        TDP_CHECK_HIP(hipMemcpyAsync(b->tr_dev, b->tr_host, sizeof(TrField) * ntr,
                                     hipMemcpyHostToDevice, s));
        TDP_CHECK_HIP(launch_tr_multi(b->tr_dev, ntr, upd, norm, b->general, tr_nblk, tr_nmax,
                                      tr_ny, tr_nx, s));
        if (norm)
            TDP_CHECK_HIP(hipMemcpyAsync(b->tr_outh, b->tr_out, sizeof(double) * 2 * nf,
                                         hipMemcpyDeviceToHost, s));
        ntr = tr_nblk = tr_ny = tr_nx = 0;
        tr_nmax = 0;
        return TDP_OK;
    };
    auto end_cycle = [&](size_t q) -> int {
        FS &S = st[q];
        ++S.restarts;
        S.ph = NEED_RES;
        if (tolmode) {
            // keep the cycle's best iterate; a cycle that did not lower the true
            // residual ends the field (only the real-linear Table 1 map is batched)
            if (S.best_k > 0 && S.best_k == S.k_used) {
                TDP_CHECK_HIP(hipMemcpyAsync(U[q], b->f[q].xv, 16 * b->f[q].N, hipMemcpyDeviceToDevice, s));
            } else if (S.best_k > 0) {
                std::copy(S.ybest.begin(), S.ybest.begin() + S.best_k, S.y.begin());
                S.k_used = S.best_k;
                TDP_CHECK(update(q, U[q], U[q]));
            }
            S.rel = S.best_rel;
            if (S.best_k == 0 && S.k_used > 0) S.ph = DONE;
        } else if (S.k_used > 0) {
            solve_y(S);
            TDP_CHECK(update(q, U[q], U[q]));
        }
        return TDP_OK;
    };
    std::vector<char> needP(nf);
    std::vector<int> Tv(periods_T, periods_T + b->ops.size());
    for (;;) {
        // stage A: residuals of fields starting a cycle (one sync for all)
        bool anyA = false;
        for (size_t q = 0; q < nf; ++q)
            if (st[q].ph == NEED_RES) {
                tr_add(q, U[q], F[q], b->f[q].rv, true, 0, nullptr, nullptr, nullptr);
                anyA = true;
            }
        if (anyA) {
            TDP_CHECK(tr_launch(false, true));
            TDP_CHECK_HIP(hipStreamSynchronize(s));
        }
        bool any = false;
        for (size_t q = 0; q < nf; ++q) {
            FS &S = st[q];
            needP[q] = 0;
            if (S.ph == NEED_RES) {
                S.rel = std::sqrt(b->tr_outh[2 * q]) / S.bnorm;
                if (!std::isfinite(S.rel) && S.its == 0 && S.restarts == 0)
                    TDP_BFAIL(TDP_EINVAL, "non-finite residual of field %zu: U holds NaN or Inf", q);
                if (tolmode && S.rel <= cfg->tol) {
                    S.status = TDP_OK;
                    S.ph = DONE;
                    continue;
                }
                if (S.its >= limit) {
                    S.ph = DONE;
                    continue;
                }
                TDP_CHECK_HIP(hipMemcpyAsync(b->f[q].pin, b->f[q].rv, 16 * b->f[q].N,
                                             hipMemcpyDeviceToDevice, s));
                S.ph = AWAIT_P0;
                needP[q] = 1;
            } else if (S.ph == NEED_HV) {
                tr_add(q, col(q, S.i), nullptr, b->f[q].pin, false, 0, nullptr, nullptr, nullptr);
                S.ph = AWAIT_P;
                needP[q] = 1;
            }
            any = any || needP[q];
        }
        TDP_CHECK(tr_launch(false, false));
        if (!any) break;
        // stage B: one batched preconditioner application
        TDP_CHECK(batch_precond(b, Tv.data(), cfg->rho, needP));
        // stage C: orthogonalisation / normalisation (one sync for all).  A
        // field starting a cycle normalises its first vector on its own; the
        // CGS2 steps of all other fields run as one batched launch sequence.
        // Every field's coefficients land in the staging array at its host
        // slot, which one copy brings to the host.
        int ngs = 0, nv_max = 0, nblk_max = 0;
        int64_t n_max = 0;
        for (size_t q = 0; q < nf; ++q) {
            if (!needP[q]) continue;
            FS &S = st[q];
            auto &fl = b->f[q];
            ++S.napply;
            if (S.ph == AWAIT_P0) {
                TDP_CHECK(norm2_async(q, fl.pout, fl.dco));
                TDP_CHECK_HIP(launch_scale_by_invnorm(col(q, 0), fl.pout, fl.dco, fl.N, s));
                TDP_CHECK_HIP(hipMemcpyAsync(b->gstage + q * hs, fl.dco, sizeof(double),
                                             hipMemcpyDeviceToDevice, s));
            } else {
                GsField &g = b->gs_host[ngs++];
                g.V = (const double2 *)fl.V;
                g.w = (double2 *)fl.pout;
                g.vnext = (double2 *)col(q, S.i + 1);
                g.red = fl.red;
                g.co = fl.dco;
                g.gather = b->gstage + q * hs;
                g.N = fl.N;
                g.nv = S.i + 1;
                g.nblk = blas_nblocks(fl.N);
                g.off2 = 2 * (m + 1);
                g.offn = 4 * (m + 1);
                g.ncopy = 4 * (m + 1) + 2;
                nv_max = std::max(nv_max, g.nv);
                nblk_max = std::max(nblk_max, g.nblk);
                n_max = std::max(n_max, fl.N);
            }
        }
        if (ngs > 0) {
            TDP_CHECK_HIP(hipMemcpyAsync(b->gs_dev, b->gs_host, sizeof(GsField) * ngs,
                                         hipMemcpyHostToDevice, s));
            TDP_CHECK_HIP(launch_gs_step_multi(b->gs_dev, ngs, nv_max, nblk_max, n_max, s));
        }
        TDP_CHECK_HIP(hipMemcpyAsync(hb, b->gstage, sizeof(double) * hs * nf, hipMemcpyDeviceToHost, s));
        TDP_CHECK_HIP(hipStreamSynchronize(s));
        // host: Givens, and (tolerance mode) the current iterates' residuals
        bool anyD = false;
        for (size_t q = 0; q < nf; ++q) {
            if (!needP[q]) continue;
            FS &S = st[q];
            if (S.ph == AWAIT_P0) {
                const double z2 = hb[q * hs];
                S.beta0 = std::sqrt(z2);
                if (S.pnorm0 < 0.0) S.pnorm0 = S.beta0;
                if (S.beta0 == 0.0) {
                    S.ph = DONE;
                    continue;
                }
                for (int k = 0; k <= m; ++k) S.gv[k] = 0.0;
                S.gv[0] = S.beta0;
                S.rel_start = S.rel_prev = S.best_rel = S.rel;
                S.best_k = 0;
                S.i = 0;
                S.k_used = 0;
                S.ph = NEED_HV;
                continue;
            }
            ++S.its;
            const int i = S.i;
            const double *h1 = hb + q * hs, *h2 = h1 + 2 * (m + 1);
            for (int k = 0; k <= i; ++k)
                HMq(S, k, i) = cplx(h1[2 * k] + h2[2 * k], h1[2 * k + 1] + h2[2 * k + 1]);
            const double hn = std::sqrt(h1[4 * (m + 1)]);
            HMq(S, i + 1, i) = hn;
            for (int k = 0; k < i; ++k) {
                const cplx a = HMq(S, k, i), c = HMq(S, k + 1, i);
                HMq(S, k, i) = S.cs[k] * a + S.sn[k] * c;
                HMq(S, k + 1, i) = -std::conj(S.sn[k]) * a + S.cs[k] * c;
            }
            const cplx a = HMq(S, i, i);
            const double rr = std::hypot(std::abs(a), hn);
            if (std::abs(a) == 0.0) {
                S.cs[i] = 0.0;
                S.sn[i] = 1.0;
                HMq(S, i, i) = hn;
            } else {
                const cplx ph = a / std::abs(a);
                S.cs[i] = std::abs(a) / rr;
                S.sn[i] = ph * hn / rr;
                HMq(S, i, i) = ph * rr;
            }
            HMq(S, i + 1, i) = 0.0;
            S.gv[i + 1] = -std::conj(S.sn[i]) * S.gv[i];
            S.gv[i] = S.cs[i] * S.gv[i];
            S.est = std::abs(S.gv[i + 1]) / S.pnorm0;
            tdp_gmres_info *inf = infos ? &infos[q] : nullptr;
            if (inf && inf->history && S.nhist < inf->history_cap) inf->history[S.nhist] = S.est;
            ++S.nhist;
            S.k_used = i + 1;
            S.i = i + 1;
            // hn stashed for stage D decisions
            h1 = nullptr;
            hb[q * hs + 4 * (m + 1) + 1] = hn;
            if (tolmode) {
                // x = U + V y and its true residual, batched below (y goes
                // through the host slot to the staging array)
                solve_y(S);
                double *hy = hb + q * hs + 4 * (m + 1) + 2;
                for (int k = 0; k < S.k_used; ++k) {
                    hy[2 * k] = S.y[k].real();
                    hy[2 * k + 1] = S.y[k].imag();
                }
                tr_add(q, b->f[q].xv, F[q], b->f[q].rv, true, S.k_used, b->f[q].xv, U[q],
                       b->gstage + q * hs + 4 * (m + 1) + 2);
                anyD = true;
            }
        }
        if (anyD) {
            TDP_CHECK_HIP(hipMemcpyAsync(b->gstage, hb, sizeof(double) * hs * nf,
                                         hipMemcpyHostToDevice, s));
            TDP_CHECK(tr_launch(true, true));
            TDP_CHECK_HIP(hipStreamSynchronize(s));
        }
        // stage D: decisions
        for (size_t q = 0; q < nf; ++q) {
            if (!needP[q] || st[q].ph != AWAIT_P) continue;
            FS &S = st[q];
            const double hn = hb[q * hs + 4 * (m + 1) + 1];
            const double est_cycle = std::abs(S.gv[S.k_used]) / S.beta0;
            bool end = false;
            if (tolmode) {
                const double relt = std::sqrt(b->tr_outh[2 * q]) / S.bnorm;
                S.rel = relt;
                if (relt < S.best_rel) {
                    S.best_rel = relt;
                    S.best_k = S.k_used;
                    std::copy(S.y.begin(), S.y.begin() + S.k_used, S.ybest.begin());
                }
                if (relt <= cfg->tol) {
                    TDP_CHECK_HIP(hipMemcpyAsync(U[q], b->f[q].xv, 16 * b->f[q].N, hipMemcpyDeviceToDevice, s));
                    ++S.restarts;
                    S.status = TDP_OK;
                    S.ph = DONE;
                    continue;
                }
                if (hn == 0.0 || !(relt <= 1e6 * S.rel_start) ||
                    (relt > 2.0 * S.rel_start * est_cycle && relt > 0.7 * S.rel_prev))
                    end = true;
                else
                    S.rel_prev = relt;
            } else if (hn == 0.0) {
                end = true;
            }
            if (!end && (S.i >= m || S.its >= limit)) end = true;
            if (!end) {
                S.ph = NEED_HV;
                continue;
            }
            TDP_CHECK(end_cycle(q));
            if (!tolmode && S.its >= limit) {
                tdp_op *op = b->ops[b->f[q].op];
                TDP_CHECK(apply_H_on(op, U[q], F[q], b->f[q].rv, s));
                TDP_CHECK(norm2_async(q, b->f[q].rv, b->f[q].dco));
                TDP_CHECK_HIP(hipMemcpyAsync(hb + q * hs, b->f[q].dco, sizeof(double), hipMemcpyDeviceToHost, s));
                TDP_CHECK_HIP(hipStreamSynchronize(s));
                S.rel = std::sqrt(hb[q * hs]) / S.bnorm;
                S.status = TDP_OK;
                S.ph = DONE;
            }
        }
    }
    TDP_CHECK_HIP(hipStreamSynchronize(s));
    int worst = TDP_OK;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t q = 0; q < nf; ++q) {
        const FS &S = st[q];
        if (S.status != TDP_OK) worst = TDP_ENOTCONV;
        if (infos) {
            tdp_gmres_info &inf = infos[q];
            inf.iters = S.its;
            inf.restarts = S.restarts;
            inf.relres_true = S.rel;
            inf.relres_prec = S.est;
            inf.switched = 0;
            inf.steps = S.napply * (int64_t)periods_T[b->f[q].op] * b->ops[b->f[q].op]->nP;
            inf.history_len = S.nhist < inf.history_cap ? S.nhist : inf.history_cap;
            inf.ms_total = ms;
            inf.ms_precond = inf.ms_H = inf.ms_arnoldi = 0.0;   // not timed per field here
        }
    }
    return worst;
}
