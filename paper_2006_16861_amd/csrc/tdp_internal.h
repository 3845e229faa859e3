// Internal declarations shared by the host library and the HIP kernels of
// libtdp.  Nothing here is part of the public ABI (include/tdp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tdp.h"

namespace tdp {

void set_error(const char *fmt, ...);
void clear_error();

#define TDP_CHECK_HIP(call)                                                              \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::tdp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                             __FILE__, __LINE__);                                        \
            return TDP_EHIP;                                                             \
        }                                                                                \
    } while (0)

#define TDP_CHECK(rc_expr)                 \
    do {                                   \
        int rc_ = (rc_expr);               \
        if (rc_ < 0) return rc_;           \
    } while (0)

// Constants of one application of the assembled stencil to a real field u,
// with the cell slowness m_cell:
//   result_i = c0 u_i + sum_{k>=1} s[k] sum_{|o|=k} u_{i+o}
//                    + sum_{k>=0} m[k] sum_{|o|=k} W_o u_{i+o},
// where o runs over the 3^d offsets, |o| = number of nonzero components
// (the Delta class of App. A) and W_o = sum of m_cell over the cells that
// contain both node i and node i+o.
template <typename T>
struct Stencil {
    T c0;
    T s[4];
    T m[4];
};

// Per-node streams (u_{j-1}, damping factor, F, the new field) are read or
// written once per step.  When a step's working set exceeds the 256 MB MALL
// they go non-temporal, so that L2 keeps the rows and planes that neighbouring
// workgroups re-read; when it fits, the normal policy keeps them cached for the
// next step.
// The choice is a template parameter of the kernels (a run-time select between
// the two load forms would be merged into one plain load).
inline bool stream_nt(int64_t bytes) { return bytes > ((int64_t)192 << 20); }
// complex128 arrays are read and written as 16-byte vectors
inline bool misaligned16(const void *p) { return ((uintptr_t)p & 15) != 0; }
template <bool NT, typename T>
__device__ __forceinline__ T ldnt(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stnt(T v, T *p)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Recurrence fields of one preconditioner application: the pairs (u0, u1)
// and, for the kernels that ping-pong (blocked 2-D, two-step 3-D), (v0, v1).
// table_free: evaluate the forcing scalars step by step instead of reading
// the op's cached table (the allocation-free entry point).
struct LoopBufs {
    void *u0, *u1, *v0, *v1;
    bool table_free;
};

// Launch geometry / variant choice for the sweep.
struct SweepCfg {
    int kernel = 1;       // 1 one step per launch, 2 temporally blocked
    int tb_depth = 0;     // steps per launch for kernel 2
};

// Device kernels (kernels.hip).  Every launcher enqueues on `s` and returns
// hipSuccess or the launch error.
struct SweepArgs {
    int ndim;
    int n[3];             // interior nodes per axis (n[2] = 1 in 2-D)
    int sc, mc;           // number of leading nonzero stiffness / mass classes
    const void *u;        // u_j
    void *up;             // in: u_{j-1}, out: u_{j+1}
    const void *m;        // cell slowness [(n0+1)(n1+1)(n2+1)]
    const void *dn;       // node factor 1/(1 + l/2)
    const void *F;        // complex right-hand side (double2 or float2)
    double *out;          // if non-null, u_{j+1} written here with stride 2
};

hipError_t launch_sweep_f64(const SweepArgs &a, const Stencil<double> &st, double fa, double fb,
                            hipStream_t s);
hipError_t launch_sweep_f32(const SweepArgs &a, const Stencil<float> &st, float fa, float fb,
                            hipStream_t s);

// Temporally blocked 2-D sweep (sweep_tb.hip): one launch = k steps.
#define TDP_TB_KMAX 16
#define TDP_MAX_STEPS ((int64_t)1 << 24)   // recurrence steps per application
#define TDP_MAX_GRAPH_LAUNCHES (1 << 17)     // kernel launches captured in one graph
struct TBCoef {
    int k;                   // steps in this launch (1..TDP_TB_KMAX, < tile half-size)
    int out_step[2];         // 1-based step whose result goes to out[i] (0: none)
    double *out[2];          // stride-2 outputs (complex128 real or imaginary part)
    double fa[TDP_TB_KMAX];  // forcing scalars of the k steps
    double fb[TDP_TB_KMAX];
};
struct TBArgs {
    int ny, nx;              // interior nodes (axis 0, axis 1)
    int sc, mc;
    int shape;               // tile shape index (see sweep_tb.hip)
    const void *u_in, *up_in;    // u_j, u_{j-1}
    void *u_out, *up_out;        // u_{j+k}, u_{j+k-1}  (distinct from the inputs)
    const void *m, *dn, *F;
    const void *rc = nullptr;    // cell damping (I_abd form only)
    double cth = 0.0;            // cos(omega_c dt) (I_abd form only)
    TBCoef cf;
};
// Batched blocked sweep: per-field descriptor (device array).  Buffers a0/a1
// hold (u_j, u_{j-1}) when parity = 0 and receive the result when parity = 1.
template <typename T>
struct BFieldT {
    int ny, nx;
    int Ns, jsnap;
    const T *m, *dn;
    const void *F;              // staged right-hand side (complex, T pairs)
    const void *Fin;            // the complex128 right-hand side it is staged from
    T *a0, *a1, *b0, *b1;
    const double *tab;          // forcing scalars (fa, fb) of steps 0..Ns-1
    double *U;                  // complex128 output
    Stencil<T> st;
};
struct TBBatchLaunch {
    const void *fields;         // device BFieldT<T>[]
    const int *list;            // device: active field indices of this launch
    const int *prefix;          // device: tile prefix sums, nlist + 1 entries
    int nlist, j0, K, parity, ntiles, shape;
    bool general;               // class pattern (3,3) instead of (3,2)
};
hipError_t launch_sweep2d_tb_batch(const TBBatchLaunch &L, bool f64, hipStream_t s);
// Start of a batched application for the n fields listed (device indices into
// the BFieldT<T> array): both recurrence fields a0, a1 zeroed and, in FP32,
// Fin converted to the staged F.  n_max: the largest field.
hipError_t launch_batch_stage_in(const void *fields, const int *list, int n, int64_t n_max,
                                 bool f64, hipStream_t s);
// Shared-medium batched tile: workgroup -> (slab, tile); a slab lists up to
// mrhs_nr(shape) fields of one medium (-1 past its end), nslab x NR ints.
struct TBMrhsLaunch {
    const void *fields;         // device BFieldT<T>[]
    const int *slabs;           // device: nslab x NR field indices
    const int *prefix;          // device: tile prefix sums, nslab + 1 entries
    int nslab, j0, K, parity, ntiles, shape;
    bool general;
};
hipError_t launch_sweep2d_tb_mrhs(const TBMrhsLaunch &L, bool f64, hipStream_t s);
int mrhs_nr(int shape, bool f64);     // right-hand sides per workgroup (0: no such shape)
int mrhs_rows(int shape, bool f64);   // extended tile rows
int tb2d_tiles(int shape, int K, int ny, int nx);

hipError_t launch_sweep2d_tb_f64(const TBArgs &a, const Stencil<double> &st, hipStream_t s);
hipError_t launch_sweep2d_tb_f32(const TBArgs &a, const Stencil<float> &st, hipStream_t s);
// blocked I_abd (shapes 4..7, mass tables without corner entries) on both
// real parts of a complex field in one launch: u_in, up_in, u_out, up_out
// complex (parts interleaved), forcing table of the real part in its Table 1
// form (the imaginary part takes (-fb, fa)), out[] complex128
hipError_t launch_sweep2d_abd2_tb_f64(const TBArgs &a, const Stencil<double> &sa,
                                      const Stencil<double> &sb, hipStream_t s);
hipError_t launch_sweep2d_abd2_tb_f32(const TBArgs &a, const Stencil<float> &sa,
                                      const Stencil<float> &sb, hipStream_t s);
int tb2d_tile_rows(int shape, bool f64);
int tb2d_tile_cols(int shape);            // 64, or 128 for the two-column shapes 9..13
inline bool tb2d_f32_only(int shape) { return shape == 2 || shape == 8 || shape == 12 || shape == 13; }
bool abd_tile_ok(int shape, bool f64);    // tile shapes of the blocked I_abd kernel

// Resident-tile 2-D sweep (sweep_res.hip): one workgroup per tile keeps its
// tile in registers for a whole run of steps and swaps k-wide halo bands with
// the neighbouring tiles through `shadow` every k steps.  Every tile must be
// resident at once (tiles <= compute units); a wait that does not end sets
// the abort word and the launch ends early with that status.
#define TDP_RES_MAXSTEPS 1024   // steps of one launch (forcing scalars staged in LDS)
#define TDP_RES_FLAG_STRIDE 32  // ints between tile flags (one 128-byte line each)
struct ResArgs {
    int ny, nx;
    int sc;
    int k;                      // steps between exchanges: 2, 4, 6 or 8
    int nsteps;                 // steps of this launch, 1..TDP_RES_MAXSTEPS
    int tiles_x, tiles_y;
    const void *u_in, *up_in;   // u_j, u_{j-1}
    void *u_out, *up_out;       // u_{j+nsteps}, u_{j+nsteps-1} (distinct from the inputs)
    const void *m, *dn, *F;
    const double *tab;          // (fa, fb) of the launch's steps
    int out_step[2];            // 1-based step whose field goes to out[i] (0: none)
    double *out[2];             // stride-2 outputs (complex128 real or imaginary part)
    void *shadow;               // [2 parities][tiles][2 levels][band] exchange buffer
    int *flags;                 // tiles x TDP_RES_FLAG_STRIDE ints, then the abort word
    int poll_limit;             // flag polls before a wait gives up
    int wait_bias;              // added to the awaited flag value (0; > 0 forces the abort path)
};
hipError_t launch_sweep2d_res_f64(const ResArgs &a, const Stencil<double> &st, hipStream_t s);
hipError_t launch_sweep2d_res_f32(const ResArgs &a, const Stencil<float> &st, hipStream_t s);
int res_tile_rows(bool f64);      // extended tile rows (64 columns)
size_t res_band_bytes(bool f64);  // exchange-buffer bytes per tile and parity (largest depth)
// tiles of the resident grid at exchange depth k (0 if k is not supported)
int res_tiles(int ny, int nx, int k, bool f64, int *tiles_x, int *tiles_y);

// 3-D sweep streamed along axis 0 (sweep3d.hip), one step per launch.
// shape 0/1/2: 8 x 64 (4 waves x 2 rows), 16 x 64 (4 waves x 4 rows), 16 x 64
// (8 waves x 2 rows) node columns per workgroup; zc planes per chunk.
hipError_t launch_sweep3d_stream_f64(const SweepArgs &a, const Stencil<double> &st, double fa,
                                     double fb, int shape, int zc, hipStream_t s);
hipError_t launch_sweep3d_stream_f32(const SweepArgs &a, const Stencil<float> &st, float fa,
                                     float fb, int shape, int zc, hipStream_t s);

// 3-D sweep streamed along axis 0, two steps per launch (sweep3d.hip):
// (u, up) = (u_j, u_{j-1}) -> (u2out, u1out) = (u_{j+2}, u_{j+1}); outputs
// distinct from the inputs; out1 / out2 (stride 2, may be null) receive
// u_{j+1} / u_{j+2} (the snapshot or the final field).
struct Stream2Args {
    int n[3];
    int sc, mc;
    int zc;                  // fewest planes per workgroup run
    int ncu;                 // compute units (one round of resident workgroups)
    const void *u, *up;
    void *u2out, *u1out;
    const void *m, *dn, *F;
    double fa[2], fb[2];     // forcing scalars of the two steps
    double *out1, *out2;
};
hipError_t launch_sweep3d_stream2_f64(const Stream2Args &a, const Stencil<double> &st, int shape,
                                      hipStream_t s);
hipError_t launch_sweep3d_stream2_f32(const Stream2Args &a, const Stencil<float> &st, int shape,
                                      hipStream_t s);
// queries the residency of the shape's kernels (call before any stream capture)
void sweep3d_stream2_prepare(bool f64, int shape);

// complex-linear variant: u, up are complex fields (re, im pairs of T); `out`
// (if non-null) receives u_{j+1} as complex128.
hipError_t launch_sweep_c_f64(const SweepArgs &a, const Stencil<double> &st, double fa,
                              double fb, hipStream_t s);
hipError_t launch_sweep_c_f32(const SweepArgs &a, const Stencil<float> &st, float fa, float fb,
                              hipStream_t s);

// I_abd step on complex fields (Sec. 6): a.u = u_n, a.up = u_{n-1} (read only),
// u_{n+1} -> uout; rc the cell damping; stB the mass-class stencil of L/ImH.
hipError_t launch_sweep_abd_f64(const SweepArgs &a, void *uout, const double *rc,
                                const Stencil<double> &stA, const Stencil<double> &stB,
                                double cth, double fa, double fb, hipStream_t s);
hipError_t launch_sweep_abd_f32(const SweepArgs &a, void *uout, const float *rc,
                                const Stencil<float> &stA, const Stencil<float> &stB, float cth,
                                float fa, float fb, hipStream_t s);

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_cvt_c128_to_c64(const void *F, void *Fs, int64_t N, hipStream_t s);
hipError_t launch_cvt_f64_to_f32(const double *x, float *y, int64_t N, hipStream_t s);
hipError_t launch_phase_extract(void *U, int64_t N, double c, double s, hipStream_t st);

// y = H x   or   y = F - H x  (when F != null); complex128.  Im H = diag(rw),
// or with rc != null the mass-class stencil stI over the cell damping rc.
hipError_t launch_apply_H(int ndim, const int *n, int sc, int mc, const double *m,
                          const double *rw, const double *rc, const Stencil<double> &st,
                          const Stencil<double> &stI, const void *x, const void *F, void *y,
                          hipStream_t s);

// setup kernels
hipError_t launch_cell_slowness(int ndim, const int *n, const double *c, double *m,
                                hipStream_t s);
hipError_t launch_cell_mean(int ndim, const int *n, const double *v, double *cells,
                            hipStream_t s);
hipError_t launch_max_reduce(const double *x, int64_t N, double *partial, int nblk,
                             double *out, hipStream_t s);
hipError_t launch_node_factors(const double *R, int64_t N, double omega, double lscale,
                               double *rw, double *dn, hipStream_t s);

// Krylov kernels (complex128, FP64 reductions, deterministic order)
int blas_nblocks(int64_t N);
hipError_t launch_mdot(const void *V, int64_t ldv, int nv, const void *w, int64_t N,
                       double *partial, int nblk, double *out, hipStream_t s);
hipError_t launch_maxpy(void *w, const void *V, int64_t ldv, int nv, const double *coef,
                        double sign, int64_t N, hipStream_t s);
// one field of a batched CGS2 step (launch_gs_step_multi): V holds nv
// columns of N (column stride N); w is orthogonalised in place and vnext =
// w / |w|; red holds 2 nblk nv partial sums; co receives h1 at co[0..2nv),
// h2 at co[off2..), |w|^2 at co[offn]; its first ncopy doubles are then
// copied to gather
struct GsField {
    const double2 *V;
    double2 *w, *vnext;
    double *red, *co, *gather;
    int64_t N;
    int nv, nblk, off2, offn, ncopy;
};
hipError_t launch_gs_step_multi(const GsField *gf, int nf, int nv_max, int nblk_max,
                                int64_t n_max, hipStream_t s);
hipError_t launch_scale_by_invnorm(void *v, const void *w, const double *nrm2, int64_t N,
                                   hipStream_t s);
// The other per-field steps of the lockstep GMRES on several 2-D fields at
// once: (update) x_out = x_in + V y for fields with k > 0; r = F - H xh, or
// r = H xh when F is null, with the field's operator (m, rw, st = its H
// stencil; diagonal damping); (norm) |r|^2 to out[0] (and the imaginary
// part, 0, to out[1]) for fields with out set, through red (2 nblk doubles).
struct TrField {
    const double2 *V, *x_in;
    double2 *x_out;
    const double *y;
    const double2 *xh, *F;
    double2 *r;
    const double *m, *rw;
    double *red, *out;
    Stencil<double> st;
    int64_t N;
    int k, nblk, ny, nx;
};
hipError_t launch_tr_multi(const TrField *tf, int nf, bool update, bool norm, bool general,
                           int nblk_max, int64_t n_max, int ny_max, int nx_max, hipStream_t s);

// gradient
hipError_t launch_grad_cells(int ndim, const int *n, double w2, const double *mass,
                             const void *lam, const void *U, double *gcell, hipStream_t s);
hipError_t launch_grad_nodes(int ndim, const int *n, const double *gcell, double *grad,
                             hipStream_t s);

// Stream discipline: work is issued on the caller's stream when one is given.
// For the default (NULL) stream, which cannot be captured into a graph, the op
// owns a stream and orders it after the caller's stream at entry and before
// it at exit.
struct StreamJoin {
    hipStream_t user, own;
    hipEvent_t ev;
    StreamJoin(hipStream_t u, hipStream_t o, hipEvent_t e) : user(u), own(o), ev(e)
    {
        if (ev && hipEventRecord(ev, user) == hipSuccess) (void)hipStreamWaitEvent(own, ev, 0);
    }
    ~StreamJoin()
    {
        if (ev && hipEventRecord(ev, own) == hipSuccess) (void)hipStreamWaitEvent(user, ev, 0);
    }
};

}  // namespace tdp

struct tdp_op;
// host helpers shared by op.cpp and batch.cpp
const std::vector<double> &forcing_table(tdp_op *op, int T, double rho, int variant);
int64_t snap_lag(int nP);   // Table 1's second sample lies snap_lag(n_P) steps before the end
int apply_H_impl(const tdp_op *op, const void *x, const void *F, void *y);
// Table 1 on the fields `bufs` (4 planes of the op's field precision) with
// F staged in `f32_stage` (N complex64, FP32 fields only), issued launch by
// launch without graph capture, staging copies or forcing tables.
int precond_noalloc_impl(tdp_op *op, int T, double rho, const void *F, void *U,
                         const tdp::LoopBufs &bufs, void *f32_stage);
// Device scratch of the allocation-free entry point (noalloc.hip): looked up
// once per device at op creation, with that device current.
int noalloc_setup_device(int dev);

// The opaque operator.
struct tdp_op {
    int ndim = 0;
    int device = 0;          // HIP device current at creation
    int n[3] = {1, 1, 1};
    int64_t N = 0, Nc = 0;
    double h = 0, omega = 0;
    double S[4] = {0, 0, 0, 0}, M[4] = {0, 0, 0, 0};
    int sc = 0, mc = 0;
    int prec = TDP_F64;
    hipStream_t stream = nullptr;
    // derived parameters
    double omega_c = 0, lam_bar = 0, dt = 0, alpha = 0, beta = 0;
    int nP = 0;
    double cS = 0, cM = 0, cw = 0, g = 0;
    tdp::Stencil<double> st_step{}, st_H{};
    // cell damping (Sec. 6): Im H = omega sum_cells r_cell M_cell, integrator I_abd
    int dform = TDP_DAMP_NODE;
    double lam_im = 0, cos_th = 0;
    double *rc = nullptr;                   // cell damping r_cell
    tdp::Stencil<double> st_I{}, st_B{};    // Im H and (beta dt/(alpha omega)) Im H (mass classes)
    tdp::Stencil<float> st_B32{};
    float *rc32 = nullptr;                  // FP32 copy of the cell damping
    void *u4 = nullptr, *u5 = nullptr;      // third and fourth complex fields of the I_abd loops
    tdp::Stencil<float> st_step32{};
    // device buffers
    double *m = nullptr;       // cell slowness
    double *rw = nullptr;      // omega * R at nodes
    double *dn = nullptr;      // 1 / (1 + l/2) at nodes
    float *m32 = nullptr, *dn32 = nullptr;
    void *u0 = nullptr, *u1 = nullptr;      // recurrence fields (prec)
    void *u2 = nullptr, *u3 = nullptr;      // complex fields of the complex-linear variant
    void *v0 = nullptr, *v1 = nullptr;      // second field pair of the blocked sweep
    void *Fst = nullptr;                    // staged F (float2) for FP32
    double *scratch = nullptr;              // small device scratch
    size_t scratch_bytes = 0;
    // Krylov workspace (lazily sized)
    void *V = nullptr;
    int V_cols = 0;
    void *wv = nullptr, *tv = nullptr, *rv = nullptr, *xv = nullptr;
    double *red = nullptr;     // reduction partials
    size_t red_bytes = 0;
    double *dcoef = nullptr;   // device small vector (coefficients / results)
    double *hres = nullptr;    // pinned host mirror
    // forcing tables per (T, rho)
    std::map<std::tuple<int, double, int>, std::vector<double>> tables;
    // captured step loops, keyed by (T, rho, variant, kernel, depth, tile)
    // captured loops by (T, rho, variant, kernel, depth, tile, F, U); F = U =
    // nullptr for loops on the staging buffers
    std::map<std::tuple<int, double, int, int, int, int, const void *, const void *>,
             hipGraphExec_t> graphs;
    tdp_tuning tune{0, 0, 1, 0};
    // stream join with the caller, staging buffers of the captured loop
    hipStream_t user_stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev = nullptr;
    hipEvent_t tev[6] = {};    // GMRES phase timing: (start, end) per phase
    void *Fstage = nullptr;    // complex128 input of the captured loop (FP64)
    void *Ustage = nullptr;    // complex128 output of the captured loop
    double *gcell = nullptr;   // per-cell gradient scratch
    // resident-tile sweep (kernel 5): compute units of the device, the
    // exchange planes and tile flags, device copies of the forcing tables,
    // a pinned mirror of the abort word
    int ncu = 0;
    void *res_shadow = nullptr;
    int *res_flags = nullptr;
    int res_ntiles = 0;                    // tiles the flag array holds
    int res_aborts = 0;                    // resident launches redone with the blocked sweep
    bool res_force_abort = false;          // test hook: every resident wait gives up
    int *res_host = nullptr;
    std::map<std::tuple<int, double, int>, double *> dtables;
};
