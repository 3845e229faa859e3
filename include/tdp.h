/*
 * tdp.h -- C ABI of the MI355X time-domain preconditioner for the Helmholtz
 * equation (C. C. Stolk, "A time-domain preconditioner for the Helmholtz
 * equation").
 *
 * Problem (Sec. 1, eq. 3 and the linear system H U = F of Sec. 1):
 *     -Lap U - omega^2/c(x)^2 U + i omega R(x) U = F
 * on an interior grid of n_0 x n_1 [x n_2] nodes with spacing h and U = 0
 * outside the box (Dirichlet, Sec. 3.1).  Re H is the compact 9-point (2-D) /
 * 27-point cube (3-D) stencil assembled cell by cell (App. A): each grid cell
 * couples its corners b, g with h^-2 S[Delta] - omega^2 m_cell M[Delta],
 * Delta = number of axes on which b and g differ, m_cell the mean of 1/c^2
 * over the cell's corners (corners outside the box take the nearest interior
 * node).  Im H = diag(omega R), or with the cell damping of Sec. 6
 * (tdp_op_desc.damping = TDP_DAMP_CELL) Im H = omega sum_cells r_cell M[Delta],
 * r_cell the mean of R over the cell's corners.
 *
 * Conventions for every entry point:
 *  - Arrays are DEVICE pointers owned by the caller, contiguous, row-major
 *    [n0][n1][n2] (last axis fastest).  Complex arrays are interleaved
 *    complex128 (re, im pairs; torch.complex128), 16-byte aligned (as every
 *    element of a torch.complex128 tensor is; others get TDP_EINVAL).  Real
 *    node arrays are FP64.
 *  - All work is issued on the op's stream (tdp_op_desc.stream).  Calls that
 *    return results to the host (gmres) synchronise that stream.
 *  - Return value: TDP_OK (0), a positive status for a completed call with a
 *    caveat, or a negative error.  On a negative return nothing was written
 *    to the output arrays.  tdp_last_error() gives a message (per thread).
 *  - The op never keeps caller pointers after a call returns.  Input and
 *    output arrays of one call must not overlap.
 *  - One op must not be used by two host threads at the same time.
 */
#ifndef TDP_H
#define TDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TDP_OK = 0,
    TDP_ENOTCONV = 1,   /* gmres: iteration limit reached, U holds the last iterate */
    TDP_EINVAL = -1,    /* invalid argument (sizes, c <= 0, R < 0, h <= 0, ...)     */
    TDP_ENOMEM = -2,    /* device allocation failed                                 */
    TDP_EHIP = -3,      /* HIP runtime error                                        */
    TDP_ECFL = -4       /* requested steps per period violate the CFL bound         */
};

typedef enum { TDP_F64 = 0, TDP_F32 = 1 } tdp_prec;

/* Damping discretisation and the integrator it selects.
 *  TDP_DAMP_NODE  Im H = diag(omega R): I_acd (Def. 2), Table 1 / Def. 4.
 *  TDP_DAMP_CELL  Im H = omega sum_cells r_cell M[Delta], not diagonal: the
 *                 explicit I_abd of Sec. 6 (Def. 6) and S_T^abd (Def. 7). */
typedef enum { TDP_DAMP_NODE = 0, TDP_DAMP_CELL = 1 } tdp_damping;

typedef struct tdp_op tdp_op;

/* Operator description (Sec. 2.2: the preconditioner's parameters follow from
 * H alone).
 *  ndim              2 or 3
 *  n[0..ndim-1]      interior nodes per axis (>= 1, <= 2^20); n[ndim..2]
 *                    ignored.  The node-per-thread kernels launch 4 rows of
 *                    axis ndim-2 and one plane of axis 0 (3-D) per block row,
 *                    so 2-D n[0] <= 262139 and 3-D n[0] <= 65534,
 *                    n[1] <= 262139 (else TDP_EINVAL); N <= 2^36.
 *  h                 grid spacing (> 0)
 *  omega             physical angular frequency (> 0)
 *  c                 device, [N] wave speed at the nodes (> 0)
 *  R                 device, [N] damping at the nodes (>= 0), or NULL for 0
 *  stiff, mass       HOST, ndim+1 cell-table entries each (by Delta = 0..d);
 *                    NULL selects the classical fourth-order compact scheme:
 *                    2-D S = {5/6, -1/3, -1/6},  M = {1/6, 1/24, 0}
 *                    3-D S = {1/2, -1/12, -1/12, 0}, M = {1/16, 1/48, 0, 0}.
 *                    The second-order scheme of Sec. 3.1 (5- / 7-point
 *                    Laplacian, lumped mass) is
 *                    2-D S = {1, -1/2, 0},       M = {1/4, 0, 0}
 *                    3-D S = {3/4, -1/4, 0, 0},  M = {1/8, 0, 0, 0};
 *                    its mass term uses the cell slowness, so at a node it
 *                    weighs 1/c^2 over the surrounding 3^d nodes.
 *                    The cell tables must be positive semidefinite as element
 *                    matrices with max eigenvalue of M <= 2^-d (App. A bound).
 *  steps_per_period  n_P; 0 selects the smallest multiple of 4 above the CFL
 *                    bound of Sec. 2.2 (Table 1's default), -1 the smallest
 *                    integer >= 3 above it; a given value must be >= 3 and
 *                    above that bound, else TDP_ECFL.  When 4 does not
 *                    divide n_P, Table 1 takes its second sample q =
 *                    round(n_P/4) steps before the end and obtains Im U by
 *                    the 2x2 solve the paper suggests for that case
 *                    (Sec. 2.3): u_{N_s-q} = cos(phi) Re U + sin(phi) Im U,
 *                    phi = 2 pi q/n_P.
 *  prec              precision of the recurrence fields (Table 1 loop).
 *                    Krylov vectors, H and the residuals are always FP64.
 *  stream            hipStream_t every call of this op issues its work on.
 *                    NULL (the default stream) makes the op use a private
 *                    stream ordered after / before the default stream at
 *                    each call's entry / exit (the step loop is captured
 *                    into a graph, which the default stream cannot hold).
 *  damping           tdp_damping (0 = TDP_DAMP_NODE).  TDP_DAMP_CELL: omega_c,
 *                    dt and n_P follow Sec. 6.1 (omega_c^2 = k_max^2 +
 *                    (beta/theta)(1 - cos theta) lam_im, theta = omega_c dt =
 *                    2 pi/n_P the largest for which 4I - K - 2L > 0 holds on
 *                    the bounds); FP64 or FP32 fields; preconditioning is S_T^abd
 *                    (tdp_precond_apply returns TDP_EINVAL, GMRES uses the
 *                    complex-linear map whatever its variant); not batched. */
typedef struct {
    int ndim;
    int64_t n[3];
    double h;
    double omega;
    const double *c;
    const double *R;
    const double *stiff;
    const double *mass;
    int steps_per_period;
    int prec;
    void *stream;
    int damping;
} tdp_op_desc;

/* Derived parameters (Sec. 2.2, Prop. 1): omega_c = omega sqrt(max m_cell)
 * (computational frequency), dt = 2 pi / (omega_c n_P),
 * alpha = (omega_c dt)^2 / (4 sin^2(omega_c dt / 2)),
 * beta = omega_c dt / sin(omega_c dt), lam_bar = upper bound on lambda_max(A),
 * lam_im = upper bound on lambda_max(Im H) with the cell damping (else 0).
 * res_aborts: resident-tile launches (tuning kernel 5) that ended early
 * because not every tile was resident; each such application was redone
 * with the blocked sweep, and the op's tuning went back to auto. */
typedef struct {
    double omega_c, dt, alpha, beta, lam_bar;
    int n_P;
    int ndim;
    int64_t N;
    double lam_im;
    int res_aborts;
} tdp_op_info;

/* GMRES configuration (Sec. 2.4: left preconditioning P H U = P F with
 * P = S_T of Table 1).
 *  restart      Krylov dimension m per cycle (>= 1)
 *  max_iters    limit on preconditioned operator applications (>= 1)
 *  periods_T    T, periods per preconditioner application (N_s = T n_P
 *               <= 2^24 in every entry point, else TDP_EINVAL)
 *  rho          window parameter in (0, 1]; <= 0 means rho = 1/T
 *  tol          target for the true relative residual ||F - H U|| / ||F||
 *  x0_given     1: U holds the initial guess on entry; 0: start from 0
 *  fixed_iters  > 0: run exactly this many iterations (restarting every
 *               `restart`), no early stop
 *  variant      0: P = Table 1 (real field, 7 words per node-step);
 *               1: P = Definition 4 as stated (complex field, 10 words) */
typedef struct {
    int restart, max_iters, periods_T;
    double rho, tol;
    int x0_given;
    int fixed_iters;
    int variant;
} tdp_gmres_cfg;

/* GMRES report (host struct).  With TDP_LOG=1 in the environment the solve
 * also prints one line per cycle and a summary to stderr.  history (host,
 * may be NULL) receives the
 * Givens estimate of ||P r|| / ||P r_0|| after each iteration, up to
 * history_cap entries.  switched = 1 when a tolerance-mode solve with
 * variant 0 rejected a cycle and continued with variant 1 (see
 * tdp_gmres_solve). */
typedef struct {
    int iters, restarts;
    double relres_true, relres_prec;
    int64_t steps;           /* recurrence steps executed               */
    double ms_total;         /* host wall time of the call              */
    double *history;
    int history_cap, history_len;
    int switched;
    double ms_precond;       /* GPU time of the preconditioner applications,
                                of the H-applies and of the Gram-Schmidt
                                kernels (HIP events on the op's stream; 0
                                in the batched form)                     */
    double ms_H, ms_arnoldi;
} tdp_gmres_info;

/* Create an operator: validates the description, copies c and R, computes
 * the cell slowness, omega_c, n_P, dt, alpha, beta and per-node damping
 * factors, and allocates the recurrence fields.  Sec. 2.2, App. A. */
int tdp_op_create(const tdp_op_desc *desc, tdp_op **out);

/* Free an operator and its device buffers (NULL is accepted). */
int tdp_op_destroy(tdp_op *op);

/* Copy the derived parameters to *out (host). */
int tdp_op_query(const tdp_op *op, tdp_op_info *out);

/* y = H x.  x, y: device complex128 [N].  Sec. 1 (H U = F), App. A. */
int tdp_apply_H(const tdp_op *op, const void *x, void *y);

/* U = S_T F, the real-field algorithm of Table 1 (Sec. 2.3): zero fields,
 * N_s = T n_P steps of the integrator I_acd (Def. 2) driven by
 * chi(1 - j/N_s) [cos(2 pi j/n_P) Re F - sin(2 pi j/n_P) Im F], then
 * U = u_{N_s} + i u_{N_s - n_P/4} (for 4 not dividing n_P, Im U from the
 * 2x2 solve described at steps_per_period).  chi is the sine-square window with
 * parameter rho (rho <= 0: rho = 1/T).  F, U: device complex128 [N]. */
int tdp_precond_apply(const tdp_op *op, int periods_T, double rho, const void *F, void *U);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * U = S_T F as tdp_precond_apply (Table 1, same kernels and tuning), with the
 * recurrence fields (and, for FP32 fields, the complex64 copy of F) in one
 * static device array of TDP_NOALLOC_MAX_BYTES per GPU instead of buffers of
 * the op.  The call allocates nothing (no hipMalloc, hipFree, graph
 * instantiation or forcing-table cache); its launches are issued directly on
 * the op's stream.  Needs 32 bytes per node with FP64 fields and 24 with FP32
 * fields (each part rounded up to 256 bytes): FP64 grids up to 2^21 nodes.
 * Larger grids return TDP_EINVAL before any work is issued.  Every call on
 * one GPU uses that GPU's one array, and each call starts by zeroing the
 * fields it uses: calls that overlap in time on one GPU (two streams, two
 * ops, two host threads) race and give wrong results.  Ops with the cell
 * damping return TDP_EINVAL, as tdp_precond_apply does.
 * F, U: device complex128 [N], distinct. */
#define TDP_NOALLOC_MAX_BYTES (64u << 20)
int tdp_precond_apply_noalloc(const tdp_op *op, int periods_T, double rho, const void *F,
                              void *U);

/* U = S_T F by Definition 4 (Sec. 2.3) as stated: the integrator I_acd on a
 * complex field driven by chi(1 - j/N_s) e^{i 2 pi j/n_P} F from zero fields,
 * U = e^{-i 2 pi T} u_{N_s} = u_{N_s}.  Complex-linear, unlike Table 1 whose
 * output is only real-linear.  The recurrence has real coefficients, so the
 * real and imaginary parts run as two real passes of the blocked (2-D) or
 * streamed (3-D) kernels; with tdp_tuning.kernel = 1 as one complex pass
 * (10 instead of 7 words per node-step).
 * With TDP_DAMP_CELL this is S_T^abd (Sec. 6, Def. 7): the same forcing
 * driving I_abd (Def. 6).  Its recurrence has real coefficients too: in 2-D
 * (mass tables without corner entries) the blocked I_abd kernel advances
 * both real parts k steps per launch, else, and with
 * tdp_tuning.kernel = 1, on the complex field one step per launch (10 words
 * per node-step; u_{n-1} is read with its neighbours, so u_{n+1} goes to a
 * third field).
 * F, U: device complex128 [N]. */
int tdp_precond_apply_complex(const tdp_op *op, int periods_T, double rho, const void *F,
                              void *U);

/* Solve H U = F with left-preconditioned restarted GMRES (Sec. 2.4).
 * After every iteration the current iterate x0 + V y is formed and its true
 * relative residual ||F - H x|| / ||F|| evaluated in FP64; the solve stops as
 * soon as it is <= tol.  A cycle ends after `restart` iterations, or earlier
 * when the true residual stalls while the Givens estimate of the
 * preconditioned residual keeps falling (relt > 2 rel_start est_cycle and
 * relt > 0.7 rel_prev; the Table 1 map is only real-linear, so the Arnoldi
 * relation holds only approximately).  A cycle keeps its iterate with the
 * smallest true residual, and stops early if that residual runs away (> 1e6
 * times the cycle's start, or not finite).  A variant-0 cycle that does not
 * lower the true residual is rejected (x unchanged) and the solve continues
 * with variant 1, whose complex-linear map GMRES handles exactly (when T is
 * short, Table 1's real-linearity defect makes the complex least-squares
 * update useless); a variant-1 cycle keeps its last iterate in that case.
 * Returns TDP_OK, or TDP_ENOTCONV with the accepted iterate in U.
 * F, U: device complex128 [N]; info: host or NULL. */
int tdp_gmres_solve(const tdp_op *op, const tdp_gmres_cfg *cfg, const void *F, void *U,
                    tdp_gmres_info *info);

/* Gradient of a real loss with respect to the squared slowness m = 1/c^2 at
 * the nodes, given U = H^-1 F and the adjoint field lam = H^-H (dL/dU*):
 * dL/dm_cell = omega^2 Re sum_{b,g in cell} M[Delta(b,g)] conj(lam_b) U_g
 * (since dH/dm_cell = -omega^2 M_cell), mapped to the nodes by the adjoint of
 * the corner averaging that defines m_cell.  lam, U: device complex128 [N];
 * grad: device FP64 [N] (overwritten). */
int tdp_grad_m(const tdp_op *op, const void *lam, const void *U, double *grad);

/* Tuning of the recurrence sweep (no effect on results beyond rounding).
 *  kernel       0 auto (kernel, depth and tile chosen by the library: the
 *               blocked 2-D sweep on tile 5 (FP64) or 8 (FP32) at depth 8, with
 *               the cell damping on tile 7 (FP64) or 4 (FP32); in 3-D the
 *               two-step streamed sweep for tables without corner entries
 *               (FP64 tile 1; FP32 tile 2, tile 1 below 3 * 2^20 nodes) and
 *               the one-step streamed sweep on tile 0 otherwise; tb_depth and
 *               tile ignored),
 *               1 one step per launch, 2 temporally blocked (2-D; with the
 *               cell damping, tiles 5 and 7 in FP64 and 4..7 in FP32, mass
 *               tables without corner entries), 3 streamed along axis 0 (3-D, Table 1
 *               variant), 4 streamed along axis 0 with two steps per launch
 *               (3-D, Table 1 variant), 5 resident tiles (2-D, node
 *               damping, tables without corner mass entries: each tile,
 *               88x64 in FP64 and 112x64 in FP32, stays on one compute unit
 *               for up to 1024 steps per launch and swaps k-wide halo bands
 *               with its neighbours through global memory every k steps; the
 *               tiles must fit the compute units and all be resident at
 *               once: when other work holds compute units a wait gives up,
 *               the application is redone with the blocked sweep and the
 *               op's tuning goes back to auto (tdp_op_info.res_aborts);
 *               where kernel 5 does not apply it falls back to the auto
 *               choice); inapplicable choices fall back to 1
 *  tb_depth     kernel 2: steps per launch, 1..16 (0 auto);
 *               kernel 5: steps between halo exchanges, 2, 4, 6 or 8 (0: 4);
 *               kernel 3: planes per chunk (0 auto: 32, halved down
 *               to 8 until the launch has about 8192 waves); kernel 4: the
 *               fewest planes per workgroup run (0: 8; the launch is one
 *               round of resident workgroups sharing the (column block,
 *               plane) units equally, so this only limits how finely a
 *               small grid is split)
 *  use_graph    1 capture the step loop in a hipGraph and replay it (loops
 *               of more than 2^17 launches are issued directly)
 *  tile         kernel 2 tile (rows x columns): 0 64x64 (8 rows per lane x
 *               8 waves), 1 64x64 (4 x 16 waves), 2 128x64 (FP32 only),
 *               3 32x64 (4 x 8 waves); 4..7 the same family with per-node
 *               coefficients in registers: 4 64x64 (4 x 16), 5 32x64 (4 x 8),
 *               6 64x64 (8 x 8), 7 32x64 (2 x 16), 8 128x64 (8 x 16, FP32 only);
 *               kernel 3: 0 8x64 columns (4 waves x 2
 *               rows each), 1 16x64 (4 waves x 4 rows), 2 16x64 (8 x 2);
 *               kernel 4: level 1 on a 66-wide block with a one-node rim,
 *               level 2 (the output) on its interior: 0 66x15 on 512
 *               threads (two nodes each, output 13x64), 1 66x15 on 1024
 *               threads (one node each), 2 66x31 on 1024 threads (output
 *               29x64; FP32 only, FP64 runs shape 1)                      */
typedef struct {
    int kernel;
    int tb_depth;
    int use_graph;
    int tile;
} tdp_tuning;

int tdp_op_set_tuning(tdp_op *op, const tdp_tuning *t);

/* Test hook of the resident sweep's recovery path (tuning kernel 5): with
 * on = 1, each resident launch of this op waits for a flag value that no
 * tile writes, gives up after 16 polls and ends early, as it does when its
 * tiles are not all resident; the application is then redone with the
 * blocked sweep and counted in tdp_op_info.res_aborts.  on = 0 restores the
 * normal waits.  Returns TDP_OK or TDP_EINVAL. */
int tdp_op_force_resident_abort(tdp_op *op, int on);

/* Autotuner: times each sweep variant applicable to this op (one step per
 * launch; blocked tile shapes x depths 2-10, 12, 16 (4 x depth
 * at most the tile's rows) and the resident tiles at exchange depths 2, 4, 6,
 * 8 for the 2-D Table 1 loop; the blocked I_abd tiles
 * x depths 2, 3, 4, 6, 8 with the 2-D cell damping; in 3-D the one-step
 * streamed shapes x chunk lengths 4, 8, 16, 32, 64 and the two-step shapes x
 * shortest runs 8 and 32) over
 * periods_T periods with HIP events on the op's stream, and makes
 * the fastest the op's tuning.  best (host, may be NULL) receives it; table
 * (host, may be NULL) receives up to cap rows of {kernel, tb_depth, tile,
 * microseconds per step}.  Returns the number of candidates timed (> 0) or a
 * negative error.  Overwrites the op's internal staging buffers only. */
int tdp_op_autotune(tdp_op *op, int periods_T, double rho, int variant, tdp_tuning *best,
                    double *table, int cap);
int tdp_op_get_tuning(const tdp_op *op, tdp_tuning *t);

/* ---------------------------------------------------------------------
 * Batched form: many right-hand sides per operator and many operators of
 * uneven sizes (2-D, one precision, one stream, one stencil class pattern)
 * solved together.  Field q enumerates (op 0, rhs 0..nrhs[0]-1), (op 1, ...).
 * One batched preconditioner application (Table 1) advances every live field
 * by k steps per launch of the blocked sweep, each with its own medium,
 * forcing table and step count.  The live right-hand sides of one operator
 * (two or more) go through the shared-medium tile: one workgroup advances a
 * slab of several of them over one tile, loading the medium (cell slowness,
 * damping) and folding its stencil coefficients once for the slab, so a
 * node-step moves 5 + 2/slab words per right-hand side instead of 7.  The
 * application is replayed from one hipGraph (at most
 * 2^17 launches, i.e. max N_s <= 2^17 k, else TDP_EINVAL); GMRES runs
 * per field in lockstep and takes the same decisions as tdp_gmres_solve.
 * The batch keeps pointers to the ops: they must outlive it.  Ops with the
 * cell damping are refused (TDP_EINVAL). */
typedef struct tdp_batch tdp_batch;

int tdp_batch_create(tdp_op *const *ops, int nops, const int *nrhs, tdp_batch **out);
int tdp_batch_destroy(tdp_batch *b);

/* Steps per launch (1..15), tile shape of single fields (as tdp_tuning.tile)
 * and shared-medium tile of the batched blocked sweep.  medium_tile: -1 runs
 * every field on its own tile; 0..2 select rows per lane x waves and
 * right-hand sides per workgroup:
 *   FP32 fields  0: 4 x 8, 4 (32 x 64 tile)   1: 6 x 8, 2 (48 x 64)    2: 8 x 8, 2 (64 x 64)
 *   FP64 fields  0: 2 x 16, 3 (32 x 64)       1: 4 x 8, 2 (32 x 64)    2: 2 x 16, 2 (32 x 64)
 * Default: depth 8, tile 8 (FP32) or 4 (FP64), medium tile 0.  4 x depth
 * must not exceed either tile's rows (else TDP_EINVAL). */
int tdp_batch_set_tuning(tdp_batch *b, int depth, int tile, int medium_tile);

/* Autotuner of the batched sweep: times one batched application for every
 * depth (4, 6, 8) x single-field tile shape with every field on its own tile
 * (medium_tile -1), then every shared-medium tile with that depth's best
 * single-field tile, and keeps the fastest.  table (host, may be NULL) receives up to cap rows {depth, tile,
 * medium_tile, milliseconds per application}.  Returns the number of
 * candidates timed or a negative error. */
int tdp_batch_autotune(tdp_batch *b, const int *periods_T, double rho, double *table, int cap);

/* U[q] = S_T F[q] for every field (Table 1).  periods_T: host [nops];
 * F, U: host arrays of device complex128 pointers, one per field. */
int tdp_batch_precond(tdp_batch *b, const int *periods_T, double rho, const void *const *F,
                      void *const *U);

/* Solve every field (cfg->variant must be 0) with the iteration of
 * tdp_gmres_solve in lockstep; a field whose cycle is rejected stops there
 * (TDP_ENOTCONV, best iterate in U) since only Table 1 is batched.
 * infos: host [nfields] or NULL.  Returns TDP_OK if every field converged,
 * TDP_ENOTCONV otherwise. */
int tdp_batch_solve(tdp_batch *b, const tdp_gmres_cfg *cfg, const int *periods_T,
                    const void *const *F, void *const *U, tdp_gmres_info *infos);

/* Message of the last failing call on this thread ("" if none). */
const char *tdp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
