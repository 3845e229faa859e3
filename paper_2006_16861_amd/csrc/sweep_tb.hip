// Temporally blocked 2-D recurrence sweeps: one launch advances a real field
// by k <= TB_KMAX steps.
//
// Each workgroup owns an extended tile of EY x EX nodes (EX = 64 = one wave
// across x, EY = R rows per lane x W waves).  Values within s nodes of the
// tile edge are wrong after s steps (their neighbours outside the tile are
// taken as 0), so after k steps the inner (EY - 2k) x (EX - 2k) nodes are
// exact and are the ones written back.  Nodes outside the domain stay 0
// (Dirichlet).  HBM traffic per node-step falls from 7 words to about
// (6 (EY EX) / (out area) + 2) / k words.  Three tile updates live here:
//  - tb_tile (shapes 0..3): u_j and the cell slowness of the tile in LDS;
//    u_{j-1}, the damping factor and the right-hand side in registers
//    (Table 1 loop, I_acd of Def. 2);
//  - tb_tile2 (shapes 4..8, the default): per-node coefficients and the rows
//    of u_j, u_{j-1} in registers, x-neighbours by DPP, only each wave's edge
//    rows through LDS (same integrator);
//  - tb_tile_abd2: the same register form for I_abd (Sec. 6, cell damping) on
//    both real parts of the complex field at once.
//
// Workgroups are mapped XCD-aware: the hardware deals consecutive workgroup
// ids round-robin to the 8 XCDs, so id -> tile is remapped to give each XCD a
// contiguous band of tiles (halo rows shared by neighbouring tiles then hit in
// that XCD's L2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tdp_internal.h"
#include "lanes.h"

namespace tdp {

// assembled 9-point stencil from LDS (same formula as eval_stencil in
// kernels.hip, specialised to 2-D): uc(r, e) is the field at tile row r,
// column e (padded by one zero row/column on each side), cl the cells.
template <int SC, int MC, typename T>
__device__ __forceinline__ T stencil9(const T *__restrict__ ul, int us, const T *__restrict__ cl,
                                      int cs, const Stencil<T> &st)
{
    // ul points at the node, us = LDS row stride; cl points at the cell with
    // storage (y, x) of the node (its lower-left cell), cs = cell row stride.
    const T uC = ul[0];
    const T uW = ul[-1], uE = ul[1], uS = ul[-us], uN = ul[us];
    const T uSW = ul[-us - 1], uSE = ul[-us + 1], uNW = ul[us - 1], uNE = ul[us + 1];
    const T mSW = cl[0], mSE = cl[1], mNW = cl[cs], mNE = cl[cs + 1];
    T r = st.c0 * uC;
    const T e1 = (uW + uE) + (uS + uN);
    const T e2 = (uSW + uSE) + (uNW + uNE);
    r += st.s[1] * e1;
    if (SC > 2) r += st.s[2] * e2;
    if (MC > 0) r += st.m[0] * (((mSW + mSE) + (mNW + mNE)) * uC);
    if (MC > 1)
        r += st.m[1] * ((mSW + mNW) * uW + (mSE + mNE) * uE + (mSW + mSE) * uS + (mNW + mNE) * uN);
    if (MC > 2) r += st.m[2] * (mSW * uSW + mSE * uSE + mNW * uNW + mNE * uNE);
    return r;
}

// One tile of the blocked sweep: extended tile origin (gy0, gx0) (the exact
// output starts k rows/columns further in), k steps with forcing scalars
// fa[s], fb[s] (scaled by g), outputs of step out_step[i] (1-based) to out[i].
template <typename T, int SC, int MC, int R, int W>
__device__ __forceinline__ void tb_tile(T *__restrict__ ul, T *__restrict__ cl,
                                        const T *__restrict__ u_in, const T *__restrict__ up_in,
                                        T *__restrict__ u_out, T *__restrict__ up_out,
                                        const T *__restrict__ m, const T *__restrict__ dn,
                                        const typename V2t<T>::type *__restrict__ F, int ny,
                                        int nx, const Stencil<T> &st, int k, int halo,
                                        int gy0, int gx0, const double *fa, const double *fb,
                                        int fstride, const int *out_step, double *const *out)
{
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;          // LDS row stride of u (one zero pad each side)
    constexpr int CS = EX + 1;          // LDS row stride of the cells
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;

    // zero the LDS pads (rows 0 and EY+1, columns 0 and EX+1)
    for (int t = threadIdx.x; t < US; t += 64 * W) {
        ul[t] = T(0);
        ul[(EY + 1) * US + t] = T(0);
    }
    for (int t = threadIdx.x; t < EY + 2; t += 64 * W) {
        ul[t * US] = T(0);
        ul[t * US + EX + 1] = T(0);
    }
    // cells (storage rows gy0 .. gy0+EY, columns gx0 .. gx0+EX) and node data
    // are all loaded into registers before any of it goes to LDS, so the tile
    // load is one memory round trip
    constexpr int NCL = (EY + 1) * (EX + 1);
    constexpr int CPT = (NCL + 64 * W - 1) / (64 * W);
    T cv[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int t = threadIdx.x + q * 64 * W;
        const int cy = t / (EX + 1), cx = t % (EX + 1);
        const int sy = gy0 + cy, sx = gx0 + cx;
        const bool ok = t < NCL && (unsigned)sy <= (unsigned)ny && (unsigned)sx <= (unsigned)nx;
        cv[q] = ok ? m[(int64_t)sy * (nx + 1) + sx] : T(0);
    }
    T uprev[R], d[R], fr[R], fi[R], uc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = wv * R + i;
        const int gy = gy0 + r;
        const bool in = xin && (unsigned)gy < (unsigned)ny;
        const int64_t g = (int64_t)gy * nx + gx;
        uc[i] = uprev[i] = d[i] = fr[i] = fi[i] = T(0);
        if (in) {
            uc[i] = u_in[g];
            uprev[i] = up_in[g];
            d[i] = dn[g];
            const auto f = F[g];
            fr[i] = f.x;
            fi[i] = f.y;
        }
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int t = threadIdx.x + q * 64 * W;
        if (t < NCL) cl[(t / (EX + 1)) * CS + t % (EX + 1)] = cv[q];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) ul[(wv * R + i + 1) * US + lane + 1] = uc[i];
    __syncthreads();

    T unew[R];
    for (int s = 0; s < k; ++s) {
        const T fas = (T)fa[s * fstride], fbs = (T)fb[s * fstride];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = wv * R + i;
            const T acc = stencil9<SC, MC>(&ul[(r + 1) * US + lane + 1], US, &cl[r * CS + lane],
                                           CS, st);
            unew[i] = d[i] * (acc + fas * fr[i] + fbs * fi[i]) - (T(2) * d[i] - T(1)) * uprev[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = wv * R + i;
            T *p = &ul[(r + 1) * US + lane + 1];
            uprev[i] = *p;
            *p = unew[i];
        }
        // outputs of this step (snapshot of Table 1 / final field): the
        // exact region only
        if (s + 1 == out_step[0] || s + 1 == out_step[1]) {
            double *o = (s + 1 == out_step[0]) ? out[0] : out[1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = wv * R + i;
                const int gy = gy0 + r;
                if (r >= halo && r < EY - halo && lane >= halo && lane < EX - halo && xin &&
                    (unsigned)gy < (unsigned)ny)
                    o[2 * ((int64_t)gy * nx + gx)] = (double)unew[i];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = wv * R + i;
        const int gy = gy0 + r;
        if (r >= halo && r < EY - halo && lane >= halo && lane < EX - halo && xin &&
            (unsigned)gy < (unsigned)ny) {
            const int64_t g = (int64_t)gy * nx + gx;
            u_out[g] = ul[(r + 1) * US + lane + 1];
            up_out[g] = uprev[i];
        }
    }
}

// Second form of the tile update: the cell-mass sums do not change in time,
// so each lane folds them once per launch into per-node stencil coefficients
// held in registers (centre, W, E, S, N; the corners too when they are not
// zero), each already multiplied by the node's damping factor d, so that a
// step is
//   u_{j+1} = sum_q c_q u_j(q) + fa d Re F + fb d Im F + (1 - 2d) u_{j-1}.
// Each wave owns R consecutive tile rows and keeps u_j and u_{j-1} of its
// nodes in registers (u_{j+1} overwrites u_{j-1}; the two arrays swap roles
// every step).  The x-neighbours come from the adjacent lanes by DPP shifts,
// and only the wave's first and last rows go through LDS, where the waves
// above and below read them (two LDS copies, one barrier per step).  No cells
// are kept in LDS.
// After s+1 steps only rows s+1 .. EY-2-s still feed the exact region, so a
// wave whose rows all lie outside that window skips the step (its stale rows
// are never read again).  The exact-region, Dirichlet and output rules are
// those of tb_tile.
// cur[rs - 1 .. rs + 1] and cur[rn - 1 .. rn + 1] hold the halo rows south
// and north of the wave's rows at x-1, x, x+1; the wave's first and last new
// rows go to nxt[wf] and nxt[wl].
template <typename T, int SC, int MC, int R, int NCO>
__device__ __forceinline__ void tb2_step(const T *__restrict__ cur, T *__restrict__ nxt, int rs,
                                         int rn, int wf, int wl, const T (&co)[R][NCO],
                                         const T (&fr)[R], const T (&fi)[R], const T (&e)[R],
                                         const T (&a)[R], T (&b)[R], T fas, T fbs)
{
    constexpr bool CORNER = MC > 2 || SC > 2;
    // rows r0-1 .. r0+R at x-1, x, x+1: the two halo rows from LDS, the own
    // rows from registers and the neighbouring lanes
    T cw[R + 2], cc[R + 2], ce[R + 2];
    cw[0] = cur[rs - 1];
    cc[0] = cur[rs];
    ce[0] = cur[rs + 1];
    cw[R + 1] = cur[rn - 1];
    cc[R + 1] = cur[rn];
    ce[R + 1] = cur[rn + 1];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        cc[i + 1] = a[i];
        cw[i + 1] = lane_west(a[i]);
        ce[i + 1] = lane_east(a[i]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        // node row r0+i: centre cc[i+1], S cc[i], N cc[i+2]
        T acc = co[i][0] * cc[i + 1];
        acc += co[i][1] * cw[i + 1];
        acc += co[i][2] * ce[i + 1];
        acc += co[i][3] * cc[i];
        acc += co[i][4] * cc[i + 2];
        if (MC > 2) {
            acc += co[i][5] * cw[i];
            acc += co[i][6] * ce[i];
            acc += co[i][7] * cw[i + 2];
            acc += co[i][8] * ce[i + 2];
        } else if (CORNER) {
            acc += co[i][5] * ((cw[i] + ce[i]) + (cw[i + 2] + ce[i + 2]));
        }
        acc += fas * fr[i];
        acc += fbs * fi[i];
        b[i] = acc + e[i] * b[i];
    }
    // the wave's first and last rows for its neighbours' next step
    nxt[wf] = b[0];
    nxt[wl] = b[R - 1];
}

template <typename T, int SC, int MC, int R, int W>
__device__ __forceinline__ void tb_tile2(T *__restrict__ ul, const T *__restrict__ u_in,
                                         const T *__restrict__ up_in, T *__restrict__ u_out,
                                         T *__restrict__ up_out, const T *__restrict__ m,
                                         const T *__restrict__ dn,
                                         const typename V2t<T>::type *__restrict__ F, int ny,
                                         int nx, const Stencil<T> &st, int k, int halo, int gy0,
                                         int gx0, const double *fa, const double *fb,
                                         int fstride, const int *out_step, double *const *out)
{
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;
    constexpr int UB = (EY + 2) * US;
    constexpr int NCO = MC > 2 ? 9 : (SC > 2 ? 6 : 5);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;

    // per-node coefficients from the cells around each node (storage rows
    // gy0+r0 .. gy0+r0+R, columns gx and gx+1), times d
    T co[R][NCO];
    T fr[R], fi[R], e[R];
    T u0[R], u1[R];   // u_j and u_{j-1} of the wave's nodes
    {
        T ca[R + 1], cb[R + 1], d[R];
        // row offsets are wave-uniform (scalar); only the column is per lane
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const T *mrow = m + (int64_t)sy * (nx + 1);
            ca[i] = (rok && (unsigned)gx <= (unsigned)nx) ? mrow[gx] : T(0);
            cb[i] = (rok && (unsigned)(gx + 1) <= (unsigned)nx) ? mrow[gx + 1] : T(0);
        }
        // the node data of all R rows are requested before any of it is used,
        // so the tile load is a single memory round trip
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = gy0 + r0 + i;
            const bool in = xin && (unsigned)gy < (unsigned)ny;
            const int64_t row = (int64_t)gy * nx;
            u0[i] = u1[i] = d[i] = fr[i] = fi[i] = T(0);
            if (in) {
                u0[i] = (u_in + row)[gx];
                u1[i] = (up_in + row)[gx];
                d[i] = (dn + row)[gx];
                const auto f = (F + row)[gx];
                fr[i] = f.x;
                fi[i] = f.y;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            fold_node<T, SC, MC, NCO>(st, d[i], ca[i], cb[i], ca[i + 1], cb[i + 1], co[i]);
            fr[i] *= d[i];
            fi[i] *= d[i];
            e[i] = T(1) - T(2) * d[i];
        }
    }
    // LDS copy c holds, at row r+1, tile row r of level c (mod 2) for the
    // first and last row of every wave; row 0, row EY+1 and the first and
    // last column of both copies are the zero pad
    for (int t = threadIdx.x; t < US; t += 64 * W) {
        ul[t] = ul[UB + t] = T(0);
        ul[(EY + 1) * US + t] = ul[UB + (EY + 1) * US + t] = T(0);
    }
    for (int t = threadIdx.x; t < EY + 2; t += 64 * W) {
        ul[t * US] = ul[UB + t * US] = T(0);
        ul[t * US + EX + 1] = ul[UB + t * US + EX + 1] = T(0);
    }
    ul[(r0 + 1) * US + lane + 1] = u0[0];
    ul[(r0 + R) * US + lane + 1] = u0[R - 1];
    __syncthreads();

    // LDS offsets of the halo rows r0-1 (south) and r0+R (north) at column x
    const int rs = r0 * US + lane + 1, rn = (r0 + R + 1) * US + lane + 1;
    const bool xout = lane >= halo && lane < EX - halo && xin;
    auto snapshot = [&](int s, const T(&v)[R]) {
        if (s + 1 == out_step[0] || s + 1 == out_step[1]) {
            double *o = (s + 1 == out_step[0]) ? out[0] : out[1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i;
                const int gy = gy0 + r;
                if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout)
                    (o + 2 * (int64_t)gy * nx)[2 * gx] = (double)v[i];
            }
        }
    };
    // rows whose new value is still read by a later step or written out
    auto active = [&](int s) { return r0 + R > s + 1 && r0 < EY - 1 - s; };
    // two steps (the register arrays swap roles); false once k is reached
    auto step_pair = [&](int s) -> bool {
        if (active(s)) {
            tb2_step<T, SC, MC, R, NCO>(ul, ul + UB, rs, rn, rs + US, rn - US, co, fr, fi, e, u0,
                                        u1, (T)fa[s * fstride], (T)fb[s * fstride]);
            snapshot(s, u1);
        }
        __syncthreads();
        if (s + 1 == k) return false;
        if (active(s + 1)) {
            tb2_step<T, SC, MC, R, NCO>(ul + UB, ul, rs, rn, rs + US, rn - US, co, fr, fi, e, u1,
                                        u0, (T)fa[(s + 1) * fstride], (T)fb[(s + 1) * fstride]);
            snapshot(s + 1, u0);
        }
        __syncthreads();
        return s + 2 < k;
    };
    if constexpr (MC > 2) {
        for (int s = 0; step_pair(s); s += 2) {
        }
    } else {
        // unrolled up to the deepest depth: the scalar bookkeeping and the
        // forcing scalars leave the step loop (5% of a depth-8 launch); the
        // tables with corner mass terms would spill registers unrolled
#pragma unroll
        for (int s = 0; s < TDP_TB_KMAX; s += 2)
            if (!step_pair(s)) break;
    }
    // every output row lies in a wave that ran every step: level k is in u1
    // for odd k, in u0 for even k
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = r0 + i;
        const int gy = gy0 + r;
        if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout) {
            const int64_t row = (int64_t)gy * nx;
            (u_out + row)[gx] = (k & 1) ? u1[i] : u0[i];
            (up_out + row)[gx] = (k & 1) ? u0[i] : u1[i];
        }
    }
}

// Fourth form, for taller tiles (tables without corner mass terms): the
// stencil weights are kept without the damping factor d, and d is applied
// once per update,
//   u_{j+1} = d (sum_q w_q u_j(q) + fa Re F + fb Im F - 2 u_{j-1}) + u_{j-1},
// which needs no 1 - 2d factor and lets neighbouring nodes share weights: the
// weight of the edge between rows i and i+1 of a column is stored once
// (R + 1 per lane), the corner weight is one uniform constant, and F lives
// in LDS (read once per node-update).  The step walks a rolling window of
// three rows and the edge rows use packed slots (as in tb_tile_mrhs).
// Per-node register state drops from 11 to about 7 words, so 5 or 6 rows per
// lane fit the budget of two workgroups per CU in FP64: more work per
// barrier, a smaller share of halo rows and fewer workgroups per launch.
template <typename T, int SC, int R>
__device__ __forceinline__ void tb4_step(const T *__restrict__ cur, T *__restrict__ nxt, int rs,
                                         int rn, int wf, int wl,
                                         const typename V2t<T>::type *__restrict__ fl,
                                         const T (&wc)[R], const T (&ww)[R], const T (&we)[R],
                                         const T (&wy)[R + 1], const T (&d)[R], T s2,
                                         const T (&a)[R], T (&b)[R], T fas, T fbs)
{
    // rows i-1 (p), i (c), i+1 (x) at x-1, x, x+1
    T pc = cur[rs];
    T pp = cur[rs - 1] + cur[rs + 1];
    T cw = lane_west(a[0]), cc = a[0], ce = lane_east(a[0]);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        T xw, xc, xe;
        if (i + 1 < R) {
            xc = a[i + 1];
            xw = lane_west(xc);
            xe = lane_east(xc);
        } else {
            xw = cur[rn - 1];
            xc = cur[rn];
            xe = cur[rn + 1];
        }
        const T xp = xw + xe;
        const auto f = fl[i * 64];
        T acc = wc[i] * cc;
        acc += ww[i] * cw;
        acc += we[i] * ce;
        acc += wy[i] * pc;
        acc += wy[i + 1] * xc;
        if (SC > 2) acc += s2 * (pp + xp);
        acc += fas * f.x;
        acc += fbs * f.y;
        acc += T(-2) * b[i];
        b[i] = d[i] * acc + b[i];
        pc = cc;
        pp = cw + ce;
        cw = xw;
        cc = xc;
        ce = xe;
    }
    nxt[wf] = b[0];
    nxt[wl] = b[R - 1];
}

template <typename T, int SC, int R, int W>
__device__ __forceinline__ void tb_tile4(T *__restrict__ xl, const T *__restrict__ u_in,
                                         const T *__restrict__ up_in, T *__restrict__ u_out,
                                         T *__restrict__ up_out, const T *__restrict__ m,
                                         const T *__restrict__ dn,
                                         const typename V2t<T>::type *__restrict__ F, int ny,
                                         int nx, const Stencil<T> &st, int k, int halo, int gy0,
                                         int gx0, const double *fa, const double *fb,
                                         const int *out_step, double *const *out)
{
    using V2 = typename V2t<T>::type;
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;
    constexpr int CB = (2 * W + 2) * US;
    V2 *fl_all = (V2 *)(xl + 2 * CB);      // F of the tile, [EY][64]
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;

    // weights from the four cells around each node (stiffness + cell mass);
    // zero with d at nodes outside the domain, which then stay 0
    T wc[R], ww[R], we[R], wy[R + 1], d[R];
    T u0[R], u1[R];
    {
        T ca[R + 1], cb[R + 1];
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const T *mrow = m + (int64_t)sy * (nx + 1);
            ca[i] = (rok && (unsigned)gx <= (unsigned)nx) ? mrow[gx] : T(0);
            cb[i] = (rok && (unsigned)(gx + 1) <= (unsigned)nx) ? mrow[gx + 1] : T(0);
        }
        // every row's loads are issued before F goes to LDS: storing a row as
        // soon as it is loaded would cost one memory round trip per row
        V2 f[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = gy0 + r0 + i;
            const bool in = xin && (unsigned)gy < (unsigned)ny;
            const int64_t row = (int64_t)gy * nx;
            u0[i] = u1[i] = d[i] = T(0);
            f[i].x = f[i].y = T(0);
            if (in) {
                u0[i] = (u_in + row)[gx];
                u1[i] = (up_in + row)[gx];
                d[i] = (dn + row)[gx];
                f[i] = (F + row)[gx];
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) fl_all[(r0 + i) * 64 + lane] = f[i];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const T mSW = ca[i], mSE = cb[i], mNW = ca[i + 1], mNE = cb[i + 1];
            wc[i] = st.c0 + st.m[0] * ((mSW + mSE) + (mNW + mNE));
            ww[i] = st.s[1] + st.m[1] * (mSW + mNW);
            we[i] = st.s[1] + st.m[1] * (mSE + mNE);
        }
#pragma unroll
        for (int i = 0; i <= R; ++i) wy[i] = st.s[1] + st.m[1] * (ca[i] + cb[i]);
    }
    const T s2 = st.s[2];
    for (int t = threadIdx.x; t < 2 * CB; t += 64 * W) xl[t] = T(0);
    __syncthreads();
    const int rs = 2 * wv * US + lane + 1, rn = (2 * wv + 3) * US + lane + 1;
    const int wf = (2 * wv + 1) * US + lane + 1, wl = (2 * wv + 2) * US + lane + 1;
    xl[wf] = u0[0];
    xl[wl] = u0[R - 1];
    __syncthreads();

    const V2 *fl = fl_all + r0 * 64 + lane;
    const bool xout = lane >= halo && lane < EX - halo && xin;
    auto snapshot = [&](int s, const T(&v)[R]) {
        if (s + 1 == out_step[0] || s + 1 == out_step[1]) {
            double *o = (s + 1 == out_step[0]) ? out[0] : out[1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i;
                const int gy = gy0 + r;
                if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout)
                    (o + 2 * (int64_t)gy * nx)[2 * gx] = (double)v[i];
            }
        }
    };
    auto active = [&](int s) { return r0 + R > s + 1 && r0 < EY - 1 - s; };
    T *c0 = xl, *c1 = xl + CB;
    auto step_pair = [&](int s) -> bool {
        if (active(s)) {
            tb4_step<T, SC, R>(c0, c1, rs, rn, wf, wl, fl, wc, ww, we, wy, d, s2, u0, u1,
                               (T)fa[s], (T)fb[s]);
            snapshot(s, u1);
        }
        __syncthreads();
        if (s + 1 == k) return false;
        if (active(s + 1)) {
            tb4_step<T, SC, R>(c1, c0, rs, rn, wf, wl, fl, wc, ww, we, wy, d, s2, u1, u0,
                               (T)fa[s + 1], (T)fb[s + 1]);
            snapshot(s + 1, u0);
        }
        __syncthreads();
        return s + 2 < k;
    };
#pragma unroll
    for (int s = 0; s < TDP_TB_KMAX; s += 2)
        if (!step_pair(s)) break;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = r0 + i;
        const int gy = gy0 + r;
        if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout) {
            const int64_t row = (int64_t)gy * nx;
            (u_out + row)[gx] = (k & 1) ? u1[i] : u0[i];
            (up_out + row)[gx] = (k & 1) ? u0[i] : u1[i];
        }
    }
}

template <typename T, int SC, int R, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4)))
void k_sweep2d_tb4(
    const T *__restrict__ u_in, const T *__restrict__ up_in, T *__restrict__ u_out,
    T *__restrict__ up_out, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2t<T>::type *__restrict__ F, int ny, int nx, Stencil<T> st, TBCoef cf,
    int tiles_x, int ntiles, int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    // two packed copies of the edge rows, then F of the tile (2 words per node)
    __shared__ T xl[2 * (2 * W + 2) * (EX + 2) + 2 * EY * EX];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int k = cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    tb_tile4<T, SC, R, W>(xl, u_in, up_in, u_out, up_out, m, dn, F, ny, nx, st, k, k,
                          ty * OY - k, tx * OX - k, cf.fa, cf.fb, cf.out_step, cf.out);
}

// Third form: each lane holds two adjacent columns (x = 2 lane, 2 lane + 1),
// so a wave spans 128 columns.  Against one column per lane this halves the
// share of columns lost to the halo at a given depth and the DPP moves per
// node (the inner x-neighbours of the pair are the lane's own values; only
// the outer ones cross lanes).  Coefficients, the exact region, the skipped
// waves and the outputs follow tb_tile2.  Each wave passes its first and
// last rows through LDS in packed slots (2W + 2 rows per copy; wave w writes
// slots 2w + 1 and 2w + 2 and reads slots 2w and 2w + 3, slots 0 and 2W + 1
// stay zero); a slot holds columns -2 .. EX + 1 so that the lane's pair is
// one 16-byte access.
template <typename T, int SC, int MC, int R, int NCO>
__device__ __forceinline__ void tb3_step(const T *__restrict__ cur, T *__restrict__ nxt, int rs,
                                         int rn, int wf, int wl, const T (&co)[R][2][NCO],
                                         const T (&fr)[R][2], const T (&fi)[R][2],
                                         const T (&e)[R][2], const T (&a)[R][2],
                                         T (&b)[R][2], T fas, T fbs)
{
    constexpr bool CORNER = MC > 2 || SC > 2;
    // rows r0-1 .. r0+R at columns 2l-1, 2l, 2l+1, 2l+2 (LDS offsets base +
    // 1 .. base + 4 of a slot whose column x sits at x + 2)
    T v[R + 2][4];
    v[0][0] = cur[rs + 1];
    v[0][1] = cur[rs + 2];
    v[0][2] = cur[rs + 3];
    v[0][3] = cur[rs + 4];
    v[R + 1][0] = cur[rn + 1];
    v[R + 1][1] = cur[rn + 2];
    v[R + 1][2] = cur[rn + 3];
    v[R + 1][3] = cur[rn + 4];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        v[i + 1][0] = lane_west(a[i][1]);
        v[i + 1][1] = a[i][0];
        v[i + 1][2] = a[i][1];
        v[i + 1][3] = lane_east(a[i][0]);
    }
    T ps[R + 2][2];     // x-1 + x+1 of each row, shared by the corner terms above and below
    if (!(MC > 2) && CORNER) {
#pragma unroll
        for (int j = 0; j < R + 2; ++j) {
            ps[j][0] = v[j][0] + v[j][2];
            ps[j][1] = v[j][1] + v[j][3];
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T acc = co[i][c][0] * v[i + 1][c + 1];
            acc += co[i][c][1] * v[i + 1][c];
            acc += co[i][c][2] * v[i + 1][c + 2];
            acc += co[i][c][3] * v[i][c + 1];
            acc += co[i][c][4] * v[i + 2][c + 1];
            if (MC > 2) {
                acc += co[i][c][5] * v[i][c];
                acc += co[i][c][6] * v[i][c + 2];
                acc += co[i][c][7] * v[i + 2][c];
                acc += co[i][c][8] * v[i + 2][c + 2];
            } else if (CORNER) {
                acc += co[i][c][5] * (ps[i][c] + ps[i + 2][c]);
            }
            acc += fas * fr[i][c];
            acc += fbs * fi[i][c];
            b[i][c] = acc + e[i][c] * b[i][c];
        }
    }
    nxt[wf] = b[0][0];
    nxt[wf + 1] = b[0][1];
    nxt[wl] = b[R - 1][0];
    nxt[wl + 1] = b[R - 1][1];
}

template <typename T, int SC, int MC, int R, int W>
__device__ __forceinline__ void tb_tile3(T *__restrict__ xl, const T *__restrict__ u_in,
                                         const T *__restrict__ up_in, T *__restrict__ u_out,
                                         T *__restrict__ up_out, const T *__restrict__ m,
                                         const T *__restrict__ dn,
                                         const typename V2t<T>::type *__restrict__ F, int ny,
                                         int nx, const Stencil<T> &st, int k, int halo, int gy0,
                                         int gx0, const double *fa, const double *fb,
                                         const int *out_step, double *const *out)
{
    constexpr int EX = 128, EY = R * W;
    constexpr int US = EX + 4;
    constexpr int CB = (2 * W + 2) * US;
    constexpr int NCO = MC > 2 ? 9 : (SC > 2 ? 6 : 5);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gxl = gx0 + 2 * lane;      // the lane's first column

    T co[R][2][NCO], fr[R][2], fi[R][2], e[R][2];
    T u0[R][2], u1[R][2];
    {
        // cells at storage columns gxl, gxl + 1, gxl + 2 of rows gy0+r0 .. gy0+r0+R
        T cm[R + 1][3], d[R][2];
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const T *mrow = m + (int64_t)sy * (nx + 1);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                cm[i][c] = (rok && (unsigned)(gxl + c) <= (unsigned)nx) ? mrow[gxl + c] : T(0);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = gy0 + r0 + i;
            const int64_t row = (int64_t)gy * nx;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool in = (unsigned)gy < (unsigned)ny && (unsigned)(gxl + c) < (unsigned)nx;
                u0[i][c] = u1[i][c] = d[i][c] = fr[i][c] = fi[i][c] = T(0);
                if (in) {
                    u0[i][c] = (u_in + row)[gxl + c];
                    u1[i][c] = (up_in + row)[gxl + c];
                    d[i][c] = (dn + row)[gxl + c];
                    const auto f = (F + row)[gxl + c];
                    fr[i][c] = f.x;
                    fi[i][c] = f.y;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                fold_node<T, SC, MC, NCO>(st, d[i][c], cm[i][c], cm[i][c + 1], cm[i + 1][c],
                                          cm[i + 1][c + 1], co[i][c]);
                fr[i][c] *= d[i][c];
                fi[i][c] *= d[i][c];
                e[i][c] = T(1) - T(2) * d[i][c];
            }
    }
    for (int t = threadIdx.x; t < 2 * CB; t += 64 * W) xl[t] = T(0);
    __syncthreads();
    const int rs = 2 * wv * US + 2 * lane, rn = (2 * wv + 3) * US + 2 * lane;
    const int wf = (2 * wv + 1) * US + 2 * lane + 2, wl = (2 * wv + 2) * US + 2 * lane + 2;
    xl[wf] = u0[0][0];
    xl[wf + 1] = u0[0][1];
    xl[wl] = u0[R - 1][0];
    xl[wl + 1] = u0[R - 1][1];
    __syncthreads();

    auto xok = [&](int c) {
        const int x = 2 * lane + c;
        return x >= halo && x < EX - halo && (unsigned)(gxl + c) < (unsigned)nx;
    };
    auto snapshot = [&](int s, const T(&v)[R][2]) {
        if (s + 1 == out_step[0] || s + 1 == out_step[1]) {
            double *o = (s + 1 == out_step[0]) ? out[0] : out[1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i;
                const int gy = gy0 + r;
                if (r < halo || r >= EY - halo || (unsigned)gy >= (unsigned)ny) continue;
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (xok(c)) (o + 2 * (int64_t)gy * nx)[2 * (gxl + c)] = (double)v[i][c];
            }
        }
    };
    auto active = [&](int s) { return r0 + R > s + 1 && r0 < EY - 1 - s; };
    T *c0 = xl, *c1 = xl + CB;
    for (int s = 0; s < k; s += 2) {
        if (active(s)) {
            tb3_step<T, SC, MC, R, NCO>(c0, c1, rs, rn, wf, wl, co, fr, fi, e, u0, u1,
                                        (T)fa[s], (T)fb[s]);
            snapshot(s, u1);
        }
        __syncthreads();
        if (s + 1 == k) break;
        if (active(s + 1)) {
            tb3_step<T, SC, MC, R, NCO>(c1, c0, rs, rn, wf, wl, co, fr, fi, e, u1, u0,
                                        (T)fa[s + 1], (T)fb[s + 1]);
            snapshot(s + 1, u0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = r0 + i;
        const int gy = gy0 + r;
        if (r < halo || r >= EY - halo || (unsigned)gy >= (unsigned)ny) continue;
        const int64_t row = (int64_t)gy * nx;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (xok(c)) {
                (u_out + row)[gxl + c] = (k & 1) ? u1[i][c] : u0[i][c];
                (up_out + row)[gxl + c] = (k & 1) ? u0[i][c] : u1[i][c];
            }
    }
}

// 1024-thread workgroups need the 128-VGPR budget of four waves per SIMD;
// 512-thread ones ask for it too when their per-node state (about 11 words
// per node, 2R nodes per lane) leaves room, so that two workgroups share a CU.
template <typename T, int R, int W>
constexpr int tb3_waves_per_eu()
{
    return (W >= 16 || 2 * R * 11 * (int)sizeof(T) / 4 <= 100) ? 4 : 2;
}

template <typename T, int SC, int MC, int R, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(tb3_waves_per_eu<T, R, W>())))
void k_sweep2d_tb3(
    const T *__restrict__ u_in, const T *__restrict__ up_in, T *__restrict__ u_out,
    T *__restrict__ up_out, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2t<T>::type *__restrict__ F, int ny, int nx, Stencil<T> st, TBCoef cf,
    int tiles_x, int ntiles, int per_xcd)
{
    constexpr int EX = 128, EY = R * W;
    __shared__ T xl[2 * (2 * W + 2) * (EX + 4)];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int k = cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    tb_tile3<T, SC, MC, R, W>(xl, u_in, up_in, u_out, up_out, m, dn, F, ny, nx, st, k, k,
                              ty * OY - k, tx * OX - k, cf.fa, cf.fb, cf.out_step, cf.out);
}

// Tiles of 32 rows are sized for two workgroups per CU: ask for the
// 128-VGPR budget that four waves per SIMD allow.
template <typename T, int SC, int MC, int R, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(R * W <= 32 ? 4 : 1)))
void k_sweep2d_tb2(
    const T *__restrict__ u_in, const T *__restrict__ up_in, T *__restrict__ u_out,
    T *__restrict__ up_out, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2t<T>::type *__restrict__ F, int ny, int nx, Stencil<T> st, TBCoef cf,
    int tiles_x, int ntiles, int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    __shared__ T ul[2 * (EY + 2) * (EX + 2)];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int k = cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    tb_tile2<T, SC, MC, R, W>(ul, u_in, up_in, u_out, up_out, m, dn, F, ny, nx, st, k, k,
                              ty * OY - k, tx * OX - k, cf.fa, cf.fb, 1, cf.out_step, cf.out);
}

template <typename T, int SC, int MC, int R, int W>
__global__ __launch_bounds__(64 * W) void k_sweep2d_tb(
    const T *__restrict__ u_in, const T *__restrict__ up_in, T *__restrict__ u_out,
    T *__restrict__ up_out, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2t<T>::type *__restrict__ F, int ny, int nx, Stencil<T> st, TBCoef cf,
    int tiles_x, int ntiles, int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    __shared__ T ul[(EY + 2) * (EX + 2)];
    __shared__ T cl[(EY + 1) * (EX + 1)];
    // XCD-aware tile id
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int k = cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    tb_tile<T, SC, MC, R, W>(ul, cl, u_in, up_in, u_out, up_out, m, dn, F, ny, nx, st, k, k,
                             ty * OY - k, tx * OX - k, cf.fa, cf.fb, 1, cf.out_step, cf.out);
}

// Batched form: one launch advances every field of the work list by up to K
// steps; workgroup -> (field, tile) through the per-launch tile prefix sums.
template <typename T, int SC, int MC, int R, int W, bool V2F>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(R * W <= 32 ? 4 : 1)))
void k_sweep2d_tb_batch(
    const BFieldT<T> *__restrict__ fields, const int *__restrict__ list,
    const int *__restrict__ prefix, int nlist, int j0, int K, int parity, int ntiles,
    int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    __shared__ T ul[(V2F ? 2 : 1) * (EY + 2) * (EX + 2)];
    __shared__ T cl[V2F ? 1 : (EY + 1) * (EX + 1)];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    int lo = 0, hi = nlist;            // prefix[lo] <= tile < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const BFieldT<T> &f = fields[list[lo]];
    const int t = tile - prefix[lo];
    const int OX = EX - 2 * K, OY = EY - 2 * K;
    const int tiles_x = (f.nx + OX - 1) / OX;
    const int ty = t / tiles_x, tx = t % tiles_x;
    const int k = min(K, f.Ns - j0);
    int out_step[2];
    double *out[2] = {f.U + 1, f.U};
    out_step[0] = (f.jsnap > j0 && f.jsnap <= j0 + k) ? f.jsnap - j0 : 0;
    out_step[1] = (f.Ns > j0 && f.Ns <= j0 + k) ? f.Ns - j0 : 0;
    const T *u_in = parity ? f.b0 : f.a0, *up_in = parity ? f.b1 : f.a1;
    T *u_out = parity ? f.a0 : f.b0, *up_out = parity ? f.a1 : f.b1;
    if (V2F)
        tb_tile2<T, SC, MC, R, W>(ul, u_in, up_in, u_out, up_out, f.m, f.dn,
                                  (const typename V2t<T>::type *)f.F, f.ny, f.nx, f.st, k, K,
                                  ty * OY - K, tx * OX - K, f.tab + 2 * j0, f.tab + 2 * j0 + 1,
                                  2, out_step, out);
    else
        tb_tile<T, SC, MC, R, W>(ul, cl, u_in, up_in, u_out, up_out, f.m, f.dn,
                                 (const typename V2t<T>::type *)f.F, f.ny, f.nx, f.st, k, K,
                                 ty * OY - K, tx * OX - K, f.tab + 2 * j0, f.tab + 2 * j0 + 1, 2,
                                 out_step, out);
}

// Shared-medium form of the batched tile: one workgroup advances up to NR
// right-hand sides of one medium over the same extended tile.  The medium's
// per-node coefficients (cell slowness and damping factor) are loaded and
// folded once for all of them; each right-hand side keeps its own u_j,
// u_{j-1} and d-scaled F in registers, and the NR updates of a node are
// independent FMA chains with the same coefficients.  Each wave passes only
// its first and last rows through LDS, packed per right-hand side as 2W + 2
// rows per copy (wave w writes slots 2w + 1 and 2w + 2 and reads slots 2w and
// 2w + 3; slots 0 and 2W + 1 and the end columns are the zero pad).
template <typename T, int SC, int MC, int R, int W, int NR>
__device__ __forceinline__ void tb_tile_mrhs(T *__restrict__ xl, const BFieldT<T> *__restrict__ fields,
                                             const int *__restrict__ slab, int k, int halo,
                                             int gy0, int gx0, int j0, int parity)
{
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;
    constexpr int CB = (2 * W + 2) * US;      // one copy of one right-hand side
    constexpr int NCO = MC > 2 ? 9 : (SC > 2 ? 6 : 5);
    const BFieldT<T> &f0 = fields[slab[0]];
    const int ny = f0.ny, nx = f0.nx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;
    int nr = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) nr += slab[q] >= 0 ? 1 : 0;

    T co[R][NCO], e[R];
    T fr[NR][R], fi[NR][R];
    T u0[NR][R], u1[NR][R];
    {
        T ca[R + 1], cb[R + 1], d[R];
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const T *mrow = f0.m + (int64_t)sy * (nx + 1);
            ca[i] = (rok && (unsigned)gx <= (unsigned)nx) ? mrow[gx] : T(0);
            cb[i] = (rok && (unsigned)(gx + 1) <= (unsigned)nx) ? mrow[gx + 1] : T(0);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = gy0 + r0 + i;
            d[i] = (xin && (unsigned)gy < (unsigned)ny) ? (f0.dn + (int64_t)gy * nx)[gx] : T(0);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const BFieldT<T> &f = fields[slab[q >= nr ? 0 : q]];
            const T *u_in = parity ? f.b0 : f.a0, *up_in = parity ? f.b1 : f.a1;
            const auto *F = (const typename V2t<T>::type *)f.F;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int gy = gy0 + r0 + i;
                const bool in = q < nr && xin && (unsigned)gy < (unsigned)ny;
                const int64_t row = (int64_t)gy * nx;
                u0[q][i] = u1[q][i] = fr[q][i] = fi[q][i] = T(0);
                if (in) {
                    u0[q][i] = (u_in + row)[gx];
                    u1[q][i] = (up_in + row)[gx];
                    const auto fv = (F + row)[gx];
                    fr[q][i] = fv.x;
                    fi[q][i] = fv.y;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            fold_node<T, SC, MC, NCO>(f0.st, d[i], ca[i], cb[i], ca[i + 1], cb[i + 1], co[i]);
            e[i] = T(1) - T(2) * d[i];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                fr[q][i] *= d[i];
                fi[q][i] *= d[i];
            }
        }
    }
    for (int t = threadIdx.x; t < NR * 2 * CB; t += 64 * W) xl[t] = T(0);
    __syncthreads();
    const int rs = 2 * wv * US + lane + 1, rn = (2 * wv + 3) * US + lane + 1;
    const int wf = (2 * wv + 1) * US + lane + 1, wl = (2 * wv + 2) * US + lane + 1;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        xl[2 * q * CB + wf] = u0[q][0];
        xl[2 * q * CB + wl] = u0[q][R - 1];
    }
    __syncthreads();

    const bool xout = lane >= halo && lane < EX - halo && xin;
    const int out_snap = (f0.jsnap > j0 && f0.jsnap <= j0 + k) ? f0.jsnap - j0 : 0;
    const int out_fin = (f0.Ns > j0 && f0.Ns <= j0 + k) ? f0.Ns - j0 : 0;
    auto snapshot = [&](int s, int q, const T(&v)[R]) {
        if (q < nr && (s + 1 == out_snap || s + 1 == out_fin)) {
            double *o = fields[slab[q]].U + (s + 1 == out_snap ? 1 : 0);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i;
                const int gy = gy0 + r;
                if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout)
                    (o + 2 * (int64_t)gy * nx)[2 * gx] = (double)v[i];
            }
        }
    };
    auto active = [&](int s) { return r0 + R > s + 1 && r0 < EY - 1 - s; };
    const double *tab = f0.tab + 2 * j0;
    auto step_pair = [&](int s) -> bool {
        if (active(s)) {
            const T fas = (T)tab[2 * s], fbs = (T)tab[2 * s + 1];
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q < nr) {
                    tb2_step<T, SC, MC, R, NCO>(xl + 2 * q * CB, xl + (2 * q + 1) * CB, rs, rn, wf,
                                                wl, co, fr[q], fi[q], e, u0[q], u1[q], fas, fbs);
                    snapshot(s, q, u1[q]);
                }
        }
        __syncthreads();
        if (s + 1 == k) return false;
        if (active(s + 1)) {
            const T fas = (T)tab[2 * s + 2], fbs = (T)tab[2 * s + 3];
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q < nr) {
                    tb2_step<T, SC, MC, R, NCO>(xl + (2 * q + 1) * CB, xl + 2 * q * CB, rs, rn, wf,
                                                wl, co, fr[q], fi[q], e, u1[q], u0[q], fas, fbs);
                    snapshot(s + 1, q, u0[q]);
                }
        }
        __syncthreads();
        return s + 2 < k;
    };
    if constexpr (MC > 2) {
        for (int s = 0; step_pair(s); s += 2) {
        }
    } else {
#pragma unroll
        for (int s = 0; s < TDP_TB_KMAX; s += 2)
            if (!step_pair(s)) break;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q >= nr) continue;
        const BFieldT<T> &f = fields[slab[q]];
        T *u_out = parity ? f.a0 : f.b0, *up_out = parity ? f.a1 : f.b1;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = r0 + i;
            const int gy = gy0 + r;
            if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout) {
                const int64_t row = (int64_t)gy * nx;
                (u_out + row)[gx] = (k & 1) ? u1[q][i] : u0[q][i];
                (up_out + row)[gx] = (k & 1) ? u0[q][i] : u1[q][i];
            }
        }
    }
}

// One launch advances every slab of the work list by up to K steps:
// workgroup -> (slab, tile) through the per-launch tile prefix sums; a slab
// lists up to NR fields of one medium (-1 past its end).
// Register budget: 1024-thread workgroups need four waves per SIMD (128
// VGPRs); 512-thread ones ask for the same when their per-node state is
// small (two workgroups per CU), else for two waves per SIMD (256 VGPRs).
template <typename T, int R, int W, int NR>
constexpr int mrhs_waves_per_eu()
{
    return (W >= 16 || R * (7 + 4 * NR) * (int)sizeof(T) / 4 <= 100) ? 4 : 2;
}

template <typename T, int SC, int MC, int R, int W, int NR>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(mrhs_waves_per_eu<T, R, W, NR>())))
void k_sweep2d_tb_mrhs(const BFieldT<T> *__restrict__ fields, const int *__restrict__ slabs,
                       const int *__restrict__ prefix, int nslab, int j0, int K, int parity,
                       int ntiles, int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    __shared__ T xl[NR * 2 * (2 * W + 2) * (EX + 2)];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    int lo = 0, hi = nslab;            // prefix[lo] <= tile < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const int *slab = slabs + NR * lo;
    const BFieldT<T> &f = fields[slab[0]];
    const int t = tile - prefix[lo];
    const int OX = EX - 2 * K, OY = EY - 2 * K;
    const int tiles_x = (f.nx + OX - 1) / OX;
    const int ty = t / tiles_x, tx = t % tiles_x;
    const int k = min(K, f.Ns - j0);
    tb_tile_mrhs<T, SC, MC, R, W, NR>(xl, fields, slab, k, K, ty * OY - K, tx * OX - K, j0, parity);
}

// One step of the frequency-adapted backward-differences damped leapfrog
// I_abd (Sec. 6) with the cell damping, blocked like tb_tile2, on one real
// part of the complex field of S_T^abd.  Its recurrence has real coefficients,
//   x_{n+1} = A[x_n] + B[x_{n-1} - cos(theta) x_n] - x_{n-1} + fa Re F + fb Im F,
// with A the I_acd step stencil over the cell slowness and B the damping
// stencil (mass classes only) over the cell damping, so the real and
// imaginary parts of the field are two such recurrences: forcing scalars
// (fa, -fb) and (fb, fa) of the complex forcing (fa + i fb) F.  B reads
// w = x_{n-1} - cos(theta) x_n at the neighbours, so every wave passes the
// first and last rows of both x_n and w through LDS; the x-neighbours of both
// come from DPP.  A step still reaches one node, so the exact region, the
// window of rows a wave must update and the output rules are those of
// tb_tile2.  Mass tables with corner entries are not covered here.
// tb_tile_abd2 below applies it to both parts.
template <typename T, int R, int US>
__device__ __forceinline__ void abd_step(const T *__restrict__ xc, const T *__restrict__ wc,
                                         T *__restrict__ xn, T *__restrict__ wn, int rs, int rn,
                                         const T (&ca)[R][6], const T (&cb)[R][5],
                                         const T (&fr)[R], const T (&fi)[R], T cth,
                                         const T (&a)[R], T (&b)[R], T fas, T fbs)
{
    // x at rows r0-1 .. r0+R and x-1, x, x+1; w at rows r0-1 .. r0+R and x
    T xw[R + 2], xx[R + 2], xe[R + 2], ww[R + 2];
    xw[0] = xc[rs - 1];
    xx[0] = xc[rs];
    xe[0] = xc[rs + 1];
    ww[0] = wc[rs];
    xw[R + 1] = xc[rn - 1];
    xx[R + 1] = xc[rn];
    xe[R + 1] = xc[rn + 1];
    ww[R + 1] = wc[rn];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        xx[i + 1] = a[i];
        xw[i + 1] = lane_west(a[i]);
        xe[i + 1] = lane_east(a[i]);
        ww[i + 1] = b[i] - cth * a[i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        T acc = ca[i][0] * xx[i + 1];
        acc += ca[i][1] * xw[i + 1];
        acc += ca[i][2] * xe[i + 1];
        acc += ca[i][3] * xx[i];
        acc += ca[i][4] * xx[i + 2];
        acc += ca[i][5] * ((xw[i] + xe[i]) + (xw[i + 2] + xe[i + 2]));
        acc += cb[i][0] * ww[i + 1];
        acc += cb[i][1] * lane_west(ww[i + 1]);
        acc += cb[i][2] * lane_east(ww[i + 1]);
        acc += cb[i][3] * ww[i];
        acc += cb[i][4] * ww[i + 2];
        acc += fas * fr[i];
        acc += fbs * fi[i];
        b[i] = acc - b[i];
    }
    // the wave's first and last rows of x_{n+1} and w_{n+1} = x_n - cos(theta) x_{n+1}
    xn[rs + US] = b[0];
    xn[rn - US] = b[R - 1];
    wn[rs + US] = a[0] - cth * b[0];
    wn[rn - US] = a[R - 1] - cth * b[R - 1];
}

// I_abd on both real parts of the complex field of S_T^abd in one launch.
// The two recurrences share A, B and F and differ only in their forcing
// scalars: the real part takes (fa, fb) of the launch's table (the Table 1
// form, fa Re F + fb Im F = Re of the complex forcing) and the imaginary part
// (-fb, fa), which is Im of the same complex forcing.  So one tile loads the
// cells and F and folds A and B once for both, keeps x_n and x_{n-1} of both
// parts in registers, and gives every step two independent updates.  Fields
// are complex (the two parts interleaved).  LDS holds, per part, two copies
// of x and of w; each copy keeps only the wave edge rows, in packed slots:
// wave v's first row at slot 2v+1 and its last at 2v+2, so its south and
// north neighbours (the previous wave's last row, the next wave's first) sit
// at 2v and 2v+3, and slots 0 and 2W+1 are the zero pads of the tile.
template <typename T, int R, int W>
__device__ __forceinline__ void tb_tile_abd2(T *__restrict__ ul,
                                             const typename V2t<T>::type *__restrict__ u_in,
                                             const typename V2t<T>::type *__restrict__ up_in,
                                             typename V2t<T>::type *__restrict__ u_out,
                                             typename V2t<T>::type *__restrict__ up_out,
                                             const T *__restrict__ m, const T *__restrict__ rc,
                                             const typename V2t<T>::type *__restrict__ F, int ny,
                                             int nx, const Stencil<T> &sa, const Stencil<T> &sb,
                                             T cth, int k, int halo, int gy0, int gx0,
                                             const double *fa, const double *fb,
                                             const int *out_step, double *const *out)
{
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;
    constexpr int CB = (2 * W + 2) * US;     // one copy of one part's x or w
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;

    // per-node coefficients of A (over the slowness; centre, W, E, S, N and
    // the corner weight) and B (over the damping; centre, W, E, S, N) from the
    // four cells around each node.  They are zero at nodes outside the domain,
    // which then stay 0 (Dirichlet): I_abd has no damping factor d that would
    // zero their update as in tb_tile2.
    T ca[R][6], cb[R][5];
    T fr[R], fi[R];
    T u0[2][R], u1[2][R];   // x_n and x_{n-1} of the real (0) and imaginary (1) part
    {
        T ma[R + 1], mb[R + 1], ra[R + 1], rb[R + 1];
        T on[R];
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const int64_t row = (int64_t)sy * (nx + 1);
            const bool ok0 = rok && (unsigned)gx <= (unsigned)nx;
            const bool ok1 = rok && (unsigned)(gx + 1) <= (unsigned)nx;
            ma[i] = ok0 ? (m + row)[gx] : T(0);
            mb[i] = ok1 ? (m + row)[gx + 1] : T(0);
            ra[i] = ok0 ? (rc + row)[gx] : T(0);
            rb[i] = ok1 ? (rc + row)[gx + 1] : T(0);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = gy0 + r0 + i;
            const bool in = xin && (unsigned)gy < (unsigned)ny;
            const int64_t row = (int64_t)gy * nx;
            u0[0][i] = u0[1][i] = u1[0][i] = u1[1][i] = fr[i] = fi[i] = T(0);
            on[i] = in ? T(1) : T(0);
            if (in) {
                const auto a = (u_in + row)[gx];
                const auto b = (up_in + row)[gx];
                const auto f = (F + row)[gx];
                u0[0][i] = a.x;
                u0[1][i] = a.y;
                u1[0][i] = b.x;
                u1[1][i] = b.y;
                fr[i] = f.x;
                fi[i] = f.y;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            {
                const T SW = ma[i], SE = mb[i], NW = ma[i + 1], NE = mb[i + 1];
                ca[i][0] = on[i] * (sa.c0 + sa.m[0] * ((SW + SE) + (NW + NE)));
                ca[i][1] = on[i] * (sa.s[1] + sa.m[1] * (SW + NW));
                ca[i][2] = on[i] * (sa.s[1] + sa.m[1] * (SE + NE));
                ca[i][3] = on[i] * (sa.s[1] + sa.m[1] * (SW + SE));
                ca[i][4] = on[i] * (sa.s[1] + sa.m[1] * (NW + NE));
                ca[i][5] = on[i] * sa.s[2];
            }
            {
                const T SW = ra[i], SE = rb[i], NW = ra[i + 1], NE = rb[i + 1];
                cb[i][0] = on[i] * (sb.c0 + sb.m[0] * ((SW + SE) + (NW + NE)));
                cb[i][1] = on[i] * sb.m[1] * (SW + NW);
                cb[i][2] = on[i] * sb.m[1] * (SE + NE);
                cb[i][3] = on[i] * sb.m[1] * (SW + SE);
                cb[i][4] = on[i] * sb.m[1] * (NW + NE);
            }
        }
    }
    // copies per part p: x0 at (4p)CB, x1 at (4p+1)CB, w0 at (4p+2)CB, w1 at (4p+3)CB
    for (int t = threadIdx.x; t < 8 * CB; t += 64 * W) ul[t] = T(0);
    __syncthreads();
    const int rs = 2 * wv * US + lane + 1, rn = (2 * wv + 3) * US + lane + 1;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        ul[4 * p * CB + rs + US] = u0[p][0];
        ul[4 * p * CB + rn - US] = u0[p][R - 1];
        ul[(4 * p + 2) * CB + rs + US] = u1[p][0] - cth * u0[p][0];
        ul[(4 * p + 2) * CB + rn - US] = u1[p][R - 1] - cth * u0[p][R - 1];
    }
    __syncthreads();

    const bool xout = lane >= halo && lane < EX - halo && xin;
    // complex outputs: both parts of a node in one 16-byte (8-byte) store
    auto snapshot = [&](int s, const T(&v0)[R], const T(&v1)[R]) {
        if (s + 1 == out_step[0] || s + 1 == out_step[1]) {
            double *o = (s + 1 == out_step[0]) ? out[0] : out[1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i;
                const int gy = gy0 + r;
                if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout)
                    ((double2 *)o)[(int64_t)gy * nx + gx] = make_double2((double)v0[i], (double)v1[i]);
            }
        }
    };
    auto active = [&](int s) { return r0 + R > s + 1 && r0 < EY - 1 - s; };
    for (int s = 0; s < k; s += 2) {
        if (active(s)) {
            const T fa0 = (T)fa[s], fb0 = (T)fb[s];
#pragma unroll
            for (int p = 0; p < 2; ++p)
                abd_step<T, R, US>(ul + 4 * p * CB, ul + (4 * p + 2) * CB, ul + (4 * p + 1) * CB,
                                   ul + (4 * p + 3) * CB, rs, rn, ca, cb, fr, fi, cth, u0[p], u1[p],
                                   p ? -fb0 : fa0, p ? fa0 : fb0);
            snapshot(s, u1[0], u1[1]);
        }
        __syncthreads();
        if (s + 1 == k) break;
        if (active(s + 1)) {
            const T fa0 = (T)fa[s + 1], fb0 = (T)fb[s + 1];
#pragma unroll
            for (int p = 0; p < 2; ++p)
                abd_step<T, R, US>(ul + (4 * p + 1) * CB, ul + (4 * p + 3) * CB, ul + 4 * p * CB,
                                   ul + (4 * p + 2) * CB, rs, rn, ca, cb, fr, fi, cth, u1[p], u0[p],
                                   p ? -fb0 : fa0, p ? fa0 : fb0);
            snapshot(s + 1, u0[0], u0[1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = r0 + i;
        const int gy = gy0 + r;
        if (r >= halo && r < EY - halo && (unsigned)gy < (unsigned)ny && xout) {
            const int64_t row = (int64_t)gy * nx;
            typename V2t<T>::type a, b;
            a.x = (k & 1) ? u1[0][i] : u0[0][i];
            a.y = (k & 1) ? u1[1][i] : u0[1][i];
            b.x = (k & 1) ? u0[0][i] : u1[0][i];
            b.y = (k & 1) ? u0[1][i] : u1[1][i];
            (u_out + row)[gx] = a;
            (up_out + row)[gx] = b;
        }
    }
}

template <typename T, int R, int W>
__global__ __launch_bounds__(64 * W) void k_sweep2d_abd_tb2(
    const typename V2t<T>::type *__restrict__ u_in, const typename V2t<T>::type *__restrict__ up_in,
    typename V2t<T>::type *__restrict__ u_out, typename V2t<T>::type *__restrict__ up_out,
    const T *__restrict__ m, const T *__restrict__ rc, const typename V2t<T>::type *__restrict__ F,
    int ny, int nx, Stencil<T> sa, Stencil<T> sb, T cth, TBCoef cf, int tiles_x, int ntiles,
    int per_xcd)
{
    constexpr int EX = 64, EY = R * W;
    __shared__ T ul[8 * (2 * W + 2) * (EX + 2)];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int k = cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    tb_tile_abd2<T, R, W>(ul, u_in, up_in, u_out, up_out, m, rc, F, ny, nx, sa, sb, cth, k, k,
                          ty * OY - k, tx * OX - k, cf.fa, cf.fb, cf.out_step, cf.out);
}

template <typename T, int R, int W>
static hipError_t launch_abd_tb2_t(const TBArgs &a, const Stencil<T> &sa, const Stencil<T> &sb,
                                   hipStream_t s)
{
    using V2 = typename V2t<T>::type;
    constexpr int EX = 64, EY = R * W;
    const int k = a.cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    if (k < 1 || k > TDP_TB_KMAX || OX < 1 || OY < 1) return hipErrorInvalidValue;
    const int tiles_x = (a.nx + OX - 1) / OX, tiles_y = (a.ny + OY - 1) / OY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL((k_sweep2d_abd_tb2<T, R, W>), dim3(8 * per_xcd), dim3(64 * W), 0, s,
                       (const V2 *)a.u_in, (const V2 *)a.up_in, (V2 *)a.u_out, (V2 *)a.up_out,
                       (const T *)a.m, (const T *)a.rc, (const V2 *)a.F, a.ny, a.nx, sa, sb,
                       (T)a.cth, a.cf, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_tb2_t(const TBArgs &a, const Stencil<T> &st, hipStream_t s)
{
    constexpr int EX = 64, EY = R * W;
    const int k = a.cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int tiles_x = (a.nx + OX - 1) / OX, tiles_y = (a.ny + OY - 1) / OY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const T *u = (const T *)a.u_in, *up = (const T *)a.up_in;
    T *uo = (T *)a.u_out, *upo = (T *)a.up_out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2t<T>::type *)a.F;
    if (a.sc <= 3 && a.mc <= 2)
        hipLaunchKernelGGL((k_sweep2d_tb2<T, 3, 2, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn,
                           F, a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_sweep2d_tb2<T, 3, 3, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn,
                           F, a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_tb4_t(const TBArgs &a, const Stencil<T> &st, hipStream_t s)
{
    constexpr int EX = 64, EY = R * W;
    const int k = a.cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    if (k < 1 || k > TDP_TB_KMAX || OX < 1 || OY < 1) return hipErrorInvalidValue;
    const int tiles_x = (a.nx + OX - 1) / OX, tiles_y = (a.ny + OY - 1) / OY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const T *u = (const T *)a.u_in, *up = (const T *)a.up_in;
    T *uo = (T *)a.u_out, *upo = (T *)a.up_out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2t<T>::type *)a.F;
    if (a.mc > 2) return hipErrorInvalidValue;     // corner mass terms: per-cell corner weights
    if (a.sc > 2)
        hipLaunchKernelGGL((k_sweep2d_tb4<T, 3, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn, F,
                           a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_sweep2d_tb4<T, 2, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn, F,
                           a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_tb3_t(const TBArgs &a, const Stencil<T> &st, hipStream_t s)
{
    constexpr int EX = 128, EY = R * W;
    const int k = a.cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    if (k < 1 || k > TDP_TB_KMAX || OY < 1) return hipErrorInvalidValue;
    const int tiles_x = (a.nx + OX - 1) / OX, tiles_y = (a.ny + OY - 1) / OY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const T *u = (const T *)a.u_in, *up = (const T *)a.up_in;
    T *uo = (T *)a.u_out, *upo = (T *)a.up_out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2t<T>::type *)a.F;
    if (a.sc <= 3 && a.mc <= 2)
        hipLaunchKernelGGL((k_sweep2d_tb3<T, 3, 2, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn,
                           F, a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_sweep2d_tb3<T, 3, 3, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn,
                           F, a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_tb_t(const TBArgs &a, const Stencil<T> &st, hipStream_t s)
{
    constexpr int EX = 64, EY = R * W;
    const int k = a.cf.k;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int tiles_x = (a.nx + OX - 1) / OX, tiles_y = (a.ny + OY - 1) / OY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const T *u = (const T *)a.u_in, *up = (const T *)a.up_in;
    T *uo = (T *)a.u_out, *upo = (T *)a.up_out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2t<T>::type *)a.F;
    if (a.sc <= 3 && a.mc <= 2)
        hipLaunchKernelGGL((k_sweep2d_tb<T, 3, 2, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn, F,
                           a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_sweep2d_tb<T, 3, 3, R, W>), grd, blk, 0, s, u, up, uo, upo, m, dn, F,
                           a.ny, a.nx, st, a.cf, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_tb_batch_t(const TBBatchLaunch &L, hipStream_t s)
{
    const int per_xcd = (L.ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const BFieldT<T> *f = (const BFieldT<T> *)L.fields;
    const bool v2 = L.shape >= 4;
#define TDP_BL(SC, MC, V) \
    hipLaunchKernelGGL((k_sweep2d_tb_batch<T, SC, MC, R, W, V>), grd, blk, 0, s, f, L.list, \
                       L.prefix, L.nlist, L.j0, L.K, L.parity, L.ntiles, per_xcd)
    if (L.general) {
        if (v2) TDP_BL(3, 3, true);
        else TDP_BL(3, 3, false);
    } else {
        if (v2) TDP_BL(3, 2, true);
        else TDP_BL(3, 2, false);
    }
#undef TDP_BL
    return hipGetLastError();
}

// Start of a batched application: every listed field's recurrence fields
// are zeroed and (FP32) its right-hand side is rounded to the staged copy,
// one launch for all fields (block y is the list entry).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_stage_in(const BFieldT<T> *__restrict__ fields,
                                                        const int *__restrict__ list)
{
    const BFieldT<T> &f = fields[list[blockIdx.y]];
    const int64_t N = (int64_t)f.ny * f.nx;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (sizeof(T) == 4) {
            const double2 v = ((const double2 *)f.Fin)[i];
            ((float2 *)f.F)[i] = make_float2((float)v.x, (float)v.y);
        }
        f.a0[i] = T(0);
        f.a1[i] = T(0);
    }
}

hipError_t launch_batch_stage_in(const void *fields, const int *list, int n, int64_t n_max,
                                 bool f64, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > 65535) return hipErrorInvalidValue;
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>((n_max + 255) / 256, 1), 2048);
    if (f64)
        hipLaunchKernelGGL(k_batch_stage_in<double>, dim3(blocks, n), dim3(256), 0, s,
                           (const BFieldT<double> *)fields, list);
    else
        hipLaunchKernelGGL(k_batch_stage_in<float>, dim3(blocks, n), dim3(256), 0, s,
                           (const BFieldT<float> *)fields, list);
    return hipGetLastError();
}

hipError_t launch_sweep2d_tb_batch(const TBBatchLaunch &L, bool f64, hipStream_t s)
{
    if (f64) {
        switch (L.shape) {
        case 1: case 4: return launch_tb_batch_t<double, 4, 16>(L, s);
        case 3: case 5: return launch_tb_batch_t<double, 4, 8>(L, s);
        case 7: return launch_tb_batch_t<double, 2, 16>(L, s);
        case 2: case 8: return hipErrorInvalidValue;  // FP32-only shapes
        default: return launch_tb_batch_t<double, 8, 8>(L, s);
        }
    }
    switch (L.shape) {
    case 1: case 4: return launch_tb_batch_t<float, 4, 16>(L, s);
    case 2: return launch_tb_batch_t<float, 8, 16>(L, s);
    case 3: case 5: return launch_tb_batch_t<float, 4, 8>(L, s);
    case 7: return launch_tb_batch_t<float, 2, 16>(L, s);
    case 8: return launch_tb_batch_t<float, 8, 16>(L, s);
    default: return launch_tb_batch_t<float, 8, 8>(L, s);
    }
}

template <typename T, int R, int W, int NR>
static hipError_t launch_tb_mrhs_t(const TBMrhsLaunch &L, hipStream_t s)
{
    const int per_xcd = (L.ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * W);
    const BFieldT<T> *f = (const BFieldT<T> *)L.fields;
    if (L.general)
        hipLaunchKernelGGL((k_sweep2d_tb_mrhs<T, 3, 3, R, W, NR>), grd, blk, 0, s, f, L.slabs,
                           L.prefix, L.nslab, L.j0, L.K, L.parity, L.ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_sweep2d_tb_mrhs<T, 3, 2, R, W, NR>), grd, blk, 0, s, f, L.slabs,
                           L.prefix, L.nslab, L.j0, L.K, L.parity, L.ntiles, per_xcd);
    return hipGetLastError();
}

// Shared-medium tiles (rows per lane R x waves W, right-hand sides per
// workgroup NR; 64 columns):
//   FP32  0: 4 x 8, NR 4 (32 x 64)    1: 6 x 8, NR 2 (48 x 64)     2: 8 x 8, NR 2 (64 x 64)
//   FP64  0: 2 x 16, NR 3 (32 x 64)   1: 4 x 8, NR 2 (32 x 64)     2: 2 x 16, NR 2 (32 x 64)
hipError_t launch_sweep2d_tb_mrhs(const TBMrhsLaunch &L, bool f64, hipStream_t s)
{
    if (f64) {
        switch (L.shape) {
        case 0: return launch_tb_mrhs_t<double, 2, 16, 3>(L, s);
        case 1: return launch_tb_mrhs_t<double, 4, 8, 2>(L, s);
        case 2: return launch_tb_mrhs_t<double, 2, 16, 2>(L, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (L.shape) {
    case 0: return launch_tb_mrhs_t<float, 4, 8, 4>(L, s);
    case 1: return launch_tb_mrhs_t<float, 6, 8, 2>(L, s);
    case 2: return launch_tb_mrhs_t<float, 8, 8, 2>(L, s);
    default: return hipErrorInvalidValue;
    }
}

int mrhs_nr(int shape, bool f64)
{
    static const int nr32[3] = {4, 2, 2}, nr64[3] = {3, 2, 2};
    return (shape < 0 || shape > 2) ? 0 : (f64 ? nr64[shape] : nr32[shape]);
}

int mrhs_rows(int shape, bool f64)
{
    static const int r32[3] = {32, 48, 64}, r64[3] = {32, 32, 32};
    return (shape < 0 || shape > 2) ? 0 : (f64 ? r64[shape] : r32[shape]);
}

int tb2d_tiles(int shape, int K, int ny, int nx)
{
    const int EY = tb2d_tile_rows(shape, true), EX = 64;
    const int OX = EX - 2 * K, OY = EY - 2 * K;
    return ((nx + OX - 1) / OX) * ((ny + OY - 1) / OY);
}

// Tile shapes (rows per lane R x waves W; the tile is 64 columns wide).
// Shapes 0..3 use tb_tile (cells in LDS), 4..7 tb_tile2 (coefficients in
// registers, column reuse):
//   0: 8 x 8  -> 64 x 64, 512 threads     4: 4 x 16 -> 64 x 64, 1024 threads
//   1: 4 x 16 -> 64 x 64, 1024 threads    5: 4 x 8  -> 32 x 64, 512 threads
//   2: 8 x 16 -> 128 x 64 (FP32 only)     6: 8 x 8  -> 64 x 64, 512 threads
//   3: 4 x 8  -> 32 x 64, 512 threads     7: 2 x 16 -> 32 x 64, 1024 threads
//   8: 8 x 16 -> 128 x 64 with per-node coefficients (FP32 only)
// Shapes 9..13 use tb_tile3 (two columns per lane, 128 columns):
//   9: 2 x 16 -> 32 x 128, 1024 threads   10: 4 x 8 -> 32 x 128, 512 threads
//  11: 2 x 8  -> 16 x 128, 512 threads    12: 4 x 16 -> 64 x 128 (FP32 only)
//  13: 8 x 8  -> 64 x 128 (FP32 only)
// Shapes 14..15 use tb_tile4 (weights without d, F in LDS, rolling row
// window; tables without corner mass terms):
//  14: 5 x 8  -> 40 x 64, 512 threads    15: 6 x 8 -> 48 x 64, 512 threads
int tb2d_tile_rows(int shape, bool f64)
{
    (void)f64;
    switch (shape) {
    case 2: case 8: return 128;
    case 3: case 5: case 7: case 9: case 10: return 32;
    case 11: return 16;
    case 14: return 40;
    case 15: return 48;
    default: return 64;
    }
}

int tb2d_tile_cols(int shape) { return shape >= 9 && shape <= 13 ? 128 : 64; }

bool abd_tile_ok(int shape, bool f64)
{
    return f64 ? (shape == 5 || shape == 7) : (shape >= 4 && shape <= 7);
}

hipError_t launch_sweep2d_tb_f64(const TBArgs &a, const Stencil<double> &st, hipStream_t s)
{
    switch (a.shape) {
    case 1: return launch_tb_t<double, 4, 16>(a, st, s);
    case 3: return launch_tb_t<double, 4, 8>(a, st, s);
    case 4: return launch_tb2_t<double, 4, 16>(a, st, s);
    case 5: return launch_tb2_t<double, 4, 8>(a, st, s);
    case 6: return launch_tb2_t<double, 8, 8>(a, st, s);
    case 7: return launch_tb2_t<double, 2, 16>(a, st, s);
    case 9: return launch_tb3_t<double, 2, 16>(a, st, s);
    case 10: return launch_tb3_t<double, 4, 8>(a, st, s);
    case 11: return launch_tb3_t<double, 2, 8>(a, st, s);
    case 14: return launch_tb4_t<double, 5, 8>(a, st, s);
    case 15: return launch_tb4_t<double, 6, 8>(a, st, s);
    case 2: case 8: case 12: case 13: return hipErrorInvalidValue;     // FP32-only shapes
    default: return launch_tb_t<double, 8, 8>(a, st, s);
    }
}

// I_abd on both parts of a complex field: shapes 4..7 as for tb_tile2 in
// FP32, 5 and 7 in FP64 (its 17 words of per-node state do not fit the
// register file in the others); mass tables with corner entries are refused
// (the one-step kernel runs them)
hipError_t launch_sweep2d_abd2_tb_f64(const TBArgs &a, const Stencil<double> &sa,
                                      const Stencil<double> &sb, hipStream_t s)
{
    if (a.sc > 3 || a.mc > 2) return hipErrorInvalidValue;
    switch (a.shape) {
    case 5: return launch_abd_tb2_t<double, 4, 8>(a, sa, sb, s);
    case 7: return launch_abd_tb2_t<double, 2, 16>(a, sa, sb, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep2d_abd2_tb_f32(const TBArgs &a, const Stencil<float> &sa,
                                      const Stencil<float> &sb, hipStream_t s)
{
    if (a.sc > 3 || a.mc > 2) return hipErrorInvalidValue;
    switch (a.shape) {
    case 4: return launch_abd_tb2_t<float, 4, 16>(a, sa, sb, s);
    case 5: return launch_abd_tb2_t<float, 4, 8>(a, sa, sb, s);
    case 6: return launch_abd_tb2_t<float, 8, 8>(a, sa, sb, s);
    case 7: return launch_abd_tb2_t<float, 2, 16>(a, sa, sb, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep2d_tb_f32(const TBArgs &a, const Stencil<float> &st, hipStream_t s)
{
    switch (a.shape) {
    case 1: return launch_tb_t<float, 4, 16>(a, st, s);
    case 2: return launch_tb_t<float, 8, 16>(a, st, s);
    case 3: return launch_tb_t<float, 4, 8>(a, st, s);
    case 4: return launch_tb2_t<float, 4, 16>(a, st, s);
    case 5: return launch_tb2_t<float, 4, 8>(a, st, s);
    case 6: return launch_tb2_t<float, 8, 8>(a, st, s);
    case 7: return launch_tb2_t<float, 2, 16>(a, st, s);
    case 8: return launch_tb2_t<float, 8, 16>(a, st, s);
    case 9: return launch_tb3_t<float, 2, 16>(a, st, s);
    case 10: return launch_tb3_t<float, 4, 8>(a, st, s);
    case 11: return launch_tb3_t<float, 2, 8>(a, st, s);
    case 12: return launch_tb3_t<float, 4, 16>(a, st, s);
    case 13: return launch_tb3_t<float, 8, 8>(a, st, s);
    case 14: return launch_tb4_t<float, 5, 8>(a, st, s);
    case 15: return launch_tb4_t<float, 6, 8>(a, st, s);
    default: return launch_tb_t<float, 8, 8>(a, st, s);
    }
}

}  // namespace tdp
