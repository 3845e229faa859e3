// Resident-tile 2-D recurrence sweep: the Table 1 loop on the real field
// (integrator I_acd of Def. 2) for tables without corner mass terms, with
// every tile held on chip for a whole run of steps.
//
// The blocked kernels of sweep_tb.hip reload their tile and refold its
// coefficients for every k steps, and a launch of them is bound by that
// prologue and by the scheduling of a few thousand workgroups.  Here one
// workgroup per compute unit owns one tile for up to TDP_RES_MAXSTEPS steps:
// - at the start it loads the extended tile (exact region plus a k-wide halo)
//   once, folds the cell slowness into per-node coefficients premultiplied
//   by the damping factor d, and keeps d F in LDS;
// - it then advances k steps at a time in registers, exactly as the blocked
//   tile does (rows per lane, DPP x-neighbours, edge rows through LDS, one
//   barrier per step);
// - after each block of k steps it publishes the k-wide border band of its
//   exact region (u_j and u_{j-1}) to its slot of a global exchange buffer
//   and raises its flag; each wave then waits for the flags of the
//   neighbours whose bands it reads (west and east, and the three tiles above
//   or below for the waves holding top or bottom halo rows: the tile as a
//   whole waits for all eight) and reads its halo from their bands.
// A band is packed: the k top rows and the k bottom rows of the exact region
// (full width), then the k left and the k right columns of the rows between
// them, each a row-major block.  It is staged in LDS and copied out with whole-line
// stores; a halo node is read from the band of the tile that owns it.
// The exchange buffer and flags are accessed only with agent-scope relaxed
// atomics, which the compiler emits with the coherent cache policy (sc1):
// they bypass the per-XCD L2 state that is not kept coherent between XCDs.
// A tile's band stores are complete (s_waitcnt) before its flag store is
// issued, and its neighbours issue their band loads only after reading that
// flag, so no L2 writeback or invalidate (the cost of a release/acquire
// fence at agent scope) is needed.  Bands are double-buffered by block
// parity: a tile rewrites a parity only after its neighbours have raised the
// next block's flag, i.e. after they have read that parity.
// Every tile must be resident at once.  A wait that exceeds its poll limit,
// or sees another tile's abort, raises the abort word and the whole grid
// leaves early; the host checks that word after the launch.
#include <hip/hip_runtime.h>

#include "tdp_internal.h"
#include "lanes.h"

namespace tdp {

namespace {

constexpr int kResW = 8;            // waves per workgroup (2 per SIMD)
constexpr int kResR64 = 11;         // rows per lane, FP64: 88 x 64 extended tile
constexpr int kResR32 = 14;         // rows per lane, FP32: 112 x 64 (one word per node value)
constexpr int kResKMax = 8;

// values per level of the largest band (depth 8) of a tile with EY rows
constexpr int res_band_max(int EY) { return 2 * kResKMax * (64 - 2 * kResKMax) + 2 * (EY - 4 * kResKMax) * kResKMax; }

template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_coh(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A zero the optimiser cannot see through.  Added once per block to the
// tile's row origin, it keeps the per-row addresses and conditions of the
// exchange and snapshot code inside the block loop: hoisted, the eleven rows'
// worth of them would take the registers the tile needs.
__device__ __forceinline__ int opaque_zero()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

// One step of the wave's R rows (the blocked tile's second form with d F read
// from LDS): rows r0-1 .. r0+R at x-1, x, x+1 are walked as a rolling window
// of three rows; the halo rows south and north come from the edge-row slots
// cur[rs - 1 .. rs + 1] and cur[rn - 1 .. rn + 1]; the new first and last
// rows go to nxt[wf] and nxt[wl].  b holds u_{j-1} on entry and u_{j+1} on
// exit.  The corner weight d s_2 is rebuilt from e = 1 - 2d as
// s_2/2 - (s_2/2) e, one FMA instead of a register per node.
template <typename T, int SC, int R>
__device__ __forceinline__ void res_step(const T *__restrict__ cur, T *__restrict__ nxt, int rs,
                                         int rn, int wf, int wl,
                                         const typename V2t<T>::type *__restrict__ fl,
                                         const T (&co)[R][5], const T (&e)[R], T s2h,
                                         const T (&a)[R], T (&b)[R], T fas, T fbs)
{
    constexpr bool CORNER = SC > 2;
    T pc = cur[rs];
    T ps = cur[rs - 1] + cur[rs + 1];        // W + E of the row below
    T cw = lane_west(a[0]), cc = a[0], ce = lane_east(a[0]);
    T cs = cw + ce;
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
        const T xs = xw + xe;
        const auto f = fl[i * 64];
        T acc = co[i][0] * cc;
        acc += co[i][1] * cw;
        acc += co[i][2] * ce;
        acc += co[i][3] * pc;
        acc += co[i][4] * xc;
        if (CORNER) acc += (s2h - s2h * e[i]) * (ps + xs);
        acc += fas * f.x;
        acc += fbs * f.y;
        b[i] = acc + e[i] * b[i];
        pc = cc;
        ps = cs;
        cw = xw;
        cc = xc;
        ce = xe;
        cs = xs;
        // keep the window a window: hoisting later rows' shifts would make
        // every row's neighbours live at once
        __builtin_amdgcn_sched_barrier(0);
    }
    nxt[wf] = b[0];
    nxt[wl] = b[R - 1];
}

template <typename T, int SC, int R, int W>
__global__ __launch_bounds__(64 * W) void k_sweep2d_res(ResArgs a, Stencil<T> st)
{
    using V2 = typename V2t<T>::type;
    constexpr int EX = 64, EY = R * W;
    constexpr int US = EX + 2;
    constexpr int CB = (2 * W + 2) * US;          // packed edge-row slots of one copy
    __shared__ T xl[2 * CB];
    __shared__ V2 fl_all[EY * EX];                // d F of the extended tile
    __shared__ double fab[2 * TDP_RES_MAXSTEPS];  // forcing scalars of the launch
    __shared__ T sband[2 * res_band_max(EY)];      // the band being published
    __shared__ int s_abort;

    const int ny = a.ny, nx = a.nx, k = a.k, nsteps = a.nsteps;
    const int OX = EX - 2 * k, OY = EY - 2 * k;
    const int tile = blockIdx.x;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int gy0 = ty * OY - k, gx0 = tx * OX - k;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wv * R;
    const int gx = gx0 + lane;
    const bool xin = (unsigned)gx < (unsigned)nx;
    // the exact region of this tile (clipped to the domain)
    const int ey0 = ty * OY, ey1 = min(ny, ey0 + OY);
    const int ex0 = tx * OX, ex1 = min(nx, ex0 + OX);
    const bool xexact = gx >= ex0 && gx < ex1;
    // the band is defined on the unclipped tile: a border cut by
    // the domain edge has no neighbour to publish to
    const bool xband = xexact && (gx < ex0 + k || gx >= ex0 + OX - k);
    const bool xhalo = lane < k || lane >= k + OX;
    const int band = 2 * k * OX + 2 * (OY - 2 * k) * k;   // values per level
    const int ntl = a.tiles_x * a.tiles_y;
    // per lane: the owner tile column and local column of its x
    const int txo = gx >= 0 ? gx / OX : -1, lxo = gx - txo * OX;
    const int lx = gx - ex0;                               // local column in this tile
    T *const shadow = (T *)a.shadow;
    int *const flags = a.flags;
    int *const abort_word = a.flags + a.tiles_x * a.tiles_y * TDP_RES_FLAG_STRIDE;

    if (threadIdx.x == 0) s_abort = 0;
    for (int t = threadIdx.x; t < 2 * nsteps; t += 64 * W) fab[t] = a.tab[t];
    for (int t = threadIdx.x; t < 2 * CB; t += 64 * W) xl[t] = T(0);

    // the extended tile: cells, u_j, u_{j-1}, d, F; every load is issued
    // before the first use
    T co[R][5], e[R];        // centre, W, E, S, N times d; 1 - 2d
    const T s2h = T(0.5) * st.s[2];
    T u0[R], u1[R];
    {
        const T *m = (const T *)a.m;
        const T *dn = (const T *)a.dn;
        const V2 *F = (const V2 *)a.F;
        const T *u_in = (const T *)a.u_in, *up_in = (const T *)a.up_in;
        T ca[R + 1], cb[R + 1], d[R];
        V2 f[R];
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int sy = gy0 + r0 + i;
            const bool rok = (unsigned)sy <= (unsigned)ny;
            const T *mrow = m + (int64_t)sy * (nx + 1);
            ca[i] = (rok && (unsigned)gx <= (unsigned)nx) ? mrow[gx] : T(0);
            cb[i] = (rok && (unsigned)(gx + 1) <= (unsigned)nx) ? mrow[gx + 1] : T(0);
        }
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
        for (int i = 0; i < R; ++i) {
            fold_node<T, 2, 2, 5>(st, d[i], ca[i], cb[i], ca[i + 1], cb[i + 1], co[i]);
            e[i] = T(1) - T(2) * d[i];
            f[i].x *= d[i];
            f[i].y *= d[i];
            fl_all[(r0 + i) * 64 + lane] = f[i];
        }
    }
    const int rs = 2 * wv * US + lane + 1, rn = (2 * wv + 3) * US + lane + 1;
    const int wf = (2 * wv + 1) * US + lane + 1, wl = (2 * wv + 2) * US + lane + 1;
    T *const c0 = xl, *const c1 = xl + CB;
    const V2 *fl = fl_all + r0 * 64 + lane;
    __syncthreads();
    c0[wf] = u0[0];
    c0[wl] = u0[R - 1];
    __syncthreads();

    int gyw = gy0 + r0;   // first global row of the wave (made opaque per block)
    auto exact_node = [&](int i) {
        const int gy = gyw + i;
        return xexact && gy >= ey0 && gy < ey1;
    };
    auto snapshot = [&](int step, const T(&v)[R]) {   // step: 1-based within the launch
        if (step == a.out_step[0] || step == a.out_step[1]) {
            double *o = step == a.out_step[0] ? a.out[0] : a.out[1];
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (exact_node(i)) (o + 2 * (int64_t)(gyw + i) * nx)[2 * gx] = (double)v[i];
        }
    };

    // A block ends at every sample step, so that the samples are written
    // outside the unrolled steps; after a block of odd length the newest level
    // is in u1 and the two arrays swap back.
    for (int done = 0, blk = 0; done < nsteps; ++blk) {
        int kb = min(k, nsteps - done);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (a.out_step[q] > done && a.out_step[q] < done + kb) kb = a.out_step[q] - done;
        gyw = gy0 + r0 + opaque_zero();
        if (blk > 0) {
            // publish the border band of the exact region (levels j and j-1):
            // packed in LDS, then copied out with whole-line stores.  A row's
            // block of the band and its offset there are uniform; a lane adds
            // its column (top and bottom rows) or its place in the left and
            // right column blocks (the rows between)
            const int par = (blk - 1) & 1;
            const int lside = lx < k ? lx : (OY - 2 * k) * k + lx - (OX - k);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int ly = gyw + i - ey0;
                if (ly < 0 || gyw + i >= ey1) continue;
                if (ly < k || ly >= OY - k) {
                    const int rb = (ly < k ? ly : ly - (OY - 2 * k)) * OX;
                    if (xexact) {
                        sband[rb + lx] = u0[i];
                        sband[band + rb + lx] = u1[i];
                    }
                } else {
                    const int sb = 2 * k * OX + (ly - k) * k;
                    if (xband) {
                        sband[sb + lside] = u0[i];
                        sband[band + sb + lside] = u1[i];
                    }
                }
            }
            __syncthreads();
            T *const mine = shadow + ((int64_t)(par * ntl + tile) * 2) * band;
            for (int t = threadIdx.x; t < 2 * band; t += 64 * W) st_coh(mine + t, sband[t]);
            __builtin_amdgcn_s_waitcnt(0);   // the band stores are complete
            __syncthreads();
            if (threadIdx.x == 0) st_coh(flags + tile * TDP_RES_FLAG_STRIDE, blk);
            // wait for the bands of the same block that this wave reads: its
            // west and east neighbours', and those of the three tiles above
            // (below) when it holds top (bottom) halo rows.  Across its waves
            // the tile waits for all eight neighbours before the barrier after
            // the halo loads, which is also where every wave sees an abort
            {
                const int l = lane, dy = l / 3 - 1;
                const bool need = l < 9 && l != 4 &&
                                  (dy == 0 || (dy < 0 ? r0 < k : r0 + R > k + OY));
                const int nty = ty + dy, ntx = tx + l % 3 - 1;
                if (need && (unsigned)nty < (unsigned)a.tiles_y && (unsigned)ntx < (unsigned)a.tiles_x) {
                    const int *fp = flags + (nty * a.tiles_x + ntx) * TDP_RES_FLAG_STRIDE;
                    int polls = 0;
                    while (ld_coh(fp) < blk + a.wait_bias) {
                        __builtin_amdgcn_s_sleep(2);   // back off: fewer coherent polls in flight
                        if (++polls >= a.poll_limit || ld_coh(abort_word) != 0) {
                            st_coh(abort_word, 1);
                            s_abort = 1;
                            break;
                        }
                    }
                }
            }
            // the halo from the owners' bands: the owner's row and the part of
            // the address it sets are uniform (counted along the rows, no
            // division per row); a lane adds its owner's tile column and its
            // column or place in the owner's left or right column block
            int tyo = gyw >= 0 ? gyw / OY : -1, lyo = gyw - tyo * OY;
            const T *const base = shadow + (int64_t)par * ntl * 2 * band;
            const int ltile = txo * 2 * band;
            const int lsideo = lxo < k ? lxo : (OY - 2 * k) * k + lxo - (OX - k);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = r0 + i, gy = gyw + i;
                const bool hrow = r < k || r >= k + OY;
                if ((hrow || xhalo) && xin && (unsigned)gy < (unsigned)ny) {
                    const bool full = lyo < k || lyo >= OY - k;
                    const int ub = tyo * a.tiles_x * 2 * band +
                                   (full ? (lyo < k ? lyo : lyo - (OY - 2 * k)) * OX
                                         : 2 * k * OX + (lyo - k) * k);
                    const T *src = base + ub + ltile + (full ? lxo : lsideo);
                    u0[i] = ld_coh(src);
                    u1[i] = ld_coh(src + band);
                }
                if (++lyo == OY) {
                    lyo = 0;
                    ++tyo;
                }
            }
            c0[wf] = u0[0];
            c0[wl] = u0[R - 1];
            __syncthreads();
            if (s_abort) return;     // a wait gave up: halo values may be stale
        }
        bool odd = false;
#pragma unroll
        for (int s = 0; s < kResKMax; s += 2) {
            if (s >= kb) break;
            res_step<T, SC, R>(c0, c1, rs, rn, wf, wl, fl, co, e, s2h, u0, u1,
                               (T)fab[2 * (done + s)], (T)fab[2 * (done + s) + 1]);
            __syncthreads();
            if (s + 1 >= kb) {
                odd = true;
                break;
            }
            res_step<T, SC, R>(c1, c0, rs, rn, wf, wl, fl, co, e, s2h, u1, u0,
                               (T)fab[2 * (done + s + 1)], (T)fab[2 * (done + s + 1) + 1]);
            __syncthreads();
        }
        if (odd) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const T t = u0[i];
                u0[i] = u1[i];
                u1[i] = t;
            }
        }
        done += kb;
        snapshot(done, u0);
    }
    T *u_out = (T *)a.u_out, *up_out = (T *)a.up_out;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (exact_node(i)) {
            const int64_t row = (int64_t)(gyw + i) * nx;
            (u_out + row)[gx] = u0[i];
            (up_out + row)[gx] = u1[i];
        }
    }
}

}  // namespace

int res_tile_rows(bool f64) { return (f64 ? kResR64 : kResR32) * kResW; }

size_t res_band_bytes(bool f64)
{
    return f64 ? 2 * res_band_max(kResR64 * kResW) * sizeof(double)
               : 2 * res_band_max(kResR32 * kResW) * sizeof(float);
}

int res_tiles(int ny, int nx, int k, bool f64, int *tiles_x, int *tiles_y)
{
    const int rows = res_tile_rows(f64);
    if (rows == 0 || k < 2 || k > kResKMax || (k & 1) || 4 * k > rows) return 0;
    const int ox = 64 - 2 * k, oy = rows - 2 * k;
    const int tx = (nx + ox - 1) / ox, tyc = (ny + oy - 1) / oy;
    if (tiles_x) *tiles_x = tx;
    if (tiles_y) *tiles_y = tyc;
    return tx * tyc;
}

template <typename T, int R>
static hipError_t launch_res_t(const ResArgs &a, const Stencil<T> &st, hipStream_t s)
{
    const int nt = a.tiles_x * a.tiles_y;
    if (a.sc > 2)
        hipLaunchKernelGGL((k_sweep2d_res<T, 3, R, kResW>), dim3(nt), dim3(64 * kResW), 0, s, a, st);
    else
        hipLaunchKernelGGL((k_sweep2d_res<T, 2, R, kResW>), dim3(nt), dim3(64 * kResW), 0, s, a, st);
    return hipGetLastError();
}

hipError_t launch_sweep2d_res_f64(const ResArgs &a, const Stencil<double> &st, hipStream_t s)
{
    return launch_res_t<double, kResR64>(a, st, s);
}

hipError_t launch_sweep2d_res_f32(const ResArgs &a, const Stencil<float> &st, hipStream_t s)
{
    return launch_res_t<float, kResR32>(a, st, s);
}

}  // namespace tdp
