// 3-D recurrence sweep streamed along axis 0 ("2.5-D"): one step per launch
// (Table 1 loop, integrator I_acd of Def. 2).
//
// A workgroup owns a 64 x TY column of nodes in the (axis 2, axis 1) plane and
// walks a chunk of ZC planes along axis 0.  Three planes of u_j (z-1, z, z+1,
// each with a one-node halo) and the two cell planes the nodes of plane z use
// rotate through LDS, so every plane of u and of the cell slowness is fetched
// from HBM about once per step (plus the in-plane halo) instead of being
// re-read for each of its 19 or 27 uses.  u_{j-1}, the damping factor and F are
// read once per node straight from HBM, and u_{j+1} written once (non-temporal
// when the step's working set exceeds the MALL, see stream_nt).  Workgroups are ordered so each XCD
// gets a contiguous range of tiles (in-plane halo re-reads hit its L2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "tdp_internal.h"

namespace tdp {

template <typename T>
struct V2s;
template <>
struct V2s<double> {
    using type = double2;
};
template <>
struct V2s<float> {
    using type = float2;
};

// assembled stencil around one node: U(oz, oy, ox) reads the rotating u
// planes, w[e] the 8 cells (e = ex + 2 ey + 4 ez); same formula as
// eval_stencil in kernels.hip.
template <int SC, int MC, typename T, typename LoadU>
__device__ __forceinline__ T stencil27(const LoadU &U, const T *w, const Stencil<T> &st)
{
    constexpr int NC = SC > MC ? SC : MC;
    T us[4] = {T(0), T(0), T(0), T(0)};
    T ws[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const int ox = k % 3 - 1, oy = (k / 3) % 3 - 1, oz = k / 9 - 1;
        const int cls = (ox != 0) + (oy != 0) + (oz != 0);
        if (cls >= NC) continue;
        const T v = U(oz, oy, ox);
        if (cls < SC || cls == 0) us[cls] += v;
        if (cls < MC) {
            T W = T(0);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                const bool okx = ox == 0 || (ox < 0 ? ex == 0 : ex == 1);
                const bool oky = oy == 0 || (oy < 0 ? ey == 0 : ey == 1);
                const bool okz = oz == 0 || (oz < 0 ? ez == 0 : ez == 1);
                if (okx && oky && okz) W += w[e];
            }
            ws[cls] += W * v;
        }
    }
    T r = st.c0 * us[0];
#pragma unroll
    for (int k = 1; k < SC; ++k) r += st.s[k] * us[k];
#pragma unroll
    for (int k = 0; k < MC; ++k) r += st.m[k] * ws[k];
    return r;
}

// Folded form of the update for tables whose mass entries are the centre and
// face classes only (at most three stiffness and two mass classes: the
// compact and second-order schemes).  From the eight cells around a node the
// centre and the six face neighbours get one coefficient each (their
// stiffness constant plus the mass constant times the cells they share with
// the node), the twelve edge neighbours share the edge stiffness constant,
// all premultiplied by the damping factor d, so that an update is
//   u_{j+1} = sum_q c_q u_j(q) + fa d Re F + fb d Im F + (1 - 2d) u_{j-1}
// in about 22 operations instead of a fold per neighbour.  `d` is kept for
// the edge weight and the u_{j-1} factor.
template <typename T>
struct Fold3 {
    T c0, cw, ce, cs, cn, cd, cu, d;
};

// Compact form, for a fold kept in registers until a later update: two
// opposite faces share the node's eight cells between them, so their
// coefficients sum to the same cx = d (2 s_1 + m_1 sum w) on every axis.  It
// keeps the west, south and down coefficients and cx (east = cx - west, ...).
template <typename T>
struct Fold3c {
    T c0, cx, cw, cs, cd, d;
};

template <typename T>
struct CellSums {
    T w0, ww, ws, wd, wu;     // all eight cells; those with ex = 0, ey = 0, ez = 0, ez = 1
};

template <typename T>
__device__ __forceinline__ CellSums<T> cell_sums(const T (&w)[8])
{
    const T w01 = w[0] + w[1], w23 = w[2] + w[3], w45 = w[4] + w[5], w67 = w[6] + w[7];
    CellSums<T> c;
    c.wd = w01 + w23;
    c.wu = w45 + w67;
    c.ws = w01 + w45;
    c.ww = (w[0] + w[2]) + (w[4] + w[6]);
    c.w0 = c.wd + c.wu;
    return c;
}

template <typename T>
__device__ __forceinline__ Fold3<T> fold3(const T (&w)[8], T d, const Stencil<T> &st)
{
    const CellSums<T> c = cell_sums(w);
    Fold3<T> f;
    f.c0 = d * (st.c0 + st.m[0] * c.w0);
    f.cw = d * (st.s[1] + st.m[1] * c.ww);
    f.ce = d * (st.s[1] + st.m[1] * (c.w0 - c.ww));
    f.cs = d * (st.s[1] + st.m[1] * c.ws);
    f.cn = d * (st.s[1] + st.m[1] * (c.w0 - c.ws));
    f.cd = d * (st.s[1] + st.m[1] * c.wd);
    f.cu = d * (st.s[1] + st.m[1] * c.wu);
    f.d = d;
    return f;
}

template <typename T>
__device__ __forceinline__ Fold3c<T> fold3c(const T (&w)[8], T d, const Stencil<T> &st)
{
    const CellSums<T> c = cell_sums(w);
    Fold3c<T> f;
    f.c0 = d * (st.c0 + st.m[0] * c.w0);
    f.cx = d * (T(2) * st.s[1] + st.m[1] * c.w0);
    f.cw = d * (st.s[1] + st.m[1] * c.ww);
    f.cs = d * (st.s[1] + st.m[1] * c.ws);
    f.cd = d * (st.s[1] + st.m[1] * c.wd);
    f.d = d;
    return f;
}

template <typename T, typename LoadU>
__device__ __forceinline__ T edge_sum(const LoadU &U)
{
    return ((U(-1, -1, 0) + U(-1, 1, 0)) + (U(-1, 0, -1) + U(-1, 0, 1))) +
           ((U(1, -1, 0) + U(1, 1, 0)) + (U(1, 0, -1) + U(1, 0, 1))) +
           ((U(0, -1, -1) + U(0, -1, 1)) + (U(0, 1, -1) + U(0, 1, 1)));
}

// U(oz, oy, ox) reads u_j around the node; dfr, dfi = d Re F, d Im F
template <typename T, typename LoadU>
__device__ __forceinline__ T update3(const LoadU &U, const Fold3<T> &f, const Stencil<T> &st,
                                     T fa, T fb, T dfr, T dfi, T uprev)
{
    const T edges = edge_sum<T>(U);
    T acc = f.c0 * U(0, 0, 0);
    acc += f.cw * U(0, 0, -1);
    acc += f.ce * U(0, 0, 1);
    acc += f.cs * U(0, -1, 0);
    acc += f.cn * U(0, 1, 0);
    acc += f.cd * U(-1, 0, 0);
    acc += f.cu * U(1, 0, 0);
    acc += (f.d * st.s[2]) * edges;
    acc += fa * dfr;
    acc += fb * dfi;
    return acc + (T(1) - T(2) * f.d) * uprev;
}

template <typename T, typename LoadU>
__device__ __forceinline__ T update3(const LoadU &U, const Fold3c<T> &f, const Stencil<T> &st,
                                     T fa, T fb, T dfr, T dfi, T uprev)
{
    const T edges = edge_sum<T>(U);
    T acc = f.c0 * U(0, 0, 0);
    acc += f.cw * U(0, 0, -1);
    acc += (f.cx - f.cw) * U(0, 0, 1);
    acc += f.cs * U(0, -1, 0);
    acc += (f.cx - f.cs) * U(0, 1, 0);
    acc += f.cd * U(-1, 0, 0);
    acc += (f.cx - f.cd) * U(1, 0, 0);
    acc += (f.d * st.s[2]) * edges;
    acc += fa * dfr;
    acc += fb * dfi;
    return acc + (T(1) - T(2) * f.d) * uprev;
}

template <typename T, int SC, int MC, int TY, int RY, bool NTS>
__global__ __launch_bounds__(64 * TY) void k_sweep3d_stream(
    const T *__restrict__ u, T *__restrict__ up, const T *__restrict__ m,
    const T *__restrict__ dn, const typename V2s<T>::type *__restrict__ F, int nz, int ny,
    int nx, Stencil<T> st, T fa, T fb, double *__restrict__ out, int zc, int tiles_x,
    int tiles_y, int ntiles, int per_xcd)
{
    constexpr int NT = 64 * TY;
    constexpr int RT = TY * RY;              // node rows per tile
    constexpr int EX = 66, EY = RT + 2;      // u plane with halo
    constexpr int CX = 65, CY = RT + 1;      // cell plane
    constexpr int UPT = (EY * EX + NT - 1) / NT;   // plane elements staged per thread
    constexpr int CPT = (CY * CX + NT - 1) / NT;
    __shared__ T us[3][EY * EX];
    __shared__ T cs[2][CY * CX];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int bx = tile % tiles_x;
    const int by = (tile / tiles_x) % tiles_y;
    const int bz = tile / (tiles_x * tiles_y);
    const int x0 = bx * 64, y0 = by * RT, zb = bz * zc;
    const int ze = min(nz, zb + zc);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t plane = (int64_t)ny * nx;
    const int64_t cplane = (int64_t)(ny + 1) * (nx + 1);

    // global -> registers for one u plane (with halo) and one cell plane
    T ru[UPT], rc[CPT];
    auto fetch_u = [&](int p) {
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
            const int t = threadIdx.x + q * NT;
            const int r = t / EX, c = t % EX;
            const int gy = y0 - 1 + r, gx = x0 - 1 + c;
            const bool ok = t < EY * EX && (unsigned)p < (unsigned)nz &&
                            (unsigned)gy < (unsigned)ny && (unsigned)gx < (unsigned)nx;
            ru[q] = ok ? u[p * plane + (int64_t)gy * nx + gx] : T(0);
        }
    };
    auto fetch_c = [&](int qz) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int t = threadIdx.x + q * NT;
            const int r = t / CX, c = t % CX;
            const int sy = y0 + r, sx = x0 + c;
            const bool ok = t < CY * CX && (unsigned)qz <= (unsigned)nz &&
                            (unsigned)sy <= (unsigned)ny && (unsigned)sx <= (unsigned)nx;
            rc[q] = ok ? m[qz * cplane + (int64_t)sy * (nx + 1) + sx] : T(0);
        }
    };
    auto store_u = [&](int slot) {
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
            const int t = threadIdx.x + q * NT;
            if (t < EY * EX) us[slot][t] = ru[q];
        }
    };
    auto store_c = [&](int slot) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int t = threadIdx.x + q * NT;
            if (t < CY * CX) cs[slot][t] = rc[q];
        }
    };
    const int gx = x0 + tx;
    // per-node data (u_{j-1}, damping factor, F) of this thread's RY nodes of a plane
    T nup[RY], nd[RY], nfr[RY], nfi[RY];
    auto fetch_node = [&](int p) {
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int gy = y0 + ty + TY * q;
            nup[q] = nd[q] = nfr[q] = nfi[q] = T(0);
            if (gy < ny && gx < nx && p < ze) {
                const int64_t i = p * plane + (int64_t)gy * nx + gx;
                nup[q] = ldnt<NTS>(up + i);
                nd[q] = ldnt<NTS>(dn + i);
                nfr[q] = ldnt<NTS>(&F[i].x);
                nfi[q] = ldnt<NTS>(&F[i].y);
            }
        }
    };

    // prologue: u planes zb-1, zb, zb+1; cell planes zb, zb+1; node data of zb
    fetch_u(zb - 1);
    store_u(0);
    fetch_u(zb);
    store_u(1);
    fetch_u(zb + 1);
    store_u(2);
    fetch_c(zb);
    store_c(0);
    fetch_c(zb + 1);
    store_c(1);
    fetch_node(zb);
    __syncthreads();
    for (int z = zb; z < ze; ++z) {
        const int s0 = (z - zb) % 3, s1 = (z - zb + 1) % 3, s2 = (z - zb + 2) % 3;
        const int c0 = (z - zb) & 1, c1 = (z - zb + 1) & 1;
        T cup[RY], cd[RY], cfr[RY], cfi[RY];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            cup[q] = nup[q];
            cd[q] = nd[q];
            cfr[q] = nfr[q];
            cfi[q] = nfi[q];
        }
        // issue the next iteration's loads before computing this plane
        const bool more = z + 1 < ze;
        if (more) {
            fetch_u(z + 2);
            fetch_c(z + 2);
            fetch_node(z + 1);
        }
        const T *pl0 = us[s0], *pl1 = us[s1], *pl2 = us[s2];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int ry = ty + TY * q;           // row within the tile
            const int gy = y0 + ry;
            if (gy < ny && gx < nx) {
                const int base = (ry + 1) * EX + tx + 1;
                auto U = [&](int oz, int oy, int ox) -> T {
                    const T *pl = oz < 0 ? pl0 : (oz == 0 ? pl1 : pl2);
                    return pl[base + oy * EX + ox];
                };
                T w[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                    w[e] = cs[ez ? c1 : c0][(ry + ey) * CX + tx + ex];
                }
                T r;
                if constexpr (SC == 3 && MC == 2) {
                    r = update3(U, fold3(w, cd[q], st), st, fa, fb, cd[q] * cfr[q], cd[q] * cfi[q],
                                cup[q]);
                } else {
                    const T acc = stencil27<SC, MC>(U, w, st);
                    r = cd[q] * (acc + fa * cfr[q] + fb * cfi[q]) - (T(2) * cd[q] - T(1)) * cup[q];
                }
                const int64_t i = z * plane + (int64_t)gy * nx + gx;
                stnt<NTS>(r, up + i);
                if (out) out[2 * i] = (double)r;
            }
        }
        if (!more) break;
        __syncthreads();          // plane z-1 and cell plane z no longer read
        store_u(s0);              // u plane z+2 replaces plane z-1
        store_c(c0);              // cell plane z+2 replaces cell plane z
        __syncthreads();
    }
}

// Two steps per launch.  From u_j (level 0) and u_{j-1}, a workgroup computes
// level 1 (u_{j+1}) on a 66 x LY node block and level 2 (u_{j+2}) on its
// 64 x (LY-2) interior, walking along axis 0: in iteration i it forms level 1
// on plane a = zb-1+i and level 2 on plane a-2, whose level-1 inputs (planes
// a-3 .. a-1) were all formed in earlier iterations, so one barrier per plane
// orders everything.  The block's positions are dealt to the NT threads in
// row-major order (t, t + NT, ...), so a 64-wide output needs no 64-lane
// level-1 row and a 256-node axis takes exactly four column blocks.  LDS
// rings: level-0 planes in 5 slots (a-2 .. a+1 read, a+2 arriving from the
// registers it was prefetched into), level-1 planes in 4 (a written, a-3 ..
// a-1 read), cell planes in 3 (5 when level 2 refolds from the cells).  u_{j-1},
// d and F of plane a are fetched one iteration ahead.  For the compact tables a
// node's coefficients are folded once, at level 1, and carried in registers to
// its level-2 update two iterations later.  Per node and launch this reads
// u_j, u_{j-1}, m, d, F once and writes u_{j+1}, u_{j+2}: about 4 words per
// node-step instead of 7.
//
// Every column block is split along axis 0 at the same plane boundaries into
// nrun runs, one workgroup each; the host picks nrun so that the workgroups
// fill whole rounds of the resident slots (see launch_stream2_t).  Workgroups
// are ordered run-major and each XCD gets a contiguous range, so blocks that
// are neighbours in the plane walk the same planes at the same time and their
// halo re-reads hit that XCD's L2.  Outputs must not alias the inputs.

// waves per SIMD the register allocation must allow: two 512-thread FP32
// workgroups per compute unit (their LDS allows it); FP64 ones are held to
// one by their LDS
template <typename T, int NT>
constexpr int stream2_waves() { return NT >= 1024 || sizeof(T) == 4 ? 4 : 2; }

template <typename T, int SC, int MC, int NT, int LY, bool NTS>
__global__ __launch_bounds__(NT, (stream2_waves<T, NT>())) void k_sweep3d_stream2(
    const T *__restrict__ u, const T *__restrict__ up, T *__restrict__ u2o,
    T *__restrict__ u1o, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2s<T>::type *__restrict__ F, int nz, int ny, int nx, Stencil<T> st, T fa1,
    T fb1, T fa2, T fb2, double *__restrict__ out1, double *__restrict__ out2, int tiles_x,
    int ncb, int nrun, int per_xcd)
{
    constexpr int LX = 66, OX = LX - 2, OY = LY - 2;
    constexpr int NL = LX * LY;                     // level-1 positions
    constexpr int P = (NL + NT - 1) / NT;           // positions per thread
    constexpr int EX = LX + 2, NE = EX * (LY + 2);  // level-0 plane with its halo
    constexpr int CX = LX + 1, NC = CX * (LY + 1);  // cell plane
    constexpr int UPT = (NE + NT - 1) / NT, CPT = (NC + NT - 1) / NT;
    constexpr bool FOLD = SC == 3 && MC == 2;
    constexpr int NCS = FOLD ? 3 : 5;
    __shared__ T s0[5][NE];
    __shared__ T s1[4][NL];
    __shared__ T scl[NCS][NC];

    const int id = blockIdx.x;
    const int w = (id % 8) * per_xcd + id / 8;
    if (w >= ncb * nrun) return;
    const int run = w / ncb, cblk = w - run * ncb;
    const int zb = (int)((int64_t)run * nz / nrun), ze = (int)((int64_t)(run + 1) * nz / nrun);
    const int64_t plane = (int64_t)ny * nx;
    const int64_t cplane = (int64_t)(ny + 1) * (nx + 1);
    const int tid = threadIdx.x;

    // this thread's level-1 positions t = tid + q NT, at (r, c) = (t / LX,
    // t % LX) of the block: r is kept, the rest follows from it
    int rr[P];
#pragma unroll
    for (int q = 0; q < P; ++q) rr[q] = (tid + q * NT) / LX;
    auto ub = [&](int q) { return tid + q * NT + 2 * rr[q] + EX + 1; };   // level-0 LDS offset
    auto cb = [&](int q) { return tid + q * NT + rr[q]; };                // cell LDS offset
    auto inner = [&](int q) {          // interior of the block: level 2 and stored outputs
        const int t = tid + q * NT, c = t - rr[q] * LX;
        return t < NL && rr[q] >= 1 && rr[q] < LY - 1 && c >= 1 && c < LX - 1;
    };

    T ru[UPT], rc[CPT];
    int eo[UPT], co[CPT], no[P];   // in-plane offsets from the block origin, -1 outside
    T cum[P], cd[P], cfr[P], cfi[P];
    // what a node's level-2 update needs from its plane: the folded
    // coefficients with d, and d F (unfolded tables: d and F).  Three sets:
    // iteration i writes set i mod 3 (plane a) and reads set (i + 1) mod 3
    // (plane a-2, written two iterations earlier); the loop is unrolled by
    // three so that the sets stay in place
    struct Carry {
        Fold3c<T> f;
        T fr, fi;
    };
    Carry kA[P], kB[P], kC[P];

    const int x0 = (cblk % tiles_x) * OX, y0 = (cblk / tiles_x) * OY;
    const int64_t nb = (int64_t)(y0 - 1) * nx + (x0 - 1);          // node (r, c) = (0, 0)
    const int64_t eb = nb - nx - 1;                                 // level-0 item (0, 0)
    const int64_t cbase = (int64_t)(y0 - 1) * (nx + 1) + (x0 - 1);  // cell item (0, 0)
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
        const int t = tid + q * NT, r = t / EX, c = t % EX;
        const int gy = y0 - 2 + r, gx = x0 - 2 + c;
        eo[q] = t < NE && (unsigned)gy < (unsigned)ny && (unsigned)gx < (unsigned)nx ? r * nx + c : -1;
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int t = tid + q * NT, r = t / CX, c = t % CX;
        const int sy = y0 - 1 + r, sx = x0 - 1 + c;
        co[q] = t < NC && (unsigned)sy <= (unsigned)ny && (unsigned)sx <= (unsigned)nx
                    ? r * (nx + 1) + c : -1;
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int c = tid + q * NT - rr[q] * LX;
        const int gy = y0 - 1 + rr[q], gx = x0 - 1 + c;
        no[q] = tid + q * NT < NL && (unsigned)gy < (unsigned)ny && (unsigned)gx < (unsigned)nx
                    ? rr[q] * nx + c : -1;
    }
    auto slot = [&](int p) { return (p - zb + 2) % 5; };         // level-0 planes
    auto cslot = [&](int p) { return (p - zb + 2) % NCS; };      // cell planes
    auto slot1 = [&](int p) { return (p - zb + 1) & 3; };        // level-1 planes
    auto fetch_u = [&](int p) {
        const bool zin = (unsigned)p < (unsigned)nz;
        const int64_t o = p * plane + eb;
#pragma unroll
        for (int q = 0; q < UPT; ++q) ru[q] = zin && eo[q] >= 0 ? u[o + eo[q]] : T(0);
    };
    auto fetch_c = [&](int p) {
        const bool zin = (unsigned)p <= (unsigned)nz;
        const int64_t o = p * cplane + cbase;
#pragma unroll
        for (int q = 0; q < CPT; ++q) rc[q] = zin && co[q] >= 0 ? m[o + co[q]] : T(0);
    };
    auto store_u = [&](int sl) {
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
            const int t = tid + q * NT;
            if (UPT * NT == NE || t < NE) s0[sl][t] = ru[q];
        }
    };
    auto store_c = [&](int sl) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int t = tid + q * NT;
            if (CPT * NT == NC || t < NC) scl[sl][t] = rc[q];
        }
    };
    auto fetch_node = [&](int p) {
        const bool zin = (unsigned)p < (unsigned)nz;
        const int64_t o = p * plane + nb;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            cum[q] = cd[q] = cfr[q] = cfi[q] = T(0);
            if (zin && no[q] >= 0) {
                const int64_t i = o + no[q];
                cum[q] = ldnt<NTS>(up + i);
                cd[q] = ldnt<NTS>(dn + i);
                cfr[q] = ldnt<NTS>(&F[i].x);
                cfi[q] = ldnt<NTS>(&F[i].y);
            }
        }
    };

    // prologue: level-0 and cell planes zb-2, zb-1, zb; node data of plane zb-1
#pragma unroll 1
    for (int p = zb - 2; p <= zb; ++p) {
        fetch_u(p);
        fetch_c(p);
        store_u(slot(p));
        store_c(cslot(p));
    }
    fetch_node(zb - 1);
    __syncthreads();
    // level 1 on planes zb-1 .. ze, level 2 on zb .. ze-1 (two planes behind)
    const int iters = ze - zb + 3;
    auto step = [&](int it, Carry (&k0)[P], const Carry (&k2)[P]) {
        const int a = zb - 1 + it, b = a - 2;
        const bool lev1 = a <= ze, pref = a + 1 <= ze;
        if (pref) {                // planes a+2 (level 0, cells); node data of a+1 after level 1
            fetch_u(a + 2);
            fetch_c(a + 2);
        }
        // level 1 on plane a (the whole block, rim included; zero outside the grid)
        if (lev1) {
            const bool ain = (unsigned)a < (unsigned)nz;
            const bool aout = a >= zb && a < ze;
            const T *p0 = s0[slot(a - 1)], *p1 = s0[slot(a)], *p2 = s0[slot(a + 1)];
            const T *c0p = scl[cslot(a)], *c1p = scl[cslot(a + 1)];
            T *l1 = s1[slot1(a)];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int t = tid + q * NT;
                if (P * NT > NL && t >= NL) continue;
                T v = T(0);
                if (ain && no[q] >= 0) {
                    const int base = ub(q);
                    auto U = [&](int oz, int oy, int ox) -> T {
                        const T *pl = oz < 0 ? p0 : (oz == 0 ? p1 : p2);
                        return pl[base + oy * EX + ox];
                    };
                    T w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                        w[e] = (ez ? c1p : c0p)[cb(q) + ey * CX + ex];
                    }
                    if constexpr (FOLD) {
                        k0[q].f = fold3c(w, cd[q], st);
                        k0[q].fr = cd[q] * cfr[q];
                        k0[q].fi = cd[q] * cfi[q];
                        v = update3(U, k0[q].f, st, fa1, fb1, k0[q].fr, k0[q].fi, cum[q]);
                    } else {
                        const T acc = stencil27<SC, MC>(U, w, st);
                        v = cd[q] * (acc + fa1 * cfr[q] + fb1 * cfi[q]) - (T(2) * cd[q] - T(1)) * cum[q];
                        k0[q].f.d = cd[q];
                        k0[q].fr = cfr[q];
                        k0[q].fi = cfi[q];
                    }
                    if (aout && inner(q)) {
                        const int64_t i = a * plane + nb + no[q];
                        stnt<NTS>(v, u1o + i);
                        if (out1) out1[2 * i] = (double)v;
                    }
                }
                l1[t] = v;
            }
            if (pref) fetch_node(a + 1);   // plane a's node data are consumed
        }
        // level 2 on plane b (interior of the block); its level-1 planes
        // b-1 .. b+1 = a-3 .. a-1 were formed before the last barrier
        if (b >= zb) {
            const T *q0 = s1[slot1(b - 1)], *q1 = s1[slot1(b)], *q2 = s1[slot1(b + 1)];
            const T *u0c = s0[slot(b)];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if (!inner(q) || no[q] < 0) continue;
                const int base = tid + q * NT;
                auto U = [&](int oz, int oy, int ox) -> T {
                    const T *pl = oz < 0 ? q0 : (oz == 0 ? q1 : q2);
                    return pl[base + oy * LX + ox];
                };
                const T uc = u0c[ub(q)];
                T v;
                if constexpr (FOLD) {
                    v = update3(U, k2[q].f, st, fa2, fb2, k2[q].fr, k2[q].fi, uc);
                } else {
                    const T *d0p = scl[cslot(b)], *d1p = scl[cslot(b + 1)];
                    T w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                        w[e] = (ez ? d1p : d0p)[cb(q) + ey * CX + ex];
                    }
                    const T acc = stencil27<SC, MC>(U, w, st);
                    const T d2 = k2[q].f.d;
                    v = d2 * (acc + fa2 * k2[q].fr + fb2 * k2[q].fi) - (T(2) * d2 - T(1)) * uc;
                }
                const int64_t i = b * plane + nb + no[q];
                stnt<NTS>(v, u2o + i);
                if (out2) out2[2 * i] = (double)v;
            }
        }
        if (pref) {                // slots of planes a-3 (level 0) and a-1 (cells) are free
            store_u(slot(a + 2));
            store_c(cslot(a + 2));
        }
        __syncthreads();
    };
    // the scheduling barriers keep the three bodies from being interleaved,
    // which would hold more registers live than a lane has (spills)
#pragma unroll 1
    for (int it = 0; it < iters; it += 3) {
        step(it, kA, kB);
        __builtin_amdgcn_sched_barrier(0);
        if (it + 1 < iters) step(it + 1, kB, kC);
        __builtin_amdgcn_sched_barrier(0);
        if (it + 2 < iters) step(it + 2, kC, kA);
    }
}

// workgroups of one stream2 instantiation resident per compute unit, queried
// once (sweep3d_stream2_prepare runs the query before any stream capture)
template <typename T, int SC, int MC, int NT, int LY, bool NTS>
static int stream2_per_cu()
{
    static const int v = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, k_sweep3d_stream2<T, SC, MC, NT, LY, NTS>, NT, 0) != hipSuccess || nb < 1)
            nb = 1;
        return nb;
    }();
    return v;
}

template <typename T, int NT, int LY>
static void prepare_stream2_t()
{
    stream2_per_cu<T, 3, 2, NT, LY, true>();
    stream2_per_cu<T, 3, 2, NT, LY, false>();
    stream2_per_cu<T, 4, 4, NT, LY, true>();
    stream2_per_cu<T, 4, 4, NT, LY, false>();
}

// Runs per column block: the one minimising rounds x (run length + 3), the
// rounds of `slots` resident workgroups that ncb x nrun workgroups take and
// the prologue of about three planes' loads per run; runs of at least zc
// planes.  256^3 FP32 on shape 2 (36 blocks, 256 slots): 7 runs of 36-37
// planes, one round.
static int stream2_runs(int64_t ncb, int nz, int zc, int64_t slots)
{
    const int kmax = std::max(1, std::min(4096, nz / std::max(zc, 1)));
    int best_k = 1;
    double best = INFINITY;
    for (int k = 1; k <= kmax; ++k) {
        const int64_t rounds = (ncb * k + slots - 1) / slots;
        const double cost = (double)rounds * ((nz + k - 1) / k + 3);
        if (cost < best) {
            best = cost;
            best_k = k;
        }
    }
    return best_k;
}

template <typename T, int NT, int LY>
static hipError_t launch_stream2_t(const Stream2Args &a, const Stencil<T> &st, hipStream_t s)
{
    const int nz = a.n[0], ny = a.n[1], nx = a.n[2];
    constexpr int OY = LY - 2;
    const int tiles_x = (nx + 63) / 64, tiles_y = (ny + OY - 1) / OY;
    const int64_t ncb = (int64_t)tiles_x * tiles_y;
    const T *u = (const T *)a.u, *up = (const T *)a.up;
    T *u2o = (T *)a.u2out, *u1o = (T *)a.u1out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2s<T>::type *)a.F;
    const T fa1 = (T)a.fa[0], fb1 = (T)a.fb[0], fa2 = (T)a.fa[1], fb2 = (T)a.fb[1];
    const bool nt = stream_nt((int64_t)7 * sizeof(T) * nz * ny * nx);
    if (ncb * nz > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
#define TDP_S2(SC, MC, NTS)                                                                          \
    do {                                                                                             \
        const int64_t slots = (int64_t)stream2_per_cu<T, SC, MC, NT, LY, NTS>() * a.ncu;             \
        const int nrun = stream2_runs(ncb, nz, a.zc, std::max<int64_t>(slots, 1));                   \
        const int per_xcd = (int)((ncb * nrun + 7) / 8);                                             \
        hipLaunchKernelGGL((k_sweep3d_stream2<T, SC, MC, NT, LY, NTS>), dim3(8 * per_xcd), dim3(NT), \
                           0, s, u, up, u2o, u1o, m, dn, F, nz, ny, nx, st, fa1, fb1, fa2, fb2,      \
                           a.out1, a.out2, tiles_x, (int)ncb, nrun, per_xcd);                        \
    } while (0)
    if (a.sc <= 3 && a.mc <= 2) {
        if (nt) TDP_S2(3, 2, true);
        else TDP_S2(3, 2, false);
    } else {
        if (nt) TDP_S2(4, 4, true);
        else TDP_S2(4, 4, false);
    }
#undef TDP_S2
    return hipGetLastError();
}

// shape: 0 -> 512 threads on a 66 x 15 level-1 block (64 x 13 outputs, two
// positions per thread), 1 -> 1024 threads on 66 x 15 (one position per
// thread), 2 -> 1024 threads on 66 x 31 (64 x 29 outputs; FP32 only, FP64
// takes shape 1: its LDS rings would exceed 160 KB)
hipError_t launch_sweep3d_stream2_f64(const Stream2Args &a, const Stencil<double> &st, int shape,
                                      hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream2_t<double, 512, 15>(a, st, s);
    default: return launch_stream2_t<double, 1024, 15>(a, st, s);
    }
}

hipError_t launch_sweep3d_stream2_f32(const Stream2Args &a, const Stencil<float> &st, int shape,
                                      hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream2_t<float, 512, 15>(a, st, s);
    case 2: return launch_stream2_t<float, 1024, 31>(a, st, s);
    default: return launch_stream2_t<float, 1024, 15>(a, st, s);
    }
}

void sweep3d_stream2_prepare(bool f64, int shape)
{
    if (f64) {
        switch (shape) {
        case 0: prepare_stream2_t<double, 512, 15>(); break;
        default: prepare_stream2_t<double, 1024, 15>(); break;
        }
    } else {
        switch (shape) {
        case 0: prepare_stream2_t<float, 512, 15>(); break;
        case 2: prepare_stream2_t<float, 1024, 31>(); break;
        default: prepare_stream2_t<float, 1024, 15>(); break;
        }
    }
}

template <typename T, int TY, int RY>
static hipError_t launch_stream_t(const SweepArgs &a, const Stencil<T> &st, T fa, T fb, int zc,
                                  hipStream_t s)
{
    const int nz = a.n[0], ny = a.n[1], nx = a.n[2];
    const int tiles_x = (nx + 63) / 64, tiles_y = (ny + TY * RY - 1) / (TY * RY);
    const int tiles_z = (nz + zc - 1) / zc;
    const int ntiles = tiles_x * tiles_y * tiles_z;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * TY);
    const T *u = (const T *)a.u;
    T *up = (T *)a.up;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2s<T>::type *)a.F;
    const bool nt = stream_nt((int64_t)7 * sizeof(T) * nz * ny * nx);
#define TDP_S1(SC, MC, NTS)                                                                       \
    hipLaunchKernelGGL((k_sweep3d_stream<T, SC, MC, TY, RY, NTS>), grd, blk, 0, s, u, up, m, dn, F, \
                       nz, ny, nx, st, fa, fb, a.out, zc, tiles_x, tiles_y, ntiles, per_xcd)
    if (a.sc <= 3 && a.mc <= 2) {
        if (nt) TDP_S1(3, 2, true);
        else TDP_S1(3, 2, false);
    } else {
        if (nt) TDP_S1(4, 4, true);
        else TDP_S1(4, 4, false);
    }
#undef TDP_S1
    return hipGetLastError();
}

// shape: node columns per workgroup (rows x 64) and rows per thread:
//   0 -> 4 waves x 2 rows (8 x 64), 1 -> 4 waves x 4 rows (16 x 64),
//   2 -> 8 waves x 2 rows (16 x 64); zc = planes per chunk
hipError_t launch_sweep3d_stream_f64(const SweepArgs &a, const Stencil<double> &st, double fa,
                                     double fb, int shape, int zc, hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream_t<double, 4, 2>(a, st, fa, fb, zc, s);
    case 2: return launch_stream_t<double, 8, 2>(a, st, fa, fb, zc, s);
    default: return launch_stream_t<double, 4, 4>(a, st, fa, fb, zc, s);
    }
}

hipError_t launch_sweep3d_stream_f32(const SweepArgs &a, const Stencil<float> &st, float fa,
                                     float fb, int shape, int zc, hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream_t<float, 4, 2>(a, st, fa, fb, zc, s);
    case 2: return launch_stream_t<float, 8, 2>(a, st, fa, fb, zc, s);
    default: return launch_stream_t<float, 4, 4>(a, st, fa, fb, zc, s);
    }
}

}  // namespace tdp
