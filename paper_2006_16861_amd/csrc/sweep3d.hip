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
                const T acc = stencil27<SC, MC>(U, w, st);
                const T r =
                    cd[q] * (acc + fa * cfr[q] + fb * cfi[q]) - (T(2) * cd[q] - T(1)) * cup[q];
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
// level 1 (u_{j+1}) on a 64 x RT column block with a one-node halo and level 2
// (u_{j+2}) on its 62 x (RT-2) interior, walking a z-chunk: in iteration i it
// forms level 1 on plane a = zb-1+i and level 2 on plane a-1.  Level-0 planes
// and cell planes rotate through 4-slot LDS rings (the slot freed in an
// iteration receives the plane prefetched into registers), level-1 planes
// through a 3-slot ring; u_{j-1}, d and F of plane a are fetched one iteration
// ahead and kept one iteration longer for level 2.  Per node and launch this
// reads u_j, u_{j-1}, m, d, F once and writes u_{j+1}, u_{j+2}: about 4 words
// per node-step instead of 7.  Outputs must not alias the inputs.
template <typename T, int SC, int MC, int TY, int RY, bool NTS>
__global__ __launch_bounds__(64 * TY) void k_sweep3d_stream2(
    const T *__restrict__ u, const T *__restrict__ up, T *__restrict__ u2o,
    T *__restrict__ u1o, const T *__restrict__ m, const T *__restrict__ dn,
    const typename V2s<T>::type *__restrict__ F, int nz, int ny, int nx, Stencil<T> st, T fa1,
    T fb1, T fa2, T fb2, double *__restrict__ out1, double *__restrict__ out2, int zc,
    int tiles_x, int tiles_y, int ntiles, int per_xcd)
{
    constexpr int NT = 64 * TY;
    constexpr int RT = TY * RY;              // level-1 rows (one-row halo each side)
    constexpr int OX = 62, OY = RT - 2;      // level-2 (output) block
    constexpr int EX = 66, EY = RT + 2;      // level-0 plane with its halo
    constexpr int LX = 64;                   // level-1 plane: RT x 64
    constexpr int CX = 65, CY = RT + 1;      // cell plane
    constexpr int UPT = (EY * EX + NT - 1) / NT;
    constexpr int CPT = (CY * CX + NT - 1) / NT;
    __shared__ T s0[4][EY * EX];
    __shared__ T s1[3][RT * LX];
    __shared__ T scl[4][CY * CX];
    const int id = blockIdx.x;
    const int tile = (id % 8) * per_xcd + id / 8;
    if (tile >= ntiles) return;
    const int bx = tile % tiles_x;
    const int by = (tile / tiles_x) % tiles_y;
    const int bz = tile / (tiles_x * tiles_y);
    const int x0 = bx * OX, y0 = by * OY, zb = bz * zc;
    const int ze = min(nz, zb + zc);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t plane = (int64_t)ny * nx;
    const int64_t cplane = (int64_t)(ny + 1) * (nx + 1);
    auto slot = [&](int p) { return (p - zb + 2) & 3; };     // level-0 and cell planes
    auto slot1 = [&](int p) { return (p - zb + 1) % 3; };    // level-1 planes

    T ru[UPT], rc[CPT];
    auto fetch_u = [&](int p) {
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
            const int t = threadIdx.x + q * NT;
            const int r = t / EX, c = t % EX;
            const int gy = y0 - 2 + r, gx = x0 - 2 + c;
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
            const int sy = y0 - 1 + r, sx = x0 - 1 + c;
            const bool ok = t < CY * CX && (unsigned)qz <= (unsigned)nz &&
                            (unsigned)sy <= (unsigned)ny && (unsigned)sx <= (unsigned)nx;
            rc[q] = ok ? m[qz * cplane + (int64_t)sy * (nx + 1) + sx] : T(0);
        }
    };
    auto store_u = [&](int sl) {
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
            const int t = threadIdx.x + q * NT;
            if (t < EY * EX) s0[sl][t] = ru[q];
        }
    };
    auto store_c = [&](int sl) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int t = threadIdx.x + q * NT;
            if (t < CY * CX) scl[sl][t] = rc[q];
        }
    };
    const int gx = x0 - 1 + tx;
    const bool xin = (unsigned)gx < (unsigned)nx;
    // node data of plane a (level 1), fetched one iteration ahead
    T num[RY], nd[RY], nfr[RY], nfi[RY];
    auto fetch_node = [&](int p) {
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int gy = y0 - 1 + ty + TY * q;
            num[q] = nd[q] = nfr[q] = nfi[q] = T(0);
            if (xin && (unsigned)gy < (unsigned)ny && (unsigned)p < (unsigned)nz) {
                const int64_t i = p * plane + (int64_t)gy * nx + gx;
                num[q] = ldnt<NTS>(up + i);
                nd[q] = ldnt<NTS>(dn + i);
                nfr[q] = ldnt<NTS>(&F[i].x);
                nfi[q] = ldnt<NTS>(&F[i].y);
            }
        }
    };

    // prologue: level-0 and cell planes zb-2, zb-1, zb; node data of plane zb-1
#pragma unroll 1
    for (int p = zb - 2; p <= zb; ++p) {
        fetch_u(p);
        fetch_c(p);
        store_u(slot(p));
        store_c(slot(p));
    }
    fetch_node(zb - 1);
    T pd[RY], pfr[RY], pfi[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) pd[q] = pfr[q] = pfi[q] = T(0);
    __syncthreads();
    const int iters = ze - zb + 2;
    for (int it = 0; it < iters; ++it) {
        const int a = zb - 1 + it, b = a - 1;
        T cum[RY], cd[RY], cfr[RY], cfi[RY];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            cum[q] = num[q];
            cd[q] = nd[q];
            cfr[q] = nfr[q];
            cfi[q] = nfi[q];
        }
        const bool more = it + 1 < iters;
        if (more) {                    // next iteration: planes a+2, node data of a+1
            fetch_u(a + 2);
            fetch_c(a + 2);
            fetch_node(a + 1);
        }
        // level 1 on plane a (every lane and row of the block, halo included)
        const bool ain = (unsigned)a < (unsigned)nz;
        const T *p0 = s0[slot(a - 1)], *p1 = s0[slot(a)], *p2 = s0[slot(a + 1)];
        const T *c0p = scl[slot(a)], *c1p = scl[slot(a + 1)];
        T *l1 = s1[slot1(a)];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const int ry = ty + TY * q;
            const int gy = y0 - 1 + ry;
            T v = T(0);
            if (ain && xin && (unsigned)gy < (unsigned)ny) {
                const int base = (ry + 1) * EX + tx + 1;
                auto U = [&](int oz, int oy, int ox) -> T {
                    const T *pl = oz < 0 ? p0 : (oz == 0 ? p1 : p2);
                    return pl[base + oy * EX + ox];
                };
                T w[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                    w[e] = (ez ? c1p : c0p)[(ry + ey) * CX + tx + ex];
                }
                const T acc = stencil27<SC, MC>(U, w, st);
                v = cd[q] * (acc + fa1 * cfr[q] + fb1 * cfi[q]) - (T(2) * cd[q] - T(1)) * cum[q];
                if (a >= zb && a < ze && tx >= 1 && tx < 63 && ry >= 1 && ry < RT - 1) {
                    const int64_t i = a * plane + (int64_t)gy * nx + gx;
                    stnt<NTS>(v, u1o + i);
                    if (out1) out1[2 * i] = (double)v;
                }
            }
            l1[ry * LX + tx] = v;
        }
        __syncthreads();
        // level 2 on plane b (interior of the block)
        if (it >= 2) {
            const T *q0 = s1[slot1(b - 1)], *q1 = s1[slot1(b)], *q2 = s1[slot1(b + 1)];
            const T *d0p = scl[slot(b)], *d1p = scl[slot(b + 1)];
            const T *u0c = s0[slot(b)];
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                const int ry = ty + TY * q;
                const int gy = y0 - 1 + ry;
                if (tx >= 1 && tx < 63 && ry >= 1 && ry < RT - 1 && xin &&
                    (unsigned)gy < (unsigned)ny) {
                    const int base = ry * LX + tx;
                    auto U = [&](int oz, int oy, int ox) -> T {
                        const T *pl = oz < 0 ? q0 : (oz == 0 ? q1 : q2);
                        return pl[base + oy * LX + ox];
                    };
                    T w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                        w[e] = (ez ? d1p : d0p)[(ry + ey) * CX + tx + ex];
                    }
                    const T acc = stencil27<SC, MC>(U, w, st);
                    const T uc = u0c[(ry + 1) * EX + tx + 1];
                    const T v = pd[q] * (acc + fa2 * pfr[q] + fb2 * pfi[q]) - (T(2) * pd[q] - T(1)) * uc;
                    const int64_t i = b * plane + (int64_t)gy * nx + gx;
                    stnt<NTS>(v, u2o + i);
                    if (out2) out2[2 * i] = (double)v;
                }
            }
        }
        if (more) {                    // slot of plane a-2 is free in this iteration
            store_u(slot(a + 2));
            store_c(slot(a + 2));
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            pd[q] = cd[q];
            pfr[q] = cfr[q];
            pfi[q] = cfi[q];
        }
    }
}

template <typename T, int TY, int RY>
static hipError_t launch_stream2_t(const Stream2Args &a, const Stencil<T> &st, hipStream_t s)
{
    const int nz = a.n[0], ny = a.n[1], nx = a.n[2];
    constexpr int OY = TY * RY - 2;
    const int zc = a.zc;
    const int tiles_x = (nx + 61) / 62, tiles_y = (ny + OY - 1) / OY;
    const int tiles_z = (nz + zc - 1) / zc;
    const int ntiles = tiles_x * tiles_y * tiles_z;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grd(8 * per_xcd), blk(64 * TY);
    const T *u = (const T *)a.u, *up = (const T *)a.up;
    T *u2o = (T *)a.u2out, *u1o = (T *)a.u1out;
    const T *m = (const T *)a.m, *dn = (const T *)a.dn;
    const auto *F = (const typename V2s<T>::type *)a.F;
    const T fa1 = (T)a.fa[0], fb1 = (T)a.fb[0], fa2 = (T)a.fa[1], fb2 = (T)a.fb[1];
    const bool nt = stream_nt((int64_t)7 * sizeof(T) * nz * ny * nx);
#define TDP_S2(SC, MC, NTS)                                                                           \
    hipLaunchKernelGGL((k_sweep3d_stream2<T, SC, MC, TY, RY, NTS>), grd, blk, 0, s, u, up, u2o, u1o, m, \
                       dn, F, nz, ny, nx, st, fa1, fb1, fa2, fb2, a.out1, a.out2, zc, tiles_x,        \
                       tiles_y, ntiles, per_xcd)
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

// shape: 0 -> 4 waves x 2 rows (8-row level-1 block, 6 output rows),
// 1 -> 4 waves x 4 rows (16, 14), 2 -> 8 waves x 2 rows (16, 14)
hipError_t launch_sweep3d_stream2_f64(const Stream2Args &a, const Stencil<double> &st, int shape,
                                      hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream2_t<double, 4, 2>(a, st, s);
    case 2: return launch_stream2_t<double, 8, 2>(a, st, s);
    default: return launch_stream2_t<double, 4, 4>(a, st, s);
    }
}

hipError_t launch_sweep3d_stream2_f32(const Stream2Args &a, const Stencil<float> &st, int shape,
                                      hipStream_t s)
{
    switch (shape) {
    case 0: return launch_stream2_t<float, 4, 2>(a, st, s);
    case 2: return launch_stream2_t<float, 8, 2>(a, st, s);
    default: return launch_stream2_t<float, 4, 4>(a, st, s);
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
