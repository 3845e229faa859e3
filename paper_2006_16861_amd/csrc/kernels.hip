// HIP kernels of libtdp for CDNA4 (gfx950): the fused recurrence sweep of the
// time-domain preconditioner (Table 1 with the integrator I_acd of Def. 2),
// the complex H-apply, setup kernels, Krylov BLAS-1 kernels with
// deterministic FP64 reductions, and the m-gradient contraction.
//
// Data layout: node arrays row-major [n0][n1][n2] (last axis fastest); cell
// arrays [(n0+1)][(n1+1)][(n2+1)], cell with storage index (z, y, x) has lower
// corner (z-1, y-1, x-1), so the 2^d cells around node (z, y, x) are the
// storage cells (z+ez, y+ey, x+ex), e in {0,1}^d.  In 2-D the z axis is absent
// (nz = 1, z = 0) and the two node axes are (y, x) = (axis 0, axis 1).
#include <hip/hip_runtime.h>

#include "tdp_internal.h"

namespace tdp {

template <typename T>
struct V2;
template <>
struct V2<double> {
    using type = double2;
};
template <>
struct V2<float> {
    using type = float2;
};

// complex pair of the complex-linear variant's field (re, im)
template <typename T>
struct C2 {
    T x, y;
};
template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b)
{
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> &operator+=(C2<T> &a, C2<T> b)
{
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <typename T>
__device__ __forceinline__ C2<T> operator*(T s, C2<T> a)
{
    return {s * a.x, s * a.y};
}

// ---------------------------------------------------------------------------
// assembled stencil: see Stencil<T> in tdp_internal.h.  w[e] are the 2^D
// cell values around the node, e = ex + 2 ey (+ 4 ez).  U(oz, oy, ox)
// returns the field value (T, or C2<T> for a complex field) at the offset
// node (0 outside the box).
template <int D, int SC, int MC, typename T, typename LoadU>
__device__ __forceinline__ auto eval_stencil(const LoadU &U, const T *w, const Stencil<T> &st)
{
    using V = decltype(U(0, 0, 0));
    constexpr int NC = SC > MC ? SC : MC;
    constexpr int NOFF = D == 2 ? 9 : 27;
    V us[4] = {V{}, V{}, V{}, V{}};
    V ws[4] = {V{}, V{}, V{}, V{}};
#pragma unroll
    for (int k = 0; k < NOFF; ++k) {
        const int ox = k % 3 - 1, oy = (k / 3) % 3 - 1, oz = D == 3 ? k / 9 - 1 : 0;
        const int cls = (ox != 0) + (oy != 0) + (oz != 0);
        if (cls >= NC) continue;
        const V v = U(oz, oy, ox);
        if (cls < SC || cls == 0) us[cls] += v;
        if (cls < MC) {
            T W = T(0);
#pragma unroll
            for (int e = 0; e < (1 << D); ++e) {
                const int ex = e & 1, ey = (e >> 1) & 1, ez = D == 3 ? (e >> 2) & 1 : 0;
                const bool okx = ox == 0 || (ox < 0 ? ex == 0 : ex == 1);
                const bool oky = oy == 0 || (oy < 0 ? ey == 0 : ey == 1);
                const bool okz = D == 2 || oz == 0 || (oz < 0 ? ez == 0 : ez == 1);
                if (okx && oky && okz) W += w[e];
            }
            ws[cls] += W * v;
        }
    }
    V r = st.c0 * us[0];
#pragma unroll
    for (int k = 1; k < SC; ++k) r += st.s[k] * us[k];
#pragma unroll
    for (int k = 0; k < MC; ++k) r += st.m[k] * ws[k];
    return r;
}

template <int D, typename T>
__device__ __forceinline__ void load_cells(const T *__restrict__ m, int z, int y, int x, int ny,
                                           int nx, T *w)
{
    const int64_t cy = nx + 1, cz = (int64_t)(ny + 1) * (nx + 1);
    const int64_t c = (int64_t)z * cz + (int64_t)y * cy + x;
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        w[e] = m[c + ez * cz + ey * cy + ex];
    }
}

// ---------------------------------------------------------------------------
// one recurrence step (Def. 2 with the Table 1 forcing), one node per thread:
//   u_{j+1} = d (S[u_j] + fa Re F + fb Im F) - (2d - 1) u_{j-1},
// S[.] the stencil with the step constants (it equals (2 - K) u), d = 1/(1+l/2).
// u_{j+1} overwrites u_{j-1} in place.
template <int D, int SC, int MC, typename T, bool NT>
__global__ __launch_bounds__(256) void k_sweep(const T *__restrict__ u, T *__restrict__ up,
                                               const T *__restrict__ m,
                                               const T *__restrict__ dn,
                                               const typename V2<T>::type *__restrict__ F,
                                               int nz, int ny, int nx, Stencil<T> st, T fa,
                                               T fb, double *__restrict__ out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t i = ((int64_t)z * ny + y) * nx + x;
    T w[1 << D];
    load_cells<D>(m, z, y, x, ny, nx, w);
    auto U = [&](int oz, int oy, int ox) -> T {
        const bool in = (unsigned)(y + oy) < (unsigned)ny && (unsigned)(x + ox) < (unsigned)nx &&
                        (D == 2 || (unsigned)(z + oz) < (unsigned)nz);
        return in ? u[i + ((int64_t)oz * ny + oy) * nx + ox] : T(0);
    };
    const T acc = eval_stencil<D, SC, MC>(U, w, st);
    // per-node streams (read / written once per step; see stream_nt)
    const T fx = ldnt<NT>(&F[i].x), fy = ldnt<NT>(&F[i].y);
    const T d = ldnt<NT>(dn + i);
    const T r = d * (acc + fa * fx + fb * fy) - (T(2) * d - T(1)) * ldnt<NT>(up + i);
    stnt<NT>(r, up + i);
    if (out) out[2 * i] = (double)r;
}

// 2-D form of the same step for grids beyond the MALL: a thread updates RY
// consecutive rows of one column (a workgroup 64 columns x WV * RY rows), so
// each u row and cell row it loads serves up to three of its updates and the
// rows shared with the workgroups above and below are RY * WV apart instead
// of 4 (less halo re-read from HBM).
template <int SC, int MC, typename T, bool NT, int RY>
__global__ __launch_bounds__(256) void k_sweep2d_col(const T *__restrict__ u, T *__restrict__ up,
                                                     const T *__restrict__ m,
                                                     const T *__restrict__ dn,
                                                     const typename V2<T>::type *__restrict__ F,
                                                     int ny, int nx, Stencil<T> st, T fa, T fb,
                                                     double *__restrict__ out)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * RY;
    if (x >= nx || y0 >= ny) return;
    // u at rows y0-1 .. y0+RY, columns x-1, x, x+1; cells at rows y0 .. y0+RY,
    // columns x, x+1 (0 outside the box)
    T uv[RY + 2][3], cv[RY + 1][2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int y = y0 - 1 + r;
        const bool yin = (unsigned)y < (unsigned)ny;
        const T *row = u + (int64_t)y * nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int xx = x - 1 + c;
            uv[r][c] = (yin && (unsigned)xx < (unsigned)nx) ? row[xx] : T(0);
        }
    }
#pragma unroll
    for (int r = 0; r < RY + 1; ++r) {
        const int y = y0 + r;
        const T *row = m + (int64_t)y * (nx + 1);
        const bool yin = y <= ny;
        cv[r][0] = yin ? row[x] : T(0);
        cv[r][1] = yin ? row[x + 1] : T(0);
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        if (y >= ny) break;
        const int64_t i = (int64_t)y * nx + x;
        const T w[4] = {cv[r][0], cv[r][1], cv[r + 1][0], cv[r + 1][1]};
        auto U = [&](int, int oy, int ox) -> T { return uv[r + 1 + oy][1 + ox]; };
        const T acc = eval_stencil<2, SC, MC>(U, w, st);
        const T fx = ldnt<NT>(&F[i].x), fy = ldnt<NT>(&F[i].y);
        const T d = ldnt<NT>(dn + i);
        const T res = d * (acc + fa * fx + fb * fy) - (T(2) * d - T(1)) * ldnt<NT>(up + i);
        stnt<NT>(res, up + i);
        if (out) out[2 * i] = (double)res;
    }
}

template <typename T>
static hipError_t launch_sweep_t(const SweepArgs &a, const Stencil<T> &st, T fa, T fb,
                                 hipStream_t s)
{
    const int nz = a.ndim == 3 ? a.n[0] : 1;
    const int ny = a.ndim == 3 ? a.n[1] : a.n[0];
    const int nx = a.ndim == 3 ? a.n[2] : a.n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 63) / 64, (ny + 3) / 4, nz);
    const T *u = (const T *)a.u;
    T *up = (T *)a.up;
    const T *m = (const T *)a.m;
    const T *dn = (const T *)a.dn;
    const auto *F = (const typename V2<T>::type *)a.F;
    const bool nt = stream_nt((int64_t)7 * sizeof(T) * nz * ny * nx);
#define TDP_SWEEP(D, SC, MC)                                                                           \
    do {                                                                                            \
        if (nt)                                                                                     \
            hipLaunchKernelGGL((k_sweep<D, SC, MC, T, true>), grd, blk, 0, s, u, up, m, dn, F, nz, ny, nx, st, fa, fb, a.out);  \
        else                                                                                        \
            hipLaunchKernelGGL((k_sweep<D, SC, MC, T, false>), grd, blk, 0, s, u, up, m, dn, F, nz, ny, nx, st, fa, fb, a.out); \
    } while (0)
    if (a.ndim == 2 && nt) {
        // beyond the MALL: RY rows per thread (fewer halo re-reads from HBM)
        constexpr int RY = 4;
        dim3 cgrd((nx + 63) / 64, (ny + 4 * RY - 1) / (4 * RY), 1);
        if (a.sc <= 3 && a.mc <= 2)
            hipLaunchKernelGGL((k_sweep2d_col<3, 2, T, true, RY>), cgrd, dim3(256), 0, s, u, up, m,
                               dn, F, ny, nx, st, fa, fb, a.out);
        else
            hipLaunchKernelGGL((k_sweep2d_col<3, 3, T, true, RY>), cgrd, dim3(256), 0, s, u, up, m,
                               dn, F, ny, nx, st, fa, fb, a.out);
    } else if (a.ndim == 2) {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEP(2, 3, 2);
        else TDP_SWEEP(2, 3, 3);
    } else {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEP(3, 3, 2);
        else TDP_SWEEP(3, 4, 4);
    }
#undef TDP_SWEEP
    return hipGetLastError();
}

hipError_t launch_sweep_f64(const SweepArgs &a, const Stencil<double> &st, double fa, double fb,
                            hipStream_t s)
{
    return launch_sweep_t<double>(a, st, fa, fb, s);
}

hipError_t launch_sweep_f32(const SweepArgs &a, const Stencil<float> &st, float fa, float fb,
                            hipStream_t s)
{
    return launch_sweep_t<float>(a, st, fa, fb, s);
}

// ---------------------------------------------------------------------------
// complex-linear variant (Definition 4): complex field u driven by the complex
// forcing g chi_j e^{i phi_j} F; (fa, fb) = g chi_j (cos phi_j, sin phi_j).
//   u_{j+1} = d (S[u_j] + (fa + i fb) F) - (2d - 1) u_{j-1}
template <int D, int SC, int MC, typename T, bool NT>
__global__ __launch_bounds__(256) void k_sweep_c(const C2<T> *__restrict__ u,
                                                 C2<T> *__restrict__ up,
                                                 const T *__restrict__ m,
                                                 const T *__restrict__ dn,
                                                 const typename V2<T>::type *__restrict__ F,
                                                 int nz, int ny, int nx, Stencil<T> st, T fa,
                                                 T fb, double2 *__restrict__ out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t i = ((int64_t)z * ny + y) * nx + x;
    T w[1 << D];
    load_cells<D>(m, z, y, x, ny, nx, w);
    auto U = [&](int oz, int oy, int ox) -> C2<T> {
        const bool in = (unsigned)(y + oy) < (unsigned)ny && (unsigned)(x + ox) < (unsigned)nx &&
                        (D == 2 || (unsigned)(z + oz) < (unsigned)nz);
        return in ? u[i + ((int64_t)oz * ny + oy) * nx + ox] : C2<T>{T(0), T(0)};
    };
    const C2<T> acc = eval_stencil<D, SC, MC>(U, w, st);
    const T fx = ldnt<NT>(&F[i].x), fy = ldnt<NT>(&F[i].y);
    const auto f = typename V2<T>::type{fx, fy};
    const T d = ldnt<NT>(dn + i), e = T(2) * d - T(1);
    const C2<T> p = {ldnt<NT>(&up[i].x), ldnt<NT>(&up[i].y)};
    C2<T> r;
    r.x = d * (acc.x + fa * f.x - fb * f.y) - e * p.x;
    r.y = d * (acc.y + fa * f.y + fb * f.x) - e * p.y;
    stnt<NT>(r.x, &up[i].x);
    stnt<NT>(r.y, &up[i].y);
    if (out) out[i] = make_double2((double)r.x, (double)r.y);
}

template <typename T>
static hipError_t launch_sweep_c_t(const SweepArgs &a, const Stencil<T> &st, T fa, T fb,
                                   hipStream_t s)
{
    const int nz = a.ndim == 3 ? a.n[0] : 1;
    const int ny = a.ndim == 3 ? a.n[1] : a.n[0];
    const int nx = a.ndim == 3 ? a.n[2] : a.n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 63) / 64, (ny + 3) / 4, nz);
    const C2<T> *u = (const C2<T> *)a.u;
    C2<T> *up = (C2<T> *)a.up;
    const T *m = (const T *)a.m;
    const T *dn = (const T *)a.dn;
    const auto *F = (const typename V2<T>::type *)a.F;
    double2 *out = (double2 *)a.out;
    const bool nt = stream_nt((int64_t)10 * sizeof(T) * nz * ny * nx);
#define TDP_SWEEPC(D, SC, MC)                                                                          \
    do {                                                                                            \
        if (nt)                                                                                     \
            hipLaunchKernelGGL((k_sweep_c<D, SC, MC, T, true>), grd, blk, 0, s, u, up, m, dn, F, nz, ny, nx, st, fa, fb, out);  \
        else                                                                                        \
            hipLaunchKernelGGL((k_sweep_c<D, SC, MC, T, false>), grd, blk, 0, s, u, up, m, dn, F, nz, ny, nx, st, fa, fb, out); \
    } while (0)
    if (a.ndim == 2) {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEPC(2, 3, 2);
        else TDP_SWEEPC(2, 3, 3);
    } else {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEPC(3, 3, 2);
        else TDP_SWEEPC(3, 4, 4);
    }
#undef TDP_SWEEPC
    return hipGetLastError();
}

hipError_t launch_sweep_c_f64(const SweepArgs &a, const Stencil<double> &st, double fa,
                              double fb, hipStream_t s)
{
    return launch_sweep_c_t<double>(a, st, fa, fb, s);
}

hipError_t launch_sweep_c_f32(const SweepArgs &a, const Stencil<float> &st, float fa, float fb,
                              hipStream_t s)
{
    return launch_sweep_c_t<float>(a, st, fa, fb, s);
}

// ---------------------------------------------------------------------------
// frequency adapted backward-differences damped leapfrog I_abd (Sec. 6, Def. 6)
// on the complex field of S_T^abd (Def. 7), for the cell damping
// Im H = omega sum_cells r_cell M_cell:
//   u_{n+1} = (2 - K - L) u_n - (I - L) u_{n-1} + g f_n
//           = stA[u_n] + stB_r[u_{n-1} - cos(omega dt) u_n] - u_{n-1} + (fa + i fb) F,
// stA the I_acd step stencil (2 - (dt^2/alpha) A) over the cell slowness, stB_r
// the mass-class stencil of (beta dt/(alpha omega)) Im H over the cell damping.
// u_{n-1} is read at the neighbours too, so u_{n+1} goes to a third field.
template <int D, int SC, int MC, typename T, bool NT>
__global__ __launch_bounds__(256) void k_sweep_abd(const C2<T> *__restrict__ u,
                                                   const C2<T> *__restrict__ um,
                                                   C2<T> *__restrict__ uo,
                                                   const T *__restrict__ m,
                                                   const T *__restrict__ rc,
                                                   const typename V2<T>::type *__restrict__ F,
                                                   int nz, int ny, int nx, Stencil<T> stA,
                                                   Stencil<T> stB, T cth, T fa, T fb,
                                                   double2 *__restrict__ out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t i = ((int64_t)z * ny + y) * nx + x;
    T wm[1 << D], wr[1 << D];
    load_cells<D>(m, z, y, x, ny, nx, wm);
    load_cells<D>(rc, z, y, x, ny, nx, wr);
    auto inside = [&](int oz, int oy, int ox) -> bool {
        return (unsigned)(y + oy) < (unsigned)ny && (unsigned)(x + ox) < (unsigned)nx &&
               (D == 2 || (unsigned)(z + oz) < (unsigned)nz);
    };
    auto U = [&](int oz, int oy, int ox) -> C2<T> {
        return inside(oz, oy, ox) ? u[i + ((int64_t)oz * ny + oy) * nx + ox] : C2<T>{T(0), T(0)};
    };
    auto W = [&](int oz, int oy, int ox) -> C2<T> {
        if (!inside(oz, oy, ox)) return C2<T>{T(0), T(0)};
        const int64_t j = i + ((int64_t)oz * ny + oy) * nx + ox;
        const C2<T> a = um[j], b = u[j];
        return C2<T>{a.x - cth * b.x, a.y - cth * b.y};
    };
    const C2<T> acc = eval_stencil<D, SC, MC>(U, wm, stA);
    const C2<T> dmp = eval_stencil<D, 1, MC>(W, wr, stB);
    const T fx = ldnt<NT>(&F[i].x), fy = ldnt<NT>(&F[i].y);
    const C2<T> p = um[i];
    C2<T> r;
    r.x = acc.x + dmp.x - p.x + fa * fx - fb * fy;
    r.y = acc.y + dmp.y - p.y + fa * fy + fb * fx;
    stnt<NT>(r.x, &uo[i].x);
    stnt<NT>(r.y, &uo[i].y);
    if (out) out[i] = make_double2((double)r.x, (double)r.y);
}

template <typename T>
static hipError_t launch_sweep_abd_t(const SweepArgs &a, void *uout, const T *rc,
                                     const Stencil<T> &stA, const Stencil<T> &stB, T cth, T fa,
                                     T fb, hipStream_t s)
{
    const int nz = a.ndim == 3 ? a.n[0] : 1;
    const int ny = a.ndim == 3 ? a.n[1] : a.n[0];
    const int nx = a.ndim == 3 ? a.n[2] : a.n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 63) / 64, (ny + 3) / 4, nz);
    const C2<T> *u = (const C2<T> *)a.u;
    const C2<T> *um = (const C2<T> *)a.up;
    C2<T> *uo = (C2<T> *)uout;
    const T *m = (const T *)a.m;
    const auto *F = (const typename V2<T>::type *)a.F;
    double2 *out = (double2 *)a.out;
    const bool nt = stream_nt((int64_t)10 * sizeof(T) * nz * ny * nx);
#define TDP_SWEEPB(D, SC, MC)                                                                          \
    do {                                                                                            \
        if (nt)                                                                                     \
            hipLaunchKernelGGL((k_sweep_abd<D, SC, MC, T, true>), grd, blk, 0, s, u, um, uo, m, rc, F, nz, ny, nx, stA, stB, cth, fa, fb, out);  \
        else                                                                                        \
            hipLaunchKernelGGL((k_sweep_abd<D, SC, MC, T, false>), grd, blk, 0, s, u, um, uo, m, rc, F, nz, ny, nx, stA, stB, cth, fa, fb, out); \
    } while (0)
    if (a.ndim == 2) {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEPB(2, 3, 2);
        else TDP_SWEEPB(2, 3, 3);
    } else {
        if (a.sc <= 3 && a.mc <= 2) TDP_SWEEPB(3, 3, 2);
        else TDP_SWEEPB(3, 4, 4);
    }
#undef TDP_SWEEPB
    return hipGetLastError();
}

hipError_t launch_sweep_abd_f64(const SweepArgs &a, void *uout, const double *rc,
                                const Stencil<double> &stA, const Stencil<double> &stB,
                                double cth, double fa, double fb, hipStream_t s)
{
    return launch_sweep_abd_t<double>(a, uout, rc, stA, stB, cth, fa, fb, s);
}

hipError_t launch_sweep_abd_f32(const SweepArgs &a, void *uout, const float *rc,
                                const Stencil<float> &stA, const Stencil<float> &stB, float cth,
                                float fa, float fb, hipStream_t s)
{
    return launch_sweep_abd_t<float>(a, uout, rc, stA, stB, cth, fa, fb, s);
}

// ---------------------------------------------------------------------------
// complex H-apply: y = H x or y = F - H x, H = stencil + i diag(rw)
// With the cell damping (CD), Im H = omega sum_cells r_cell M_cell is the
// mass-class stencil stI over the cell damping rc instead of diag(rw).
template <int D, int SC, int MC, bool CD, bool NT>
__device__ __forceinline__ double2 apply_H_at(const double *__restrict__ m,
                                              const double *__restrict__ rw,
                                              const double *__restrict__ rc,
                                              const Stencil<double> &st, const Stencil<double> &stI,
                                              const double2 *__restrict__ xv,
                                              const double2 *__restrict__ F, int z, int y, int x,
                                              int64_t i, int nz, int ny, int nx)
{
    double w[1 << D];
    load_cells<D>(m, z, y, x, ny, nx, w);
    const double *xs = (const double *)xv;
    auto Ur = [&](int oz, int oy, int ox) -> double {
        const bool in = (unsigned)(y + oy) < (unsigned)ny && (unsigned)(x + ox) < (unsigned)nx &&
                        (D == 2 || (unsigned)(z + oz) < (unsigned)nz);
        return in ? xs[2 * (i + ((int64_t)oz * ny + oy) * nx + ox)] : 0.0;
    };
    auto Ui = [&](int oz, int oy, int ox) -> double {
        const bool in = (unsigned)(y + oy) < (unsigned)ny && (unsigned)(x + ox) < (unsigned)nx &&
                        (D == 2 || (unsigned)(z + oz) < (unsigned)nz);
        return in ? xs[2 * (i + ((int64_t)oz * ny + oy) * nx + ox) + 1] : 0.0;
    };
    const double hr = eval_stencil<D, SC, MC>(Ur, w, st);
    const double hi = eval_stencil<D, SC, MC>(Ui, w, st);
    double2 o;
    if (CD) {
        double wr[1 << D];
        load_cells<D>(rc, z, y, x, ny, nx, wr);
        o.x = hr - eval_stencil<D, 1, MC>(Ui, wr, stI);
        o.y = hi + eval_stencil<D, 1, MC>(Ur, wr, stI);
    } else {
        const double2 xc = xv[i];
        const double r = rw[i];
        o.x = hr - r * xc.y;
        o.y = hi + r * xc.x;
    }
    if (F) {
        o.x = ldnt<NT>(&F[i].x) - o.x;
        o.y = ldnt<NT>(&F[i].y) - o.y;
    }
    return o;
}

template <int D, int SC, int MC, bool CD, bool NT>
__global__ __launch_bounds__(256) void k_apply_H(const double *__restrict__ m,
                                                 const double *__restrict__ rw,
                                                 const double *__restrict__ rc,
                                                 Stencil<double> st, Stencil<double> stI,
                                                 const double2 *__restrict__ xv,
                                                 const double2 *__restrict__ F,
                                                 double2 *__restrict__ y_out, int nz, int ny,
                                                 int nx)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t i = ((int64_t)z * ny + y) * nx + x;
    const double2 o = apply_H_at<D, SC, MC, CD, NT>(m, rw, rc, st, stI, xv, F, z, y, x, i, nz, ny, nx);
    stnt<NT>(o.x, &y_out[i].x);
    stnt<NT>(o.y, &y_out[i].y);
}

hipError_t launch_apply_H(int ndim, const int *n, int sc, int mc, const double *m,
                          const double *rw, const double *rc, const Stencil<double> &st,
                          const Stencil<double> &stI, const void *x, const void *F, void *y,
                          hipStream_t s)
{
    const int nz = ndim == 3 ? n[0] : 1;
    const int ny = ndim == 3 ? n[1] : n[0];
    const int nx = ndim == 3 ? n[2] : n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 63) / 64, (ny + 3) / 4, nz);
    const double2 *xv = (const double2 *)x;
    const double2 *Fv = (const double2 *)F;
    double2 *yv = (double2 *)y;
    const bool nt = stream_nt((int64_t)56 * nz * ny * nx);
#define TDP_HAPPLY(D, SC, MC, CD)                                                                      \
    do {                                                                                            \
        if (nt)                                                                                     \
            hipLaunchKernelGGL((k_apply_H<D, SC, MC, CD, true>), grd, blk, 0, s, m, rw, rc, st, stI, xv, Fv, yv, nz, ny, nx);  \
        else                                                                                        \
            hipLaunchKernelGGL((k_apply_H<D, SC, MC, CD, false>), grd, blk, 0, s, m, rw, rc, st, stI, xv, Fv, yv, nz, ny, nx); \
    } while (0)
#define TDP_HAPPLY2(D, SC, MC) \
    do { if (rc) TDP_HAPPLY(D, SC, MC, true); else TDP_HAPPLY(D, SC, MC, false); } while (0)
    if (ndim == 2) {
        if (sc <= 3 && mc <= 2) TDP_HAPPLY2(2, 3, 2);
        else TDP_HAPPLY2(2, 3, 3);
    } else {
        if (sc <= 3 && mc <= 2) TDP_HAPPLY2(3, 3, 2);
        else TDP_HAPPLY2(3, 4, 4);
    }
#undef TDP_HAPPLY2
#undef TDP_HAPPLY
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise helpers
__global__ void k_fill_zero(uint32_t *p, int64_t nwords)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

static int grid_for(int64_t n, int per_block = 256)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t nw = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(nw)), dim3(256), 0, s, (uint32_t *)p, nw);
    return hipGetLastError();
}

__global__ void k_cvt_c128_c64(const double2 *__restrict__ a, float2 *__restrict__ b, int64_t N)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = a[i];
        b[i] = make_float2((float)v.x, (float)v.y);
    }
}

hipError_t launch_cvt_c128_to_c64(const void *F, void *Fs, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_cvt_c128_c64, dim3(grid_for(N)), dim3(256), 0, s, (const double2 *)F,
                       (float2 *)Fs, N);
    return hipGetLastError();
}

// Table 1 with 4 not dividing n_P: U.y holds u_{N_s - q}, a sample a phase
// phi = 2 pi q / n_P before U.x = u_{N_s}; the time-harmonic field gives
// u_{N_s - q} = cos(phi) Re U + sin(phi) Im U, solved here for Im U.
__global__ void k_phase_extract(double2 *__restrict__ U, int64_t N, double c, double s)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = U[i];
        U[i] = make_double2(v.x, (v.y - c * v.x) / s);
    }
}

hipError_t launch_phase_extract(void *U, int64_t N, double c, double s, hipStream_t st)
{
    hipLaunchKernelGGL(k_phase_extract, dim3(grid_for(N)), dim3(256), 0, st, (double2 *)U, N, c, s);
    return hipGetLastError();
}

__global__ void k_cvt_f64_f32(const double *__restrict__ a, float *__restrict__ b, int64_t N)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

hipError_t launch_cvt_f64_to_f32(const double *x, float *y, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_cvt_f64_f32, dim3(grid_for(N)), dim3(256), 0, s, x, y, N);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// setup: m_cell = 2^-D sum over corners of 1/c^2 (corner indices clamped);
// with INV = false the plain corner mean (cell damping r_cell from R).
template <int D, bool INV>
__global__ void k_cell_slowness(const double *__restrict__ c, double *__restrict__ m, int nz,
                                int ny, int nx)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;   // storage 0..nx
    const int y = blockIdx.y * blockDim.y + threadIdx.y;   // storage 0..ny
    const int z = blockIdx.z;                              // storage 0..nz (3-D)
    if (x > nx || y > ny) return;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        int cx = x - 1 + ex, cy = y - 1 + ey, cz = D == 3 ? z - 1 + ez : 0;
        cx = cx < 0 ? 0 : (cx >= nx ? nx - 1 : cx);
        cy = cy < 0 ? 0 : (cy >= ny ? ny - 1 : cy);
        cz = cz < 0 ? 0 : (cz >= nz ? nz - 1 : cz);
        const double v = c[((int64_t)cz * ny + cy) * nx + cx];
        s += INV ? 1.0 / (v * v) : v;
    }
    m[((int64_t)z * (ny + 1) + y) * (nx + 1) + x] = s * (1.0 / (1 << D));
}

hipError_t launch_cell_slowness(int ndim, const int *n, const double *c, double *m,
                                hipStream_t s)
{
    const int nz = ndim == 3 ? n[0] : 1;
    const int ny = ndim == 3 ? n[1] : n[0];
    const int nx = ndim == 3 ? n[2] : n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 1 + 63) / 64, (ny + 1 + 3) / 4, ndim == 3 ? nz + 1 : 1);
    if (ndim == 2)
        hipLaunchKernelGGL((k_cell_slowness<2, true>), grd, blk, 0, s, c, m, nz, ny, nx);
    else
        hipLaunchKernelGGL((k_cell_slowness<3, true>), grd, blk, 0, s, c, m, nz, ny, nx);
    return hipGetLastError();
}

hipError_t launch_cell_mean(int ndim, const int *n, const double *v, double *cells,
                            hipStream_t s)
{
    const int nz = ndim == 3 ? n[0] : 1;
    const int ny = ndim == 3 ? n[1] : n[0];
    const int nx = ndim == 3 ? n[2] : n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 1 + 63) / 64, (ny + 1 + 3) / 4, ndim == 3 ? nz + 1 : 1);
    if (ndim == 2)
        hipLaunchKernelGGL((k_cell_slowness<2, false>), grd, blk, 0, s, v, cells, nz, ny, nx);
    else
        hipLaunchKernelGGL((k_cell_slowness<3, false>), grd, blk, 0, s, v, cells, nz, ny, nx);
    return hipGetLastError();
}

// wave64 + LDS block reductions (blockDim.x == 256)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

__global__ __launch_bounds__(256) void k_max_partial(const double *__restrict__ x, int64_t N,
                                                     double *__restrict__ partial)
{
    __shared__ double sm[4];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        v = fmax(v, x[i]);
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

__global__ __launch_bounds__(256) void k_max_final(const double *__restrict__ partial, int nblk,
                                                   double *__restrict__ out)
{
    __shared__ double sm[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) v = fmax(v, partial[i]);
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

hipError_t launch_max_reduce(const double *x, int64_t N, double *partial, int nblk,
                             double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_max_partial, dim3(nblk), dim3(256), 0, s, x, N, partial);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, partial, nblk, out);
    return hipGetLastError();
}

// rw = omega R,  dn = 1 / (1 + l/2) with l = lscale R   (L of Def. 2)
__global__ void k_node_factors(const double *__restrict__ R, int64_t N, double omega,
                               double lscale, double *__restrict__ rw, double *__restrict__ dn)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = R ? R[i] : 0.0;
        rw[i] = omega * r;
        dn[i] = 1.0 / (1.0 + 0.5 * lscale * r);
    }
}

hipError_t launch_node_factors(const double *R, int64_t N, double omega, double lscale,
                               double *rw, double *dn, hipStream_t s)
{
    hipLaunchKernelGGL(k_node_factors, dim3(grid_for(N)), dim3(256), 0, s, R, N, omega, lscale,
                       rw, dn);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov BLAS-1 (complex128).  Reductions: per-block partial sums in a fixed
// order, then one block per output sums the partials in a fixed order, so
// results are bitwise reproducible run to run.
int blas_nblocks(int64_t N)
{
    int64_t b = (N + 1023) / 1024;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

__global__ __launch_bounds__(256) void k_mdot_partial(const double2 *__restrict__ V, int64_t ldv,
                                                      const double2 *__restrict__ w, int64_t N,
                                                      double *__restrict__ partial)
{
    __shared__ double sm[8];
    const int k = blockIdx.y;
    const double2 *v = V + (int64_t)k * ldv;
    double re = 0.0, im = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = v[i], b = w[i];
        re += a.x * b.x + a.y * b.y;     // conj(a) * b
        im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* p = partial + 2 * ((int64_t)k * gridDim.x + blockIdx.x);
        p[0] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        p[1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

__global__ __launch_bounds__(256) void k_mdot_final(const double *__restrict__ partial, int nblk,
                                                    double *__restrict__ out)
{
    __shared__ double sm[8];
    const int k = blockIdx.x;
    const double *p = partial + 2 * (int64_t)k * nblk;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        re += p[2 * i];
        im += p[2 * i + 1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * k] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        out[2 * k + 1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

hipError_t launch_mdot(const void *V, int64_t ldv, int nv, const void *w, int64_t N,
                       double *partial, int nblk, double *out, hipStream_t s)
{
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdot_partial, dim3(nblk, nv), dim3(256), 0, s, (const double2 *)V, ldv,
                       (const double2 *)w, N, partial);
    hipLaunchKernelGGL(k_mdot_final, dim3(nv), dim3(256), 0, s, partial, nblk, out);
    return hipGetLastError();
}

// w += sign * sum_k coef[k] V_k   (coef: device complex128 [nv])
__global__ __launch_bounds__(256) void k_maxpy(double2 *__restrict__ w,
                                               const double2 *__restrict__ V, int64_t ldv,
                                               int nv, const double *__restrict__ coef,
                                               double sign, int64_t N)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < nv; ++k) {
            const double2 v = V[(int64_t)k * ldv + i];
            const double cr = coef[2 * k], ci = coef[2 * k + 1];
            re += cr * v.x - ci * v.y;
            im += cr * v.y + ci * v.x;
        }
        double2 o = w[i];
        o.x += sign * re;
        o.y += sign * im;
        w[i] = o;
    }
}

hipError_t launch_maxpy(void *w, const void *V, int64_t ldv, int nv, const double *coef,
                        double sign, int64_t N, hipStream_t s)
{
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_maxpy, dim3(grid_for(N)), dim3(256), 0, s, (double2 *)w,
                       (const double2 *)V, ldv, nv, coef, sign, N);
    return hipGetLastError();
}

__global__ void k_scale_invnorm(double2 *v, const double2 *w,
                                const double *__restrict__ nrm2, int64_t N)
{
    const double s = 1.0 / sqrt(nrm2[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = w[i];
        v[i] = make_double2(a.x * s, a.y * s);
    }
}

hipError_t launch_scale_by_invnorm(void *v, const void *w, const double *nrm2, int64_t N,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_invnorm, dim3(grid_for(N)), dim3(256), 0, s, (double2 *)v,
                       (const double2 *)w, nrm2, N);
    return hipGetLastError();
}

// One CGS2 step of several fields at once (the lockstep GMRES of the batched
// form), as the kernels above would do it field by field: h1 = V^H w,
// w -= V h1, h2 = V^H w, w -= V h2, |w|^2, v_next = w / |w|, then each
// field's coefficients are gathered for one copy to the host.  Block z (or
// y) is the field; a field's reductions use its own block count and order,
// so the results equal the single-field kernels' bit for bit.
__global__ __launch_bounds__(256) void k_gs_dot_partial(const GsField *__restrict__ gf, int self)
{
    __shared__ double sm[8];
    const GsField g = gf[blockIdx.z];
    const int k = blockIdx.y, nv = self ? 1 : g.nv;
    if ((int)blockIdx.x >= g.nblk || k >= nv) return;
    const double2 *v = self ? g.w : g.V + (int64_t)k * g.N;
    const double2 *w = g.w;
    double re = 0.0, im = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N;
         i += (int64_t)g.nblk * blockDim.x) {
        const double2 a = v[i], b = w[i];
        re += a.x * b.x + a.y * b.y;     // conj(a) * b
        im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *p = g.red + 2 * ((int64_t)k * g.nblk + blockIdx.x);
        p[0] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        p[1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

// which: 0 -> h1, 1 -> h2, 2 -> |w|^2 (one value)
__global__ __launch_bounds__(256) void k_gs_dot_final(const GsField *__restrict__ gf, int which)
{
    __shared__ double sm[8];
    const GsField g = gf[blockIdx.y];
    const int k = blockIdx.x, nv = which == 2 ? 1 : g.nv;
    if (k >= nv) return;
    const double *p = g.red + 2 * (int64_t)k * g.nblk;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < g.nblk; i += blockDim.x) {
        re += p[2 * i];
        im += p[2 * i + 1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *out = g.co + (which == 0 ? 0 : which == 1 ? g.off2 : g.offn);
        out[2 * k] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        out[2 * k + 1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

// w -= V h (which: 0 -> h1, 1 -> h2)
__global__ __launch_bounds__(256) void k_gs_axpy(const GsField *__restrict__ gf, int which)
{
    const GsField g = gf[blockIdx.y];
    const double *coef = g.co + (which == 0 ? 0 : g.off2);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < g.nv; ++k) {
            const double2 v = g.V[(int64_t)k * g.N + i];
            const double cr = coef[2 * k], ci = coef[2 * k + 1];
            re += cr * v.x - ci * v.y;
            im += cr * v.y + ci * v.x;
        }
        double2 o = g.w[i];
        o.x += -1.0 * re;
        o.y += -1.0 * im;
        g.w[i] = o;
    }
}

__global__ __launch_bounds__(256) void k_gs_scale(const GsField *__restrict__ gf)
{
    const GsField g = gf[blockIdx.y];
    const double sc = 1.0 / sqrt(g.co[g.offn]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = g.w[i];
        g.vnext[i] = make_double2(a.x * sc, a.y * sc);
    }
}

__global__ __launch_bounds__(256) void k_gs_gather(const GsField *__restrict__ gf)
{
    const GsField g = gf[blockIdx.x];
    for (int i = threadIdx.x; i < g.ncopy; i += blockDim.x) g.gather[i] = g.co[i];
}

hipError_t launch_gs_step_multi(const GsField *gf, int nf, int nv_max, int nblk_max,
                                int64_t n_max, hipStream_t s)
{
    if (nf <= 0) return hipSuccess;
    if (nf > 65535 || nv_max > 65535) return hipErrorInvalidValue;
    const dim3 gp(nblk_max, nv_max, nf), gn(nblk_max, 1, nf), ga(grid_for(n_max), nf);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_gs_dot_partial, gp, dim3(256), 0, s, gf, 0);
        hipLaunchKernelGGL(k_gs_dot_final, dim3(nv_max, nf), dim3(256), 0, s, gf, pass);
        hipLaunchKernelGGL(k_gs_axpy, ga, dim3(256), 0, s, gf, pass);
    }
    hipLaunchKernelGGL(k_gs_dot_partial, gn, dim3(256), 0, s, gf, 1);
    hipLaunchKernelGGL(k_gs_dot_final, dim3(1, nf), dim3(256), 0, s, gf, 2);
    hipLaunchKernelGGL(k_gs_scale, ga, dim3(256), 0, s, gf);
    hipLaunchKernelGGL(k_gs_gather, dim3(nf), dim3(256), 0, s, gf);
    return hipGetLastError();
}

// The other per-field steps of the lockstep GMRES, for several 2-D fields
// at once (block z or y is the field), each as the single-field kernels
// would do it: x_out = x_in + V y (a copy and k_maxpy), r = F - H xh or
// r = H xh (k_apply_H), |r|^2 (launch_mdot with the field's own block
// count), so the results equal the field-by-field path bit for bit.
__global__ __launch_bounds__(256) void k_tr_update(const TrField *__restrict__ tf)
{
    const TrField g = tf[blockIdx.y];
    if (g.k <= 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < g.k; ++k) {
            const double2 v = g.V[(int64_t)k * g.N + i];
            const double cr = g.y[2 * k], ci = g.y[2 * k + 1];
            re += cr * v.x - ci * v.y;
            im += cr * v.y + ci * v.x;
        }
        double2 o = g.x_in[i];
        o.x += 1.0 * re;
        o.y += 1.0 * im;
        g.x_out[i] = o;
    }
}

template <int SC, int MC>
__global__ __launch_bounds__(256) void k_tr_H(const TrField *__restrict__ tf)
{
    const TrField &g = tf[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int ny = g.ny, nx = g.nx;
    if (x >= nx || y >= ny) return;
    const int64_t i = (int64_t)y * nx + x;
    g.r[i] = apply_H_at<2, SC, MC, false, false>(g.m, g.rw, nullptr, g.st, g.st, g.xh, g.F, 0, y,
                                                 x, i, 1, ny, nx);
}

__global__ __launch_bounds__(256) void k_tr_norm_partial(const TrField *__restrict__ tf)
{
    __shared__ double sm[8];
    const TrField g = tf[blockIdx.y];
    if (!g.out || (int)blockIdx.x >= g.nblk) return;
    double re = 0.0, im = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N;
         i += (int64_t)g.nblk * blockDim.x) {
        const double2 a = g.r[i], b = g.r[i];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *p = g.red + 2 * (int64_t)blockIdx.x;
        p[0] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        p[1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

__global__ __launch_bounds__(256) void k_tr_norm_final(const TrField *__restrict__ tf)
{
    __shared__ double sm[8];
    const TrField g = tf[blockIdx.x];
    if (!g.out) return;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < g.nblk; i += blockDim.x) {
        re += g.red[2 * i];
        im += g.red[2 * i + 1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = re;
        sm[4 + (threadIdx.x >> 6)] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        g.out[0] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
        g.out[1] = (sm[4] + sm[5]) + (sm[6] + sm[7]);
    }
}

hipError_t launch_tr_multi(const TrField *tf, int nf, bool update, bool norm, bool general,
                           int nblk_max, int64_t n_max, int ny_max, int nx_max, hipStream_t s)
{
    if (nf <= 0) return hipSuccess;
    if (nf > 65535 || ny_max < 1 || nx_max < 1) return hipErrorInvalidValue;
    if (update)
        hipLaunchKernelGGL(k_tr_update, dim3(grid_for(n_max), nf), dim3(256), 0, s, tf);
    const dim3 gh((nx_max + 63) / 64, (ny_max + 3) / 4, nf), bh(64, 4, 1);
    if (general)
        hipLaunchKernelGGL((k_tr_H<3, 3>), gh, bh, 0, s, tf);
    else
        hipLaunchKernelGGL((k_tr_H<3, 2>), gh, bh, 0, s, tf);
    if (norm) {
        hipLaunchKernelGGL(k_tr_norm_partial, dim3(nblk_max, nf), dim3(256), 0, s, tf);
        hipLaunchKernelGGL(k_tr_norm_final, dim3(nf), dim3(256), 0, s, tf);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gradient: g_cell = w2 Re sum_{b,g in cell} M[Delta(b,g)] conj(lam_b) U_g
struct MassTable {
    double M[4];
};

template <int D>
__global__ void k_grad_cells(const double2 *__restrict__ lam, const double2 *__restrict__ U,
                             MassTable mt, double w2, double *__restrict__ gcell, int nz,
                             int ny, int nx)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;   // storage 0..nx
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x > nx || y > ny) return;
    double2 lv[1 << D], uv[1 << D];
    bool ok[1 << D];
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int cx = x - 1 + ex, cy = y - 1 + ey, cz = D == 3 ? z - 1 + ez : 0;
        ok[e] = (unsigned)cx < (unsigned)nx && (unsigned)cy < (unsigned)ny &&
                (unsigned)cz < (unsigned)nz;
        const int64_t i = ((int64_t)cz * ny + cy) * nx + cx;
        lv[e] = ok[e] ? lam[i] : make_double2(0.0, 0.0);
        uv[e] = ok[e] ? U[i] : make_double2(0.0, 0.0);
    }
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < (1 << D); ++b)
#pragma unroll
        for (int g = 0; g < (1 << D); ++g) {
            const int cls = __popc(b ^ g);
            // Re(conj(l) u) = l.x u.x + l.y u.y
            s += mt.M[cls] * (lv[b].x * uv[g].x + lv[b].y * uv[g].y);
        }
    gcell[((int64_t)z * (ny + 1) + y) * (nx + 1) + x] = w2 * s;
}

hipError_t launch_grad_cells(int ndim, const int *n, double w2, const double *mass,
                             const void *lam, const void *U, double *gcell, hipStream_t s)
{
    const int nz = ndim == 3 ? n[0] : 1;
    const int ny = ndim == 3 ? n[1] : n[0];
    const int nx = ndim == 3 ? n[2] : n[1];
    MassTable mt{{mass[0], mass[1], mass[2], ndim == 3 ? mass[3] : 0.0}};
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 1 + 63) / 64, (ny + 1 + 3) / 4, ndim == 3 ? nz + 1 : 1);
    if (ndim == 2)
        hipLaunchKernelGGL(k_grad_cells<2>, grd, blk, 0, s, (const double2 *)lam,
                           (const double2 *)U, mt, w2, gcell, nz, ny, nx);
    else
        hipLaunchKernelGGL(k_grad_cells<3>, grd, blk, 0, s, (const double2 *)lam,
                           (const double2 *)U, mt, w2, gcell, nz, ny, nx);
    return hipGetLastError();
}

// adjoint of m_cell = 2^-D sum_e m_node(clamp(alpha + e)): per axis, the cell
// lower corners a (storage a+1) whose corner a+e clamps to node i, with the
// number of such e in {0,1}.
__device__ __forceinline__ int axis_cells(int i, int n, int *st, int *mult)
{
    int cnt = 0;
    for (int a = i - 2; a <= i + 1; ++a) {
        if (a < -1 || a > n - 1) continue;
        int mlt = 0;
        for (int e = 0; e < 2; ++e) {
            int c = a + e;
            c = c < 0 ? 0 : (c >= n ? n - 1 : c);
            mlt += c == i;
        }
        if (mlt) {
            st[cnt] = a + 1;
            mult[cnt] = mlt;
            ++cnt;
        }
    }
    return cnt;
}

template <int D>
__global__ void k_grad_nodes(const double *__restrict__ gcell, double *__restrict__ grad, int nz,
                             int ny, int nx)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    int sx[4], mx[4], sy[4], my[4], sz[4], mz[4];
    const int cxn = axis_cells(x, nx, sx, mx);
    const int cyn = axis_cells(y, ny, sy, my);
    int czn = 1;
    sz[0] = 0;
    mz[0] = 1;
    if (D == 3) czn = axis_cells(z, nz, sz, mz);
    double s = 0.0;
    for (int c = 0; c < czn; ++c)
        for (int b = 0; b < cyn; ++b)
            for (int a = 0; a < cxn; ++a)
                s += (double)(mz[c] * my[b] * mx[a]) *
                     gcell[((int64_t)sz[c] * (ny + 1) + sy[b]) * (nx + 1) + sx[a]];
    grad[((int64_t)z * ny + y) * nx + x] = s * (1.0 / (1 << D));
}

hipError_t launch_grad_nodes(int ndim, const int *n, const double *gcell, double *grad,
                             hipStream_t s)
{
    const int nz = ndim == 3 ? n[0] : 1;
    const int ny = ndim == 3 ? n[1] : n[0];
    const int nx = ndim == 3 ? n[2] : n[1];
    dim3 blk(64, 4, 1);
    dim3 grd((nx + 63) / 64, (ny + 3) / 4, nz);
    if (ndim == 2)
        hipLaunchKernelGGL(k_grad_nodes<2>, grd, blk, 0, s, gcell, grad, nz, ny, nx);
    else
        hipLaunchKernelGGL(k_grad_nodes<3>, grd, blk, 0, s, gcell, grad, nz, ny, nx);
    return hipGetLastError();
}

}  // namespace tdp
