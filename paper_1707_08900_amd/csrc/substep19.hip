// 19-point two-pass substep (Sec. 4.2, Algorithm 3, Appendix A).
//
// Pass 1 computes the divergence field d = D1x ux + D1y uy + D1z uz (stored
// with a ghost zone), the right-hand side without the (nu/3) grad(div u)
// term, and the partial RK3 register and output.  After the periodic ghost
// fill of d, pass 2 adds dt (nu/3) D1_i d to w_i and beta dt (nu/3) D1_i d to
// the output velocity.  Both passes read only axis-aligned taps (19 points).
//
// gfx950 mapping: one thread per output point, 64-wide x rows per wavefront
// (coalesced), 4 rows per workgroup; taps come through the L1/L2 caches.
#include "fd6_internal.hpp"

namespace fd6 {
namespace {

template <typename T>
__device__ __forceinline__ T d1_taps(const T* f, long long c, long long s, const T* w) {
    return w[0] * (f[c + s] - f[c - s]) + w[1] * (f[c + 2 * s] - f[c - 2 * s]) +
           w[2] * (f[c + 3 * s] - f[c - 3 * s]);
}

template <typename T>
__device__ __forceinline__ T d2_taps(const T* f, long long c, long long s, const T* w) {
    return w[0] * f[c] + w[1] * (f[c + s] + f[c - s]) + w[2] * (f[c + 2 * s] + f[c - 2 * s]) +
           w[3] * (f[c + 3 * s] + f[c - 3 * s]);
}

template <typename T, typename TW, int S>
__global__ __launch_bounds__(256) void pass19a_kernel(Geom g, Fields4<T> in, Fields4<T> out,
                                                      Fields4<TW> w, T* __restrict__ dv,
                                                      Coef<T> cf, RKCoef<TW> rk) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = g.origin + (long long)k * g.plane + (long long)j * g.px + i;
    const long long s[3] = {1, g.px, g.plane};
    T gr[3], J[3][3], u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gr[a] = d1_taps(in.f[0], c, s[a], cf.d1[a]);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        u[q] = in.f[1 + q][c];
#pragma unroll
        for (int a = 0; a < 3; ++a) J[q][a] = d1_taps(in.f[1 + q], c, s[a], cf.d1[a]);
    }
    const T div = J[0][0] + J[1][1] + J[2][2];
    dv[c] = div;
    // nu lap u_i with plain (not 4/3-weighted) second-derivative weights
    T L[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc += d2_taps(in.f[1 + q], c, s[a], cf.lp[a]);
        L[q] = acc;
    }
    T r[4];
    r[0] = -(u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2]) - div;
    const T third = T(1) / T(3);
    const T dv3 = div * third;
    const T sxy = T(0.5) * (J[0][1] + J[1][0]);
    const T sxz = T(0.5) * (J[0][2] + J[2][0]);
    const T syz = T(0.5) * (J[1][2] + J[2][1]);
    const T sxx = J[0][0] - dv3, syy = J[1][1] - dv3, szz = J[2][2] - dv3;
    const T sg[3] = {sxx * gr[0] + sxy * gr[1] + sxz * gr[2],
                     sxy * gr[0] + syy * gr[1] + syz * gr[2],
                     sxz * gr[0] + syz * gr[1] + szz * gr[2]};
    const T two_nu = cf.nu + cf.nu;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const T adv = u[0] * J[q][0] + u[1] * J[q][1] + u[2] * J[q][2];
        r[1 + q] = (L[q] + two_nu * sg[q]) - cf.cs2 * gr[q] - adv;
    }
    const long long cw = (long long)k * g.wplane + (long long)j * g.wpx + i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        TW wn;
        if constexpr (S == 1)
            wn = rk.dt * TW(r[q]);
        else
            wn = rk.alpha * w.f[q][cw] + rk.dt * TW(r[q]);
        // pass 2 completes w_u, so every substep stores it here
        w.f[q][cw] = wn;
        out.f[q][c] = T(TW(in.f[q][c]) + rk.beta * wn);
    }
}

template <typename T, typename TW>
__global__ __launch_bounds__(256) void pass19b_kernel(Geom g, const T* __restrict__ dv,
                                                      Fields4<T> out, Fields4<TW> w, Coef<T> cf,
                                                      RKCoef<TW> rk, TW cgd) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = g.origin + (long long)k * g.plane + (long long)j * g.px + i;
    const long long s[3] = {1, g.px, g.plane};
    const long long cw = (long long)k * g.wplane + (long long)j * g.wpx + i;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const TW t = cgd * TW(d1_taps(dv, c, s[q], cf.d1[q]));
        w.f[1 + q][cw] = w.f[1 + q][cw] + t;
        out.f[1 + q][c] = T(TW(out.f[1 + q][c]) + rk.beta * t);
    }
}

}  // namespace

template <typename T, typename TW>
hipError_t launch_pass19a(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, T* div,
                          const Coef<T>& c, const RKCoef<TW>& rk, int s, hipStream_t st) {
    const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)g.nz);
    switch (s) {
    case 1:
        hipLaunchKernelGGL((pass19a_kernel<T, TW, 1>), grid, dim3(256), 0, st, g, in, out, w, div,
                           c, rk);
        break;
    default:
        hipLaunchKernelGGL((pass19a_kernel<T, TW, 2>), grid, dim3(256), 0, st, g, in, out, w, div,
                           c, rk);
        break;
    }
    return hipGetLastError();
}

template <typename T, typename TW>
hipError_t launch_pass19b(const Geom& g, const T* div, Fields4<T> out, Fields4<TW> w,
                          const Coef<T>& c, const RKCoef<TW>& rk, hipStream_t st) {
    const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)g.nz);
    hipLaunchKernelGGL((pass19b_kernel<T, TW>), grid, dim3(256), 0, st, g, div, out, w, c, rk,
                       TW((double)rk.dt * c.nu3));
    return hipGetLastError();
}

#define FD6_INST19(T, TW)                                                                       \
    template hipError_t launch_pass19a<T, TW>(const Geom&, Fields4<T>, Fields4<T>, Fields4<TW>, \
                                              T*, const Coef<T>&, const RKCoef<TW>&, int,      \
                                              hipStream_t);                                    \
    template hipError_t launch_pass19b<T, TW>(const Geom&, const T*, Fields4<T>, Fields4<TW>,   \
                                              const Coef<T>&, const RKCoef<TW>&, hipStream_t);
FD6_INST19(double, double)
FD6_INST19(float, float)
FD6_INST19(float, double)

}  // namespace fd6
