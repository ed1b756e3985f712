// 19-point two-pass substep (Sec. 4.2, Algorithm 3, Appendix A).
//
// Pass 1 computes the divergence field d = D1x ux + D1y uy + D1z uz, the
// right-hand side without the (nu/3) grad(div u) term, and the partial RK3
// register and output.  Pass 2 adds dt (nu/3) D1_i d to w_i and
// beta dt (nu/3) D1_i d to the output velocity.  Both passes read only
// axis-aligned taps (19 points).
//
// This file holds the direct kernels of both passes (one thread per point,
// taps through the caches from the ghost zones), the z-sweep form of pass 2,
// and the dispatch of both passes; the z-sweep form of pass 1 shares the
// 55-point sweep.
#include "sweep_common.hpp"

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

template <typename T, typename TW, int S, bool FRC>
__global__ __launch_bounds__(256) void pass19a_kernel(Geom g, Fields4<T> in, Fields4<T> out,
                                                      Fields4<TW> w, T* __restrict__ dv,
                                                      Coef<T> cf, RKCoef<TW> rk,
                                                      ForceArgs<T> fa) {
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
    if constexpr (FRC) {  // f = a cos(k.x + phase), eq. (forcing)
        const ForceDev<T>* fd = fa.dev;
        const T ph = T(cos(fd->kx * (i * fd->dx) + fd->ky * (j * fd->dy) + fd->kz * (k * fd->dz) +
                           fd->phase));
#pragma unroll
        for (int q = 0; q < 3; ++q) r[1 + q] += fd->a[q] * ph;
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

// z-sweep form of pass 2: a TX x TY column tile sweeps a z chunk of d.
// Each step puts one plane of d (tile + 3-cell halo, periodic images
// resolved by the loader) into LDS, forms its x and y first derivatives for
// the thread's column (kept 3 planes), and pushes the centre value into a
// register queue of 7 planes for the z derivative; output plane p - 3 is
// completed from them.  Substep 3 neither reads nor writes w.
template <typename T, int NH>
struct Pass2Regs {
    T q[8];      // column of d over planes (ring)
    T dx[4], dy[4];  // x / y first derivatives of d, ring of 4 planes
    T pf;        // prefetched interior value of the next plane
    T ph[NH];    // prefetched halo values of the next plane
    double red[4];  // RED: FP64 diagnostics of the thread's column
    int bad;        // RED: points of the column with a non-finite value
};

// As in the 55-point sweep, no memory operation of a step sits behind a
// branch: a step with nothing to load or store uses descriptors of zero range.
template <typename T, int TX, int TY, int NH>
__device__ __forceinline__ void pass2_prefetch(Pass2Regs<T, NH>& R,
                                               const SweepCtx<T, TX, TY>& X, const T* dv,
                                               long long corner, unsigned bytes) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(dv + corner, bytes);
    R.pf = bload((T*)nullptr, rs, X.goff_int);
#pragma unroll
    for (int h = 0; h < NH; ++h) R.ph[h] = bload((T*)nullptr, rs, X.goff_h[h]);
}

template <int PH, int S, bool NT, bool RED, typename T, typename TW, int TX, int TY, int NH>
__device__ __forceinline__ void pass2_step(int t0, int nplanes, int zb, Pass2Regs<T, NH>& R,
                                           const SweepCtx<T, TX, TY>& X, T* lds, const Geom& g,
                                           const T* dv, const Fields4<T>& out,
                                           const Fields4<TW>& w, const Coef<T>& cf,
                                           const RKCoef<TW>& rk, TW cgd) {
    using Sh = SweepShape<T, TX, TY>;
    constexpr int W = Sh::W;
    const int t = t0 + PH;
    if (t >= nplanes) return;
    const int p = zb - kR + t;  // plane loaded in this step
    const int o = p - kR;       // output plane finished in this step
    const bool outstep = t >= 2 * kR;
    const long long ocorner = g.origin + (long long)o * g.plane - kR * g.px - kR;
    const unsigned ob = outstep ? X.plane_bytes : 0u;
    const unsigned wb = outstep ? X.wplane_bytes : 0u;
    constexpr int CP = NT ? kNonTemporal : 0;
    T ov[3] = {T(0), T(0), T(0)};
    TW wv[3] = {TW(0), TW(0), TW(0)};
    // RED (substep 3): lnrho of the output point, final since pass 1
    T lr = T(0);
    if constexpr (RED) lr = bload((T*)nullptr, plane_rsrc(out.f[0] + ocorner, ob), X.lane_o);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ov[i] = bload<CP>((T*)nullptr, plane_rsrc(out.f[1 + i] + ocorner, ob), X.lane_o);
        if constexpr (S != 3)
            wv[i] = bload<CP>((TW*)nullptr,
                              plane_rsrc(w.f[1 + i] + (long long)o * g.wplane, wb), X.lane_w);
    }
    T* buf = lds + (PH & 1) * Sh::FS;
    const int ci = (threadIdx.x / TX + kR) * W + (threadIdx.x % TX + kR);
    buf[ci] = R.pf;
#pragma unroll
    for (int h = 0; h < NH; ++h) buf[X.loff_h[h]] = R.ph[h];
    pass2_prefetch<T, TX, TY, NH>(R, X, dv, plane_corner(g, p + 1),
                                  t + 1 < nplanes ? X.plane_bytes : 0u);
    __syncthreads();

    const T* B = buf + ci;
    R.q[sl8(PH)] = B[0];
    R.dx[PH & 3] = cf.d1[0][0] * (B[1] - B[-1]) + cf.d1[0][1] * (B[2] - B[-2]) +
                   cf.d1[0][2] * (B[3] - B[-3]);
    R.dy[PH & 3] = cf.d1[1][0] * (B[W] - B[-W]) + cf.d1[1][1] * (B[2 * W] - B[-2 * W]) +
                   cf.d1[1][2] * (B[3 * W] - B[-3 * W]);
    {
        const T dz = cf.d1[2][0] * (R.q[sl8(PH - 2)] - R.q[sl8(PH - 4)]) +
                     cf.d1[2][1] * (R.q[sl8(PH - 1)] - R.q[sl8(PH - 5)]) +
                     cf.d1[2][2] * (R.q[sl8(PH)] - R.q[sl8(PH - 6)]);
        constexpr int DO = (PH + 1) & 3;  // slot of plane p - 3
        const T gd[3] = {R.dx[DO], R.dy[DO], dz};
        T un[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const TW tq = cgd * TW(gd[i]);
            if constexpr (S != 3)
                bstore<CP>(wv[i] + tq, plane_rsrc(w.f[1 + i] + (long long)o * g.wplane, wb),
                           X.lane_w);
            un[i] = T(TW(ov[i]) + rk.beta * tq);
            bstore<CP>(un[i], plane_rsrc(out.f[1 + i] + ocorner, ob), X.lane_o);
        }
        if constexpr (RED) {
            if (outstep && X.lane_o != kDropOffset) red_point(R.red, R.bad, lr, un[0], un[1], un[2]);
        }
    }
}

// RED (substep 3 only): also the FP64 diagnostics of the new state, one
// partial per workgroup at part[blockIdx.x * kReduceSlots ...].
template <typename T, typename TW, int TX, int TY, int S, bool NT, bool RED = false>
__global__ __launch_bounds__(TX* TY) void substep19_pass2(Geom g, const T* __restrict__ dv,
                                                          Fields4<T> out, Fields4<TW> w,
                                                          Coef<T> cf, RKCoef<TW> rk, TW cgd,
                                                          SweepGrid m, double* part) {
    static_assert(!RED || S == 3, "diagnostics of the final substep only");
    using Sh = SweepShape<T, TX, TY>;
    constexpr int NH = Sh::NH;
    __shared__ T lds[2 * Sh::FS];
    const TileXY tl = sweep_tile_of(g, TX, TY, m);
    if (tl.zb >= tl.ze) {  // not produced by sweep_grid; keeps every partial defined
        if constexpr (RED) {
            if (threadIdx.x == 0)
                for (int i = 0; i < 5; ++i) part[(size_t)blockIdx.x * kReduceSlots + i] = 0.0;
        }
        return;
    }
    SweepCtx<T, TX, TY> X;
    sweep_ctx_init<T, TW, TX, TY, false>(X, g, tl.tx, tl.ty);
    Pass2Regs<T, NH> R;
#pragma unroll
    for (int s = 0; s < 8; ++s) R.q[s] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) R.dx[s] = R.dy[s] = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) R.red[i] = 0.0;
    R.bad = 0;
    const int zb = tl.zb;
    const int nplanes = (tl.ze - zb) + 2 * kR;
    pass2_prefetch<T, TX, TY, NH>(R, X, dv, plane_corner(g, zb - kR), X.plane_bytes);
    for (int t0 = 0; t0 < nplanes; t0 += 8) {
        pass2_step<0, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<1, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<2, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<3, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<4, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<5, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<6, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
        pass2_step<7, S, NT, RED>(t0, nplanes, zb, R, X, lds, g, dv, out, w, cf, rk, cgd);
    }
    if constexpr (RED) red_store_n<Sh::NW>(R.red, R.bad, part);
}

}  // namespace

template <typename T, typename TW>
hipError_t launch_pass19a(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, T* div,
                          const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                          const ForceArgs<T>* frc, hipStream_t st) {
    if (tile != 0)
        return launch_pass19a_sweep<T, TW>(g, in, out, w, div, c, rk, s, tile, zchunk, frc, st);
    const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)g.nz);
    const ForceArgs<T> fa = frc ? *frc : ForceArgs<T>{nullptr, nullptr};
    auto go = [&](auto force) {
        constexpr bool FRC = decltype(force)::value;
        if (s == 1)
            hipLaunchKernelGGL((pass19a_kernel<T, TW, 1, FRC>), grid, dim3(256), 0, st, g, in, out,
                               w, div, c, rk, fa);
        else
            hipLaunchKernelGGL((pass19a_kernel<T, TW, 2, FRC>), grid, dim3(256), 0, st, g, in, out,
                               w, div, c, rk, fa);
    };
    if (frc)
        go(std::true_type{});
    else
        go(std::false_type{});
    return hipGetLastError();
}

// Pass 2 takes the column tile of the chosen shape (its register budget and
// loader options do not apply to this one-field sweep).
template <typename T, typename TW>
hipError_t launch_pass19b(const Geom& g, const T* div, Fields4<T> out, Fields4<TW> w,
                          const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                          double* partials, int part_cap, int* nparts, hipStream_t st) {
    if (nparts) *nparts = 0;
    const TW cgd = TW((double)rk.dt * c.nu3);
    return with_tile(tile, hipErrorInvalidValue, [&](auto I) -> hipError_t {
        constexpr TileCfg k = kTiles[decltype(I)::value];
        if constexpr (k.tx == 0) {
            const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4),
                            (unsigned)g.nz);
            hipLaunchKernelGGL((pass19b_kernel<T, TW>), grid, dim3(256), 0, st, g, div, out, w, c,
                               rk, cgd);
        } else {
            const int res =
                resident_blocks<substep19_pass2<T, TW, k.tx, k.ty, 2, k.nt>>(k.tx * k.ty);
            const SweepGrid sg = sweep_grid(g, k.tx, k.ty, zchunk, res);
            const dim3 grid(sg.blocks), block(k.tx * k.ty);
            // Fuse the diagnostics unless that leaves fewer than 2 waves per
            // SIMD: this light one-field sweep loses little occupancy that
            // matters, while the standalone pass re-reads the whole state
            // (measured at 512^3: 4.7% of the FP32 19-point step).
            static const bool fuse_ok = [] {
                int a = 0, b = 0;
                const int blk = k.tx * k.ty;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &a, substep19_pass2<T, TW, k.tx, k.ty, 3, k.nt, true>, blk, 0) !=
                        hipSuccess ||
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &b, substep19_pass2<T, TW, k.tx, k.ty, 3, k.nt>, blk, 0) != hipSuccess)
                    return false;
                return a > 0 && (a >= b || a * (blk / 64) >= 8);
            }();
            switch (s) {
            case 1:
                hipLaunchKernelGGL((substep19_pass2<T, TW, k.tx, k.ty, 1, k.nt>), grid, block, 0,
                                   st, g, div, out, w, c, rk, cgd, sg, nullptr);
                break;
            case 2:
                hipLaunchKernelGGL((substep19_pass2<T, TW, k.tx, k.ty, 2, k.nt>), grid, block, 0,
                                   st, g, div, out, w, c, rk, cgd, sg, nullptr);
                break;
            default:
                if (partials && nparts && fuse_ok && sg.blocks <= part_cap) {
                    hipLaunchKernelGGL((substep19_pass2<T, TW, k.tx, k.ty, 3, k.nt, true>), grid,
                                       block, 0, st, g, div, out, w, c, rk, cgd, sg, partials);
                    *nparts = sg.blocks;
                } else {
                    hipLaunchKernelGGL((substep19_pass2<T, TW, k.tx, k.ty, 3, k.nt>), grid, block,
                                       0, st, g, div, out, w, c, rk, cgd, sg, nullptr);
                }
                break;
            }
        }
        return hipGetLastError();
    });
}

#define FD6_INST19(T, TW)                                                                       \
    template hipError_t launch_pass19a<T, TW>(const Geom&, Fields4<T>, Fields4<T>, Fields4<TW>, \
                                              T*, const Coef<T>&, const RKCoef<TW>&, int, int, \
                                              int, const ForceArgs<T>*, hipStream_t);          \
    template hipError_t launch_pass19b<T, TW>(const Geom&, const T*, Fields4<T>, Fields4<TW>,   \
                                              const Coef<T>&, const RKCoef<TW>&, int, int,     \
                                              int, double*, int, int*, hipStream_t);
FD6_INST19(double, double)
FD6_INST19(float, float)
FD6_INST19(float, double)

}  // namespace fd6
