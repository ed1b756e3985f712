// 55-point fused substep (Sec. 4.1, Algorithm 2): the right-hand side of the
// continuity and momentum equations (Sec. 2.1) from sixth-order first, second
// and bidiagonal mixed differences (Sec. 2.3), followed by the 2N-RK3 update
// (Sec. 2.4) of the RK3 register w and of the output state, in one pass.
//
// Kernel design for gfx950 (the paper's K40 shared-memory cube and rolling
// cache are not reused):
//
//  * One workgroup owns a TX x TY column tile of the xy-plane and sweeps a
//    chunk of z.  Each step loads one new xy-plane (tile + 3-cell halo) of the
//    four fields from HBM into LDS (coalesced x-rows, double buffered, one
//    barrier per plane), prefetching the next plane into registers.
//  * From that plane every thread forms, for its own column, the x and y
//    first derivatives of all fields and the xy part of the linear viscous
//    term (second derivatives along x and y, xy mixed derivative).
//  * z derivatives come from a register queue holding the thread's column
//    over 7 planes.
//  * The xz and yz mixed derivatives are built by scatter: the bidiagonal
//    stencil at output plane z is sum_k c_k [A_k(z+k) - A_k(z-k)], where
//    A_k(p) = f(x+k, p) - f(x-k, p) is the same x (or y) difference the plane
//    step already forms, so each plane adds +-c_k A_k into pending
//    accumulators of the output planes p -+ k (a register ring of 8 planes).
//  * Output plane z is finished 3 planes behind the load front: the right-hand
//    side is assembled in registers and the RK3 update is written out.
//  * The z loop is unrolled by 8 so every ring index is a compile-time
//    register; the workgroup-to-tile map keeps neighbouring tiles on one XCD
//    so y-halo rows are served from that XCD's L2.
#pragma once

#include <cstdlib>

#include "fd6_internal.hpp"

namespace fd6 {
namespace {

// ---------------------------------------------------------------------------
// Shared per-point pieces
// ---------------------------------------------------------------------------

// Right-hand side from the derivatives at one point (eqs. continuity,
// navierstokes with f = 0, tensor):
//   u: centre velocity, g = grad lnrho, J[i][a] = d_a u_i,
//   L[i] = nu (lap u_i + (1/3) d_i div u) (already scaled by nu).
template <typename T>
__device__ __forceinline__ void assemble_rhs(const T u[3], const T g[3], const T J[3][3],
                                             const T L[3], T nu, T cs2, T r[4]) {
    const T div = J[0][0] + J[1][1] + J[2][2];
    r[0] = -(u[0] * g[0] + u[1] * g[1] + u[2] * g[2]) - div;
    // 2 S = J + J^T - (2/3) div I, and 2 nu S . grad lnrho = nu (2S) g
    const T d23 = div * T(2.0 / 3.0);
    const T s01 = J[0][1] + J[1][0], s02 = J[0][2] + J[2][0], s12 = J[1][2] + J[2][1];
    const T s00 = T(2) * J[0][0] - d23, s11 = T(2) * J[1][1] - d23, s22 = T(2) * J[2][2] - d23;
    const T sg[3] = {s00 * g[0] + s01 * g[1] + s02 * g[2], s01 * g[0] + s11 * g[1] + s12 * g[2],
                     s02 * g[0] + s12 * g[1] + s22 * g[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T adv = u[0] * J[i][0] + u[1] * J[i][1] + u[2] * J[i][2];
        r[1 + i] = (L[i] + nu * sg[i]) - cs2 * g[i] - adv;
    }
}

// 2N-RK3 update of one value (eq. 2N-RK_scheme, Algorithm 2):
//   w <- alpha w + dt r  (alpha(1) = 0: substep 1 does not read w)
//   out <- in + beta w   (substep 3 need not store w: the next step's
//                         substep 1 ignores it)
template <int S, typename T, typename TW>
__device__ __forceinline__ T rk_update(T in, T r, TW& w, const RKCoef<TW>& rk) {
    TW wn;
    if constexpr (S == 1)
        wn = rk.dt * TW(r);
    else
        wn = rk.alpha * w + rk.dt * TW(r);
    w = wn;
    return T(TW(in) + rk.beta * wn);
}

// ---------------------------------------------------------------------------
// Direct kernel: one thread per point, every tap read from global memory.
// Kept as the simplest statement of the per-point arithmetic.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T d1_at(const T* f, long long c, long long s, const T* w) {
    return w[0] * (f[c + s] - f[c - s]) + w[1] * (f[c + 2 * s] - f[c - 2 * s]) +
           w[2] * (f[c + 3 * s] - f[c - 3 * s]);
}

template <typename T>
__device__ __forceinline__ T d2w_at(const T* f, long long c, long long s, const T* w) {
    return w[0] * f[c] + w[1] * (f[c + s] + f[c - s]) + w[2] * (f[c + 2 * s] + f[c - 2 * s]) +
           w[3] * (f[c + 3 * s] + f[c - 3 * s]);
}

template <typename T>
__device__ __forceinline__ T mix_at(const T* f, long long c, long long sa, long long sb,
                                    const T* w) {
    T acc = T(0);
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const T t = (f[c + k * sa + k * sb] - f[c - k * sa + k * sb]) +
                    (f[c - k * sa - k * sb] - f[c + k * sa - k * sb]);
        acc += w[k - 1] * t;
    }
    return acc;
}

template <typename T, typename TW, int S>
__global__ __launch_bounds__(256) void substep55_direct(Geom g, Fields4<T> in, Fields4<T> out,
                                                        Fields4<TW> w, Coef<T> cf,
                                                        RKCoef<TW> rk) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long c = g.origin + (long long)k * g.plane + (long long)j * g.px + i;
    const long long s[3] = {1, g.px, g.plane};
    T gr[3], J[3][3], L[3], u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gr[a] = d1_at(in.f[0], c, s[a], cf.d1[a]);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        u[q] = in.f[1 + q][c];
#pragma unroll
        for (int a = 0; a < 3; ++a) J[q][a] = d1_at(in.f[1 + q], c, s[a], cf.d1[a]);
    }
    // L_i = sum_a lw[i][a] . D2_a u_i + (1/3) sum_{j != i} D_ij u_j (nu folded)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc += d2w_at(in.f[1 + q], c, s[a], cf.lw[q][a]);
        L[q] = acc;
    }
    L[0] += mix_at(in.f[2], c, s[0], s[1], cf.mw[0]) + mix_at(in.f[3], c, s[0], s[2], cf.mw[1]);
    L[1] += mix_at(in.f[1], c, s[0], s[1], cf.mw[0]) + mix_at(in.f[3], c, s[1], s[2], cf.mw[2]);
    L[2] += mix_at(in.f[1], c, s[0], s[2], cf.mw[1]) + mix_at(in.f[2], c, s[1], s[2], cf.mw[2]);
    T r[4];
    assemble_rhs(u, gr, J, L, cf.nu, cf.cs2, r);
    const long long cw = (long long)k * g.wplane + (long long)j * g.wpx + i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        TW wv = (S == 1) ? TW(0) : w.f[q][cw];
        out.f[q][c] = rk_update<S>(in.f[q][c], r[q], wv, rk);
        if (S != 3) w.f[q][cw] = wv;
    }
}

// ---------------------------------------------------------------------------
// z-sweep kernel
// ---------------------------------------------------------------------------

constexpr int sl8(int x) { return ((x % 8) + 8) % 8; }

// Raw buffer access: an SGPR descriptor for one plane of one field plus a
// 32-bit per-lane byte offset.  Loads beyond the descriptor's range return 0
// and stores beyond it are dropped, which replaces bounds branches.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufFlags = 0x00020000;        // raw, untyped access (word 3)
constexpr unsigned kDropOffset = 0x80000000u;  // beyond every plane's range

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, (int)bytes, kBufFlags);
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// LD = false: the next plane is loaded into registers and written to LDS by
// the threads; LD = true: it is copied by the buffer unit straight into LDS
// (64 consecutive dwords per wave instruction), with no staging registers.
template <typename T, int TX, int TY, bool LD = false>
struct SweepShape {
    static constexpr int NT = TX * TY;
    static constexpr int NW = NT / 64;              // wavefronts per workgroup
    static constexpr int W = TX + 2 * kR;           // LDS row length
    static constexpr int H = TY + 2 * kR;           // LDS rows
    static constexpr int PLANE = W * H;             // LDS elements per field plane
    static constexpr int HALO = 2 * kR * W + 2 * kR * TY;  // halo cells per plane
    static constexpr int NH = (HALO + NT - 1) / NT; // halo loads per thread (LD = false)
    static constexpr int DPE = (int)sizeof(T) / 4;  // dwords per element
    static constexpr int NCH = (PLANE * DPE + 63) / 64;  // 64-dword chunks per plane (LD)
    static constexpr int ND = (NCH + NW - 1) / NW;  // chunk copies per wave and field (LD)
    // field stride in LDS elements: LD pads to whole chunks; otherwise cell
    // PLANE is a dummy target for unused halo slots
    static constexpr int FS = LD ? NCH * 64 / DPE : PLANE + 1;
};

template <typename T, int NH>
struct SweepRegs {
    T q[4][8];    // raw column values of the 4 fields, ring over planes
    T L[3][8];    // pending linear viscous term of the 3 momentum components
    T dd[4][8];   // x/y first derivatives of the 4 fields, ring of 4 planes
    T pf[4];      // prefetched interior value of the next plane
    T ph[NH][4];  // prefetched halo values of the next plane
};

template <typename T, int TX, int TY, bool LD = false>
struct SweepCtx {
    using Sh = SweepShape<T, TX, TY, LD>;
    unsigned doff[Sh::ND];  // LD: byte offset (from the plane's ghost corner) of each lane's dword
    // Byte offsets, relative to the ghost corner (-3, -3) of a plane, of the
    // cells this thread loads (beyond the plane: the load returns 0; those
    // cells are only read by threads whose outputs are dropped).
    unsigned goff_int;
    unsigned goff_h[Sh::NH];
    int loff_h[Sh::NH];   // LDS slot of each halo load (dummy cell if unused)
    unsigned lane_o;      // byte offset of the output point in a state plane
    unsigned lane_w;      // byte offset of the output point in a w plane
    unsigned plane_bytes, wplane_bytes;
};


// Element index of the ghost corner (-3, -3) of interior plane p mod nz.
__device__ __forceinline__ long long plane_corner(const Geom& g, int p) {
    const int pz = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
    return g.origin + (long long)pz * g.plane - kR * g.px - kR;
}

template <typename T, int TX, int TY, int NH>
__device__ __forceinline__ void sweep_prefetch(SweepRegs<T, NH>& R, const SweepCtx<T, TX, TY>& X,
                                               const Fields4<T>& in, long long corner) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in.f[f] + corner, X.plane_bytes);
        R.pf[f] = bload((T*)nullptr, rs, X.goff_int);
#pragma unroll
        for (int h = 0; h < NH; ++h) R.ph[h][f] = bload((T*)nullptr, rs, X.goff_h[h]);
    }
}

// LDS pointer in the local address space (required by the LDS copy).
template <typename T>
using lds_t = __attribute__((address_space(3))) T*;

// LD: copy plane `corner` of the four fields into one LDS buffer.  Chunk j
// (64 dwords) is issued by wave j % NW; its lanes fetch the dwords whose byte
// offsets were precomputed in doff (periodic images included).
template <typename T, int TX, int TY>
__device__ __forceinline__ void sweep_dma(const SweepCtx<T, TX, TY, true>& X,
                                          const Fields4<T>& in, long long corner, lds_t<T> buf) {
    using Sh = SweepShape<T, TX, TY, true>;
    const int wv = threadIdx.x / 64;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in.f[f] + corner, X.plane_bytes);
#pragma unroll
        for (int js = 0; js < Sh::ND; ++js) {
            const int j = wv + js * Sh::NW;
            if (j < Sh::NCH) {
                lds_t<T> dst = buf + f * Sh::FS + j * (64 / Sh::DPE);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (__attribute__((address_space(3))) void*)dst, 4, X.doff[js], 0, 0, 0);
            }
        }
    }
}

template <int PH, int S, bool LD, typename T, typename TW, int TX, int TY, int NH>
__device__ __forceinline__ void sweep_step(int t0, int nplanes, int zb, SweepRegs<T, NH>& R,
                                           const SweepCtx<T, TX, TY, LD>& X, T* lds,
                                           lds_t<T> lds3,
                                           const Geom& g, const Fields4<T>& in,
                                           const Fields4<T>& out, const Fields4<TW>& w,
                                           const Coef<T>& cf, const RKCoef<TW>& rk) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr int W = Sh::W;
    const int t = t0 + PH;
    if (t >= nplanes) return;
    const int p = zb - kR + t;  // plane loaded in this step
    const int o = p - kR;       // output plane finished in this step
    const bool outstep = t >= 2 * kR;

    T* buf = lds + (PH & 1) * 4 * Sh::FS;
    const int ci = (threadIdx.x / TX + kR) * W + (threadIdx.x % TX + kR);
    TW wv[4] = {TW(0), TW(0), TW(0), TW(0)};
    if constexpr (!LD) {
        // RK3 register of the output point, issued early
        if constexpr (S != 1) {
            if (outstep) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    wv[f] = bload((TW*)nullptr,
                                  plane_rsrc(w.f[f] + (long long)o * g.wplane, X.wplane_bytes),
                                  X.lane_w);
            }
        }
        // prefetched plane p -> LDS buffer (PH & 1)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            buf[f * Sh::FS + ci] = R.pf[f];
#pragma unroll
            for (int h = 0; h < NH; ++h) buf[f * Sh::FS + X.loff_h[h]] = R.ph[h][f];
        }
        // next plane -> registers
        if (t + 1 < nplanes)
            sweep_prefetch<T, TX, TY, NH>(R, X, in, plane_corner(g, p + 1));
        __syncthreads();
    } else {
        // this wave's copies of plane p are complete before the barrier; after
        // it the other buffer (read in the previous step by every wave) takes
        // plane p + 1
        __syncthreads();
        if (t + 1 < nplanes)
            sweep_dma<T, TX, TY>(X, in, plane_corner(g, p + 1), lds3 + ((PH + 1) & 1) * 4 * Sh::FS);
        if constexpr (S != 1) {
            if (outstep) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    wv[f] = bload((TW*)nullptr,
                                  plane_rsrc(w.f[f] + (long long)o * g.wplane, X.wplane_bytes),
                                  X.lane_w);
            }
        }
    }

    // ---- plane quantities of plane p for this thread's column ----
    // Stencils use their integer weights; grid spacing and viscosity enter
    // through per-axis scale factors (see Coef), which keeps the runtime
    // constants few enough to stay in scalar registers.
    // all taps as non-negative constant offsets from one window base
    const T* win = buf + (ci - kR * W - kR);
    constexpr int C0 = kR * W + kR;  // centre of the window
    const T* B0 = win + C0;
    const T* B1 = win + Sh::FS + C0;
    const T* B2 = win + 2 * Sh::FS + C0;
    const T* B3 = win + 3 * Sh::FS + C0;
    constexpr int DS = PH & 3;  // first-derivative slot of plane p
    constexpr T w2[3] = {T(270), T(-27), T(2)};

    // (A) what output p - 3 still needs from plane p: the centre values (top
    // of the z queues) and the k = 3 terms of its xz / yz stencils.  The
    // first contribution to output p + 3 (from the same differences) assigns.
    {
        R.q[0][sl8(PH)] = B0[0];
        R.q[1][sl8(PH)] = B1[0];
        R.q[2][sl8(PH)] = B2[0];
        R.q[3][sl8(PH)] = B3[0];
        const T zs3[3] = {cf.mu[1] * (B3[3] - B3[-3]),                 // (1/3) Dxz uz
                          cf.mu[2] * (B3[3 * W] - B3[-3 * W]),         // (1/3) Dyz uz
                          cf.mu[1] * (B1[3] - B1[-3]) +                // (1/3) Dxz ux
                              cf.mu[2] * (B2[3 * W] - B2[-3 * W])};    // + (1/3) Dyz uy
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            R.L[i][sl8(PH - 3)] += T(2) * zs3[i];
            R.L[i][sl8(PH + 3)] = T(-2) * zs3[i];
        }
    }

    // (B) finish output plane o = p - 3 before the rest of plane p is formed,
    // so the two working sets do not overlap in registers
    if (outstep) {
        T dz[4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
            dz[f] = cf.d1[2][0] * (R.q[f][sl8(PH - 2)] - R.q[f][sl8(PH - 4)]) +
                    cf.d1[2][1] * (R.q[f][sl8(PH - 1)] - R.q[f][sl8(PH - 5)]) +
                    cf.d1[2][2] * (R.q[f][sl8(PH)] - R.q[f][sl8(PH - 6)]);
        T Lf[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int f = 1 + i;
            const T rz = T(270) * (R.q[f][sl8(PH - 2)] + R.q[f][sl8(PH - 4)]) +
                         T(-27) * (R.q[f][sl8(PH - 1)] + R.q[f][sl8(PH - 5)]) +
                         T(2) * (R.q[f][sl8(PH)] + R.q[f][sl8(PH - 6)]) +
                         T(-490) * R.q[f][sl8(PH - 3)];
            Lf[i] = R.L[i][sl8(PH - 3)] + (i == 2 ? cf.sg4[2] : cf.sg[2]) * rz;
        }
        constexpr int DO = (PH + 1) & 3;  // slot of plane p - 3
        const T gr[3] = {R.dd[DO][0], R.dd[DO][1], dz[0]};
        const T J[3][3] = {{R.dd[DO][2], R.dd[DO][3], dz[1]},
                           {R.dd[DO][4], R.dd[DO][5], dz[2]},
                           {R.dd[DO][6], R.dd[DO][7], dz[3]}};
        const T u[3] = {R.q[1][sl8(PH - 3)], R.q[2][sl8(PH - 3)], R.q[3][sl8(PH - 3)]};
        T r[4];
        assemble_rhs(u, gr, J, Lf, cf.nu, cf.cs2, r);
        // ghost corner (-3, -3) of output plane o
        const long long ocorner = g.origin + (long long)o * g.plane - kR * g.px - kR;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const T v = rk_update<S>(R.q[f][sl8(PH - 3)], r[f], wv[f], rk);
            bstore(v, plane_rsrc(out.f[f] + ocorner, X.plane_bytes), X.lane_o);
            if constexpr (S != 3)
                bstore(wv[f], plane_rsrc(w.f[f] + (long long)o * g.wplane, X.wplane_bytes),
                       X.lane_w);
        }
    }

    // (C) the rest of plane p for this column: x / y first derivatives of the
    // four fields (kept 3 planes), the xy part of the linear viscous term, and
    // the k = 1, 2 terms of the xz / yz stencils of outputs p -+ k.
    // lnrho
    R.dd[DS][0] = cf.d1[0][0] * (B0[1] - B0[-1]) + cf.d1[0][1] * (B0[2] - B0[-2]) +
                  cf.d1[0][2] * (B0[3] - B0[-3]);
    R.dd[DS][1] = cf.d1[1][0] * (B0[W] - B0[-W]) + cf.d1[1][1] * (B0[2 * W] - B0[-2 * W]) +
                  cf.d1[1][2] * (B0[3 * W] - B0[-3 * W]);
    T lx, ly, lz;           // xy parts of nu (lap u_i + (1/3) d_i div u) at plane p
    T zx[2], zy[2], zz[2];  // scaled k = 1, 2 differences feeding the xz / yz terms
    // ux
    {
        const T c = B1[0];
        T a[3], b[3];
        T rx = T(0), ry = T(0), m = T(0);
#pragma unroll
        for (int k = 1; k <= 3; ++k) {
            const T xp = B1[k], xm = B1[-k], yp = B1[k * W], ym = B1[-k * W];
            a[k - 1] = xp - xm;
            b[k - 1] = yp - ym;
            rx += w2[k - 1] * (xp + xm);
            ry += w2[k - 1] * (yp + ym);
            const T t = (B1[k * W + k] - B1[k * W - k]) + (B1[-k * W - k] - B1[-k * W + k]);
            m += w2[k - 1] * t;
        }
        R.dd[DS][2] = cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2];
        R.dd[DS][3] = cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2];
        lx = cf.kxy[0] * c + cf.sg4[0] * rx + cf.sg[1] * ry;  // (4/3) D2x + D2y
        ly = cf.mu[0] * m;                                     // (1/3) Dxy ux
#pragma unroll
        for (int k = 0; k < 2; ++k) zz[k] = cf.mu[1] * a[k];   // (1/3) Dxz ux
    }
    // uy
    {
        const T c = B2[0];
        T a[3], b[3];
        T rx = T(0), ry = T(0), m = T(0);
#pragma unroll
        for (int k = 1; k <= 3; ++k) {
            const T xp = B2[k], xm = B2[-k], yp = B2[k * W], ym = B2[-k * W];
            a[k - 1] = xp - xm;
            b[k - 1] = yp - ym;
            rx += w2[k - 1] * (xp + xm);
            ry += w2[k - 1] * (yp + ym);
            const T t = (B2[k * W + k] - B2[k * W - k]) + (B2[-k * W - k] - B2[-k * W + k]);
            m += w2[k - 1] * t;
        }
        R.dd[DS][4] = cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2];
        R.dd[DS][5] = cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2];
        ly += cf.kxy[1] * c + cf.sg[0] * rx + cf.sg4[1] * ry;  // D2x + (4/3) D2y
        lx += cf.mu[0] * m;                                     // (1/3) Dxy uy
#pragma unroll
        for (int k = 0; k < 2; ++k) zz[k] += cf.mu[2] * b[k];   // (1/3) Dyz uy
    }
    // uz
    {
        const T c = B3[0];
        T a[3], b[3];
        T rx = T(0), ry = T(0);
#pragma unroll
        for (int k = 1; k <= 3; ++k) {
            const T xp = B3[k], xm = B3[-k], yp = B3[k * W], ym = B3[-k * W];
            a[k - 1] = xp - xm;
            b[k - 1] = yp - ym;
            rx += w2[k - 1] * (xp + xm);
            ry += w2[k - 1] * (yp + ym);
        }
        R.dd[DS][6] = cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2];
        R.dd[DS][7] = cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2];
        lz = cf.kxy[2] * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            zx[k] = cf.mu[1] * a[k];  // (1/3) Dxz uz
            zy[k] = cf.mu[2] * b[k];  // (1/3) Dyz uy
        }
    }

    // Scatter: the bidiagonal xz / yz stencil at output z is
    // sum_k c_k [A_k(z + k) - A_k(z - k)], so plane p adds +c_k A_k to the
    // pending output p - k and -c_k A_k to p + k (c = 270, -27, 2); the k = 3
    // terms were added in (A).
    {
        const T* zs[3] = {zx, zy, zz};
        const T lc[3] = {lx, ly, lz};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            R.L[i][sl8(PH + 2)] += T(27) * zs[i][1];
            R.L[i][sl8(PH + 1)] += T(-270) * zs[i][0];
            R.L[i][sl8(PH)] += lc[i];
            R.L[i][sl8(PH - 1)] += T(270) * zs[i][0];
            R.L[i][sl8(PH - 2)] += T(-27) * zs[i][1];
        }
    }
}

// One tile-chunk: columns [x0, x0 + TX) x [y0, y0 + TY) of the box, output
// planes [zb, ze).  Every thread of the workgroup calls it with the same
// arguments.
template <typename T, typename TW, int TX, int TY, int S, bool LD>
__device__ __forceinline__ void sweep_tile(const Geom& g, const Fields4<T>& in,
                                           const Fields4<T>& out, const Fields4<TW>& w,
                                           const Coef<T>& cf, const RKCoef<TW>& rk, int x0,
                                           int y0, int zb, int ze, T* lds, lds_t<T> lds3) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr int NH = Sh::NH;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    SweepCtx<T, TX, TY, LD> X;
    X.plane_bytes = (unsigned)(g.plane * (long long)sizeof(T));
    X.wplane_bytes = (unsigned)(g.wplane * (long long)sizeof(TW));
    // Periodic boundary condition (Sec. 4) resolved in the loader: a halo cell
    // outside the interior reads its periodic image, so this kernel neither
    // reads nor needs the ghost zone.  Offsets are taken from the ghost corner
    // (-3, -3) of a plane; cells beyond x < nx + 3, y < ny + 3 are never used
    // by a stored point and are dropped.
    auto wrapped_off = [&](int gx, int gy) -> unsigned {  // gx, gy in [-3, ...)
        if (gx >= g.nx + kR || gy >= g.ny + kR) return kDropOffset;
        const int ix = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
        const int iy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
        return (unsigned)(((iy + kR) * g.px + (ix + kR)) * (int)sizeof(T));
    };
    if constexpr (LD) {
        // dword d = 64 j + lane of the padded plane tile, j = wave + js NW
        const int lane = threadIdx.x & 63, wv = threadIdx.x / 64;
#pragma unroll
        for (int js = 0; js < Sh::ND; ++js) {
            const int d = 64 * (wv + js * Sh::NW) + lane;
            const int e = d / Sh::DPE, half = d % Sh::DPE;
            const int r = e / Sh::W, c = e - (e / Sh::W) * Sh::W;
            const unsigned o = e < Sh::PLANE ? wrapped_off(x0 - kR + c, y0 - kR + r) : kDropOffset;
            X.doff[js] = o == kDropOffset ? kDropOffset : o + 4u * (unsigned)half;
        }
    }
    X.goff_int = wrapped_off(x0 + tx, y0 + ty);
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int e = threadIdx.x + h * Sh::NT;
        int r = 0, c = 0;
        if (e < 2 * kR * Sh::W) {
            const int row = e / Sh::W;
            r = row < kR ? row : row + TY;
            c = e - row * Sh::W;
        } else {
            const int e2 = e - 2 * kR * Sh::W;
            r = kR + e2 / (2 * kR);
            const int cc = e2 % (2 * kR);
            c = cc < kR ? cc : cc + TX;
        }
        const bool in_range = e < Sh::HALO;
        X.goff_h[h] = in_range ? wrapped_off(x0 - kR + c, y0 - kR + r) : kDropOffset;
        X.loff_h[h] = in_range ? r * Sh::W + c : Sh::PLANE;
    }
    {
        const int xo = x0 + tx, yo = y0 + ty;
        const bool store = xo < g.nx && yo < g.ny;
        // state offsets are taken from the ghost corner (-3, -3) of the plane
        auto soff = [&](int x, int y) {
            return (unsigned)(((y + kR) * g.px + (x + kR)) * (int)sizeof(T));
        };
        X.lane_o = store ? soff(xo, yo) : kDropOffset;
        X.lane_w = store ? (unsigned)((yo * g.wpx + xo) * (int)sizeof(TW)) : kDropOffset;
    }

    SweepRegs<T, NH> R;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            R.q[f][s] = T(0);
            R.dd[s >> 1][(2 * f + (s & 1))] = T(0);
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int s = 0; s < 8; ++s) R.L[i][s] = T(0);

    const int nplanes = (ze - zb) + 2 * kR;
    if constexpr (LD)
        sweep_dma<T, TX, TY>(X, in, plane_corner(g, zb - kR), lds3);
    else
        sweep_prefetch<T, TX, TY, NH>(R, X, in, plane_corner(g, zb - kR));
    for (int t0 = 0; t0 < nplanes; t0 += 8) {
        sweep_step<0, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<1, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<2, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<3, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<4, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<5, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<6, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
        sweep_step<7, S, LD>(t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, cf, rk);
    }
}

// WV > 0 asks the compiler to fit WV waves per SIMD (a register budget of
// 512 / WV per lane); 0 leaves the choice to the compiler.
template <int WV>
struct WavesAttr {
    static constexpr int lo = WV > 0 ? WV : 1;
    static constexpr int hi = WV > 0 ? WV : 8;
};

template <typename T, typename TW, int TX, int TY, int S, int WV, bool LD>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WavesAttr<WV>::lo,
                                                                         WavesAttr<WV>::hi)))
void substep55_sweep(Geom g, Fields4<T> in, Fields4<T> out,
                                                          Fields4<TW> w, Coef<T> cf,
                                                          RKCoef<TW> rk, int ntx, int nty,
                                                          int zlen, int remap) {
    using Sh = SweepShape<T, TX, TY, LD>;
    __shared__ T lds[2 * 4 * Sh::FS];

    // workgroup -> tile: consecutive tiles (x fastest, then y, then z chunk)
    // go to the same XCD, which receives every 8th workgroup
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if (remap && (nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tix = b % ntx;
    const int tiy = (b / ntx) % nty;
    const int ch = b / (ntx * nty);
    const int zb = ch * zlen;
    const int ze = min(zb + zlen, g.nz);
    if (zb >= ze) return;
    sweep_tile<T, TW, TX, TY, S, LD>(g, in, out, w, cf, rk, tix * TX, tiy * TY, zb, ze, lds,
                                     (lds_t<T>)lds);
}

// Batched form: one persistent launch advances every box of an ensemble by
// one substep.  The host lists the tile-chunks of all boxes (longest first);
// workgroup b takes list entries remap(b), remap(b) + G, ... where the remap
// gives each XCD a contiguous run of the list, so that tiles of one box share
// that XCD's L2.  Per-box geometry, pointers, coefficients and time step come
// from device memory, so a captured graph never needs re-capture when they
// change.  Per point the arithmetic is the single-box kernel's.
template <typename T, typename TW, int TX, int TY, int S, int WV, bool LD>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WavesAttr<WV>::lo,
                                                                         WavesAttr<WV>::hi)))
void substep55_batch(const BatchBox<T, TW>* __restrict__ boxes,
                                                          const BatchItem* __restrict__ items,
                                                          int nitems, int parity, TW alpha,
                                                          TW beta) {
    using Sh = SweepShape<T, TX, TY, LD>;
    __shared__ T lds[2 * 4 * Sh::FS];
    const int G = gridDim.x;
    int b = blockIdx.x;
    if ((G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
    for (int it = b; it < nitems; it += G) {
        const BatchItem wi = items[it];
        const BatchBox<T, TW>* bx = boxes + wi.box;
        const Geom g = bx->g;
        const Coef<T> cf = bx->cf;
        const Fields4<T> in = bx->st[parity], out = bx->st[parity ^ 1];
        const Fields4<TW> w = bx->w;
        const RKCoef<TW> rk{alpha, beta, bx->dt};
        sweep_tile<T, TW, TX, TY, S, LD>(g, in, out, w, cf, rk, wi.x0, wi.y0, wi.zb, wi.ze, lds,
                                         (lds_t<T>)lds);
        __syncthreads();  // the next item's first LDS write must follow every read
    }
}

// Tile configurations (TX, TY).  Index 0 is the direct kernel.
// waves: register budget target (0 = compiler's choice); ld: LDS loader.
struct TileCfg {
    int tx, ty, waves;
    bool ld;
};
constexpr TileCfg kTiles[] = {
    {0, 0, 0, false},    {64, 4, 0, false}, {64, 2, 0, false}, {32, 8, 0, false},
    {64, 8, 0, false},   {128, 4, 0, false}, {128, 2, 0, false}, {64, 6, 0, false},
    {64, 4, 3, false},   {64, 6, 3, false}, {64, 8, 0, true},   {128, 4, 0, true},
    {64, 4, 3, true},    {64, 6, 3, true},  {32, 8, 0, true},   {64, 4, 0, true}};

constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// Workgroup-to-XCD remapping of tiles (FD6_XCD_REMAP=0 disables it).
inline int xcd_remap() {
    static const int v = [] {
        const char* e = getenv("FD6_XCD_REMAP");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    return v;
}

template <typename T, typename TW, int TX, int TY, int WV = 0, bool LD = false>
hipError_t launch_sweep(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                        const Coef<T>& c, const RKCoef<TW>& rk, int s, hipStream_t st) {
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
    const long long tiles = (long long)ntx * nty;
    // enough workgroups to fill 256 CUs several times over; z chunks cost 6
    // extra planes of loads each, so keep them long
    long long want = 2048;
    int nch = (int)((want + tiles - 1) / tiles);
    int maxch = (g.nz + 15) / 16;  // chunks of at least 16 planes
    if (nch > maxch) nch = maxch;
    if (nch < 1) nch = 1;
    const int zlen = (g.nz + nch - 1) / nch;
    nch = (g.nz + zlen - 1) / zlen;
    const dim3 grid((unsigned)(tiles * nch));
    const dim3 block(TX * TY);
    const int rm = xcd_remap();
    switch (s) {
    case 1:
        hipLaunchKernelGGL((substep55_sweep<T, TW, TX, TY, 1, WV, LD>), grid, block, 0, st, g, in, out,
                           w, c, rk, ntx, nty, zlen, rm);
        break;
    case 2:
        hipLaunchKernelGGL((substep55_sweep<T, TW, TX, TY, 2, WV, LD>), grid, block, 0, st, g, in, out,
                           w, c, rk, ntx, nty, zlen, rm);
        break;
    default:
        hipLaunchKernelGGL((substep55_sweep<T, TW, TX, TY, 3, WV, LD>), grid, block, 0, st, g, in, out,
                           w, c, rk, ntx, nty, zlen, rm);
        break;
    }
    return hipGetLastError();
}

template <typename T, typename TW>
hipError_t launch_direct(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                         const Coef<T>& c, const RKCoef<TW>& rk, int s, hipStream_t st) {
    const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)g.nz);
    switch (s) {
    case 1:
        hipLaunchKernelGGL((substep55_direct<T, TW, 1>), grid, dim3(256), 0, st, g, in, out, w,
                           c, rk);
        break;
    case 2:
        hipLaunchKernelGGL((substep55_direct<T, TW, 2>), grid, dim3(256), 0, st, g, in, out, w,
                           c, rk);
        break;
    default:
        hipLaunchKernelGGL((substep55_direct<T, TW, 3>), grid, dim3(256), 0, st, g, in, out, w,
                           c, rk);
        break;
    }
    return hipGetLastError();
}

}  // namespace


template <typename T, typename TW>
hipError_t launch_substep55(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                            const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                            hipStream_t st) {
    switch (tile) {
    case 0: return launch_direct<T, TW>(g, in, out, w, c, rk, s, st);
    case 1: return launch_sweep<T, TW, 64, 4>(g, in, out, w, c, rk, s, st);
    case 2: return launch_sweep<T, TW, 64, 2>(g, in, out, w, c, rk, s, st);
    case 3: return launch_sweep<T, TW, 32, 8>(g, in, out, w, c, rk, s, st);
    case 4: return launch_sweep<T, TW, 64, 8>(g, in, out, w, c, rk, s, st);
    case 5: return launch_sweep<T, TW, 128, 4>(g, in, out, w, c, rk, s, st);
    case 6: return launch_sweep<T, TW, 128, 2>(g, in, out, w, c, rk, s, st);
    case 7: return launch_sweep<T, TW, 64, 6>(g, in, out, w, c, rk, s, st);
    case 8: return launch_sweep<T, TW, 64, 4, 3>(g, in, out, w, c, rk, s, st);
    case 9: return launch_sweep<T, TW, 64, 6, 3>(g, in, out, w, c, rk, s, st);
    case 10: return launch_sweep<T, TW, 64, 8, 0, true>(g, in, out, w, c, rk, s, st);
    case 11: return launch_sweep<T, TW, 128, 4, 0, true>(g, in, out, w, c, rk, s, st);
    case 12: return launch_sweep<T, TW, 64, 4, 3, true>(g, in, out, w, c, rk, s, st);
    case 13: return launch_sweep<T, TW, 64, 6, 3, true>(g, in, out, w, c, rk, s, st);
    case 14: return launch_sweep<T, TW, 32, 8, 0, true>(g, in, out, w, c, rk, s, st);
    case 15: return launch_sweep<T, TW, 64, 4, 0, true>(g, in, out, w, c, rk, s, st);
    default: return hipErrorInvalidValue;
    }
}


namespace {
template <typename T, typename TW, int TX, int TY, int WV = 0, bool LD = false>
hipError_t launch_batch_t(const BatchBox<T, TW>* boxes, const BatchItem* items, int nitems,
                          int grid, int parity, int s, TW alpha, TW beta, hipStream_t st) {
    const dim3 block(TX * TY);
    switch (s) {
    case 1:
        hipLaunchKernelGGL((substep55_batch<T, TW, TX, TY, 1, WV, LD>), dim3(grid), block, 0, st, boxes,
                           items, nitems, parity, alpha, beta);
        break;
    case 2:
        hipLaunchKernelGGL((substep55_batch<T, TW, TX, TY, 2, WV, LD>), dim3(grid), block, 0, st, boxes,
                           items, nitems, parity, alpha, beta);
        break;
    default:
        hipLaunchKernelGGL((substep55_batch<T, TW, TX, TY, 3, WV, LD>), dim3(grid), block, 0, st, boxes,
                           items, nitems, parity, alpha, beta);
        break;
    }
    return hipGetLastError();
}

template <typename T, typename TW, int TX, int TY, int WV = 0, bool LD = false>
int batch_occupancy_t() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, substep55_batch<T, TW, TX, TY, 2, WV, LD>,
                                                     TX * TY, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
}  // namespace


template <typename T, typename TW>
hipError_t launch_batch55(const BatchBox<T, TW>* boxes, const BatchItem* items, int nitems,
                          int grid, int parity, int s, int tile, TW alpha, TW beta,
                          hipStream_t st) {
    switch (tile) {
    case 1: return launch_batch_t<T, TW, 64, 4>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 2: return launch_batch_t<T, TW, 64, 2>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 3: return launch_batch_t<T, TW, 32, 8>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 4: return launch_batch_t<T, TW, 64, 8>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 5: return launch_batch_t<T, TW, 128, 4>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 6: return launch_batch_t<T, TW, 128, 2>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 7: return launch_batch_t<T, TW, 64, 6>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 8: return launch_batch_t<T, TW, 64, 4, 3>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 9: return launch_batch_t<T, TW, 64, 6, 3>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 10: return launch_batch_t<T, TW, 64, 8, 0, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 11: return launch_batch_t<T, TW, 128, 4, 0, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 12: return launch_batch_t<T, TW, 64, 4, 3, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 13: return launch_batch_t<T, TW, 64, 6, 3, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 14: return launch_batch_t<T, TW, 32, 8, 0, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    case 15: return launch_batch_t<T, TW, 64, 4, 0, true>(boxes, items, nitems, grid, parity, s, alpha, beta, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, typename TW>
int batch55_blocks_per_cu(int tile) {
    switch (tile) {
    case 1: return batch_occupancy_t<T, TW, 64, 4>();
    case 2: return batch_occupancy_t<T, TW, 64, 2>();
    case 3: return batch_occupancy_t<T, TW, 32, 8>();
    case 4: return batch_occupancy_t<T, TW, 64, 8>();
    case 5: return batch_occupancy_t<T, TW, 128, 4>();
    case 6: return batch_occupancy_t<T, TW, 128, 2>();
    case 7: return batch_occupancy_t<T, TW, 64, 6>();
    case 8: return batch_occupancy_t<T, TW, 64, 4, 3>();
    case 9: return batch_occupancy_t<T, TW, 64, 6, 3>();
    case 10: return batch_occupancy_t<T, TW, 64, 8, 0, true>();
    case 11: return batch_occupancy_t<T, TW, 128, 4, 0, true>();
    case 12: return batch_occupancy_t<T, TW, 64, 4, 3, true>();
    case 13: return batch_occupancy_t<T, TW, 64, 6, 3, true>();
    case 14: return batch_occupancy_t<T, TW, 32, 8, 0, true>();
    case 15: return batch_occupancy_t<T, TW, 64, 4, 0, true>();
    default: return 1;
    }
}

}  // namespace fd6
