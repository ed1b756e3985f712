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
//    register; the workgroup-to-tile map gives each XCD a near-square block
//    of neighbouring tiles, so most halo cells are served from its L2.
//  * Template switches: VS = 4 reads and writes the array-of-structures
//    layout (one 16-byte access per cell and field set); NT streams the new
//    state and the RK3 register past the caches; FRC adds the external
//    force; RED accumulates the FP64 diagnostics; P19 turns the sweep into
//    pass 1 of the 19-point method.
#pragma once

#include "sweep_common.hpp"

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

template <typename T, typename TW, int S, bool FRC>
__global__ __launch_bounds__(256) void substep55_direct(Geom g, Fields4<T> in, Fields4<T> out,
                                                        Fields4<TW> w, Coef<T> cf, RKCoef<TW> rk,
                                                        ForceArgs<T> fa) {
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
        TW wv = (S == 1) ? TW(0) : w.f[q][cw];
        out.f[q][c] = rk_update<S>(in.f[q][c], r[q], wv, rk);
        if (S != 3) w.f[q][cw] = wv;
    }
}

// ---------------------------------------------------------------------------
// z-sweep kernel
// ---------------------------------------------------------------------------

template <typename T, typename TW, int NH>
struct SweepRegs {
    T q[4][8];       // raw column values of the 4 fields, ring over planes
    T L[3][8];       // pending linear viscous term of the 3 momentum components
    T dd[4][8];      // x/y first derivatives of the 4 fields, ring of 4 planes
    T pf[4][4];      // prefetched interior values of the next plane(s)
    T ph[4][NH][4];  // prefetched halo values of the next plane(s)
    TW wq[2][4];     // RK3 register of the output point (PD = 2: loaded a step early)
    double red[4];   // fused diagnostics of the thread's column (RED): sum rho,
                     // sum rho u^2, sum lnrho, max u^2
    int bad;         // RED: points of the column with a non-finite value
    T fc, fs;        // FRC: cos / sin(kx x + ky y) of the thread's column
    T fa[3];         // FRC: force amplitude vector
};

// Memory operations of a plane step are never skipped by a branch: a step
// that has nothing to load or store gives its descriptors a zero range (loads
// return 0, stores are dropped).  Branch-free memory code lets the compiler
// count outstanding loads exactly across steps instead of draining the memory
// pipeline (stores share the load counter on this architecture).

// Loads plane `corner` of the four fields (this thread's cells) into
// register set RS; bytes = 0 loads nothing.
template <int RS, int VS, typename T, typename TW, int TX, int TY, int NH>
__device__ __forceinline__ void sweep_prefetch(SweepRegs<T, TW, NH>& R,
                                               const SweepCtx<T, TX, TY>& X,
                                               const Fields4<T>& in, long long corner,
                                               unsigned bytes) {
    if constexpr (VS == 4) {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in.f[0] + 4 * corner, bytes);
        bload_point(R.pf[RS], rs, X.goff_int);
#pragma unroll
        for (int h = 0; h < NH; ++h) bload_point(R.ph[RS][h], rs, X.goff_h[h]);
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in.f[f] + corner, bytes);
            R.pf[RS][f] = bload((T*)nullptr, rs, X.goff_int);
#pragma unroll
            for (int h = 0; h < NH; ++h) R.ph[RS][h][f] = bload((T*)nullptr, rs, X.goff_h[h]);
        }
    }
}

template <int RS, bool NT, int VS, typename T, typename TW, int NH>
__device__ __forceinline__ void load_w(SweepRegs<T, TW, NH>& R, const Fields4<TW>& w,
                                       const Geom& g, int o, unsigned wplane_bytes,
                                       unsigned lane_w) {
    constexpr int CP = NT ? kNonTemporal : 0;
    if constexpr (VS == 4) {
        bload_point<CP>(R.wq[RS], plane_rsrc(w.f[0] + 4 * (long long)o * g.wplane, wplane_bytes),
                        lane_w);
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f)
            R.wq[RS][f] = bload<CP>((TW*)nullptr,
                                    plane_rsrc(w.f[f] + (long long)o * g.wplane, wplane_bytes),
                                    lane_w);
    }
}

// LD: copy plane `corner` of the four fields into one LDS buffer.  Chunk j
// (64 dwords) is issued by wave j % NW; its lanes fetch the dwords whose byte
// offsets were precomputed in doff (periodic images included).
template <typename T, int TX, int TY>
__device__ __forceinline__ void sweep_dma(const SweepCtx<T, TX, TY, true>& X,
                                          const Fields4<T>& in, long long corner, lds_t<T> buf,
                                          unsigned bytes) {
    using Sh = SweepShape<T, TX, TY, true>;
    const int wv = threadIdx.x / 64;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in.f[f] + corner, bytes);
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

// TB selects the two stages of the substep-1+2 fusion (fused12_tile): 0 is
// the plain sweep; 1 is substep 1 over the extended region, whose new state
// goes to the LDS plane buffer tb_u (layout of the inner tile's sweep) and
// whose RK3 register, for the inner columns, to the LDS ring tb_w; 2 is
// substep 2 of the inner tile, which takes its plane from tb_u (passed as
// lds, loaded by stage 1) and its RK3 register from tb_w, and starts output
// planes 2 * kR steps later.
template <int PH, int S, int PD, bool LD, bool NT, int VS, bool P19, bool RED, bool FRC,
          int TB = 0, bool DDL = false, typename T, typename TW, int TX, int TY, int NH>
__device__ __forceinline__ void sweep_step(int t0, int nplanes, int zb, SweepRegs<T, TW, NH>& R,
                                           const SweepCtx<T, TX, TY, LD>& X, T* lds,
                                           lds_t<T> lds3, const Geom& g, const Fields4<T>& in,
                                           const Fields4<T>& out, const Fields4<TW>& w, T* dv,
                                           const Coef<T>& cf, const RKCoef<TW>& rk,
                                           const T* ftab, T* tb_u = nullptr,
                                           TW* tb_w = nullptr, T* ddl = nullptr) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr int W = Sh::W;
    static_assert(TB == 0 || (!LD && !P19 && !RED && !FRC), "fusion: plain register sweep only");
    static_assert(!DDL || TB == 0, "LDS derivative slots: plain sweep only");
    // DDL: the x / y first derivatives of a plane wait for their output in
    // this thread's LDS slots instead of registers (slot, field pair, thread)
    using T2 = T __attribute__((ext_vector_type(2)));
    T2* const dd2 = reinterpret_cast<T2*>(ddl);
    // PIPE: the pinned order of phase (C) below; it pays where one wave runs per
    // SIMD and the LDS slots left registers for the copies (FP64, the same
    // kernels as DDL)
    constexpr bool PIPE = DDL;
    const int t = t0 + PH;
    if (t >= nplanes) return;
    const int p = zb - kR + t;  // plane loaded in this step
    const int o = p - kR;       // output plane finished in this step
    const bool outstep = t >= (TB == 2 ? 4 : 2) * kR;

    T* buf = lds + (PH & 1) * 4 * Sh::FS;
    const int ci = (threadIdx.x / TX + kR) * W + (threadIdx.x % TX + kR);
    // register sets: plane p sits in set RS (PD sets, PD divides the unroll
    // of 8); the RK3 register of output o in set WS
    static_assert(PD == 1 || PD == 2 || PD == 4, "prefetch depth");
    constexpr int RS = PH % PD;
    constexpr int WS = PD >= 2 ? (PH & 1) : 0;
    if constexpr (TB == 2) {
        // plane p was written to LDS by stage 1 of this step (barrier between)
    } else if constexpr (!LD) {
        // RK3 register of an output point, issued early: PD = 1 loads the one
        // finished in this step, PD = 2 the one finished in the next step
        if constexpr (S != 1) {
            if constexpr (PD >= 2) {
                const bool next_out = t + 1 >= 2 * kR && t + 1 < nplanes;
                load_w<(PH + 1) & 1, NT, VS>(R, w, g, o + 1, next_out ? X.wplane_bytes : 0u,
                                             X.lane_w);
            } else {
                load_w<0, NT, VS>(R, w, g, o, outstep ? X.wplane_bytes : 0u, X.lane_w);
            }
        }
        // prefetched plane p -> LDS buffer (PH & 1)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            buf[f * Sh::FS + ci] = R.pf[RS][f];
#pragma unroll
            for (int h = 0; h < NH; ++h) buf[f * Sh::FS + X.loff_h[h]] = R.ph[RS][h][f];
        }
        // plane p + PD -> the register set just emptied
        sweep_prefetch<RS, VS>(R, X, in, plane_corner(g, p + PD),
                               t + PD < nplanes ? X.plane_bytes : 0u);
        __syncthreads();
    } else {
        // this wave's copies of plane p are complete before the barrier; after
        // it the other buffer (read in the previous step by every wave) takes
        // plane p + 1
        __syncthreads();
        sweep_dma<T, TX, TY>(X, in, plane_corner(g, p + 1), lds3 + ((PH + 1) & 1) * 4 * Sh::FS,
                             t + 1 < nplanes ? X.plane_bytes : 0u);
        if constexpr (S != 1) {
            load_w<0, NT, VS>(R, w, g, o, outstep ? X.wplane_bytes : 0u, X.lane_w);
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
    // The 19-point form has no mixed terms.
    {
        R.q[0][sl8(PH)] = B0[0];
        R.q[1][sl8(PH)] = B1[0];
        R.q[2][sl8(PH)] = B2[0];
        R.q[3][sl8(PH)] = B3[0];
    }
    if constexpr (!P19) {
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

    // PIPE: register copies of the fields' x / y windows (the cross and the
    // diagonals through the column), each filled from LDS one field ahead of
    // its arithmetic, with the order pinned, so that the LDS latency overlaps
    // the arithmetic before it (the output plane's for ln rho).  The
    // operations and their operands are those of the plain order.
    [[maybe_unused]] T wv[PIPE ? 4 : 1][PIPE ? 7 * W : 1];
    [[maybe_unused]] auto fill = [&](T* wf, const T* Bf) {
#pragma unroll
        for (int dy = -kR; dy <= kR; ++dy)
#pragma unroll
            for (int dx = -kR; dx <= kR; ++dx)
                if (dy == 0 || dx == 0 || dy == dx || dy == -dx)
                    wf[C0 + dy * W + dx] = Bf[dy * W + dx];
    };
    if constexpr (PIPE) {
        fill(wv[0], B0);
        __builtin_amdgcn_sched_barrier(0);
    }

    // (B) finish output plane o = p - 3 before the rest of plane p is formed,
    // so the two working sets do not overlap in registers.  In the first 6
    // steps of a chunk there is no output plane yet: the arithmetic runs on
    // the zero-initialised rings and the stores are dropped.
    {
        const unsigned ob = outstep ? X.plane_bytes : 0u;
        const unsigned wb = outstep ? X.wplane_bytes : 0u;
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
            Lf[i] = R.L[i][sl8(PH - 3)] + ((i == 2 && !P19) ? cf.sg4[2] : cf.sg[2]) * rz;
        }
        constexpr int DO = (PH + 1) & 3;  // slot of plane p - 3
        T dxy[8];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if constexpr (DDL) {
                const T2 v = dd2[(DO * 4 + f) * Sh::NT + threadIdx.x];
                dxy[2 * f] = v.x;
                dxy[2 * f + 1] = v.y;
            } else {
                dxy[2 * f] = R.dd[DO][2 * f];
                dxy[2 * f + 1] = R.dd[DO][2 * f + 1];
            }
        }
        const T gr[3] = {dxy[0], dxy[1], dz[0]};
        const T J[3][3] = {{dxy[2], dxy[3], dz[1]}, {dxy[4], dxy[5], dz[2]}, {dxy[6], dxy[7], dz[3]}};
        const T u[3] = {R.q[1][sl8(PH - 3)], R.q[2][sl8(PH - 3)], R.q[3][sl8(PH - 3)]};
        T r[4];
        assemble_rhs(u, gr, J, Lf, cf.nu, cf.cs2, r);
        if constexpr (FRC) {
            // f = a cos(k.x + phase) at the output point (eq. forcing); the
            // plane index wraps for the steps without an output plane
            // the table is read-only during the kernel: reading it through the
            // constant address space makes these scalar loads, which keep out
            // of the vector-memory counter the sweep's pipeline depends on
            const int ow = o < 0 ? o + g.nz : o;
            const __attribute__((address_space(4))) T* ct =
                (const __attribute__((address_space(4))) T*)ftab;
            const T cz = ct[2 * ow], sz = ct[2 * ow + 1];
            const T ph = R.fc * cz - R.fs * sz;
#pragma unroll
            for (int i = 0; i < 3; ++i) r[1 + i] += R.fa[i] * ph;
        }
        // ghost corner (-3, -3) of output plane o
        const long long ocorner = g.origin + (long long)o * g.plane - kR * g.px - kR;
        constexpr int CP = NT ? kNonTemporal : 0;
        T vout[4];
        TW wout[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            // stage 2 of the fusion: the register stage 1 wrote 3 steps earlier
            TW wv = S == 1 ? TW(0)
                           : (TB == 2 ? tb_w[((PH + 1) & 3) * 4 * (TX * TY) + f * (TX * TY) +
                                             threadIdx.x]
                                      : R.wq[WS][f]);
            const T v = rk_update<S>(R.q[f][sl8(PH - 3)], r[f], wv, rk);
            vout[f] = v;
            wout[f] = wv;
            if constexpr (TB == 1) {
                // new state of every extended column into the inner sweep's
                // plane buffer (its cell is this thread's index); the register
                // of the inner columns into ring slot (step & 3)
                constexpr int NI = (TX - 2 * kR) * (TY - 2 * kR);
                constexpr int FS2 = SweepShape<T, TX - 2 * kR, TY - 2 * kR>::FS;
                tb_u[(PH & 1) * 4 * FS2 + f * FS2 + threadIdx.x] = v;
                const int ix = (int)(threadIdx.x % TX) - kR, iy = (int)(threadIdx.x / TX) - kR;
                if (ix >= 0 && ix < TX - 2 * kR && iy >= 0 && iy < TY - 2 * kR)
                    tb_w[(PH & 3) * 4 * NI + f * NI + iy * (TX - 2 * kR) + ix] = wv;
            } else if constexpr (VS == 1) {
                bstore<CP>(v, plane_rsrc(out.f[f] + ocorner, ob), X.lane_o);
                if constexpr (S != 3)
                    bstore<CP>(wv, plane_rsrc(w.f[f] + (long long)o * g.wplane, wb), X.lane_w);
            }
        }
        if constexpr (VS == 4 && TB != 1) {
            bstore_point<CP>(vout, plane_rsrc(out.f[0] + 4 * ocorner, ob), X.lane_o);
            if constexpr (S != 3)
                bstore_point<CP>(wout, plane_rsrc(w.f[0] + 4 * (long long)o * g.wplane, wb),
                                 X.lane_w);
        }
        // 19-point pass 1 also stores the divergence for pass 2
        if constexpr (P19)
            bstore(J[0][0] + J[1][1] + J[2][2], plane_rsrc(dv + ocorner, ob), X.lane_o);
        // FP64 diagnostics of the new state, from the values just stored (the
        // same per-point quantities as the standalone reduction)
        if constexpr (RED) {
            if (outstep && X.lane_o != kDropOffset)
                red_point(R.red, R.bad, vout[0], vout[1], vout[2], vout[3]);
        }
    }

    // (C) the rest of plane p for this column: x / y first derivatives of the
    // four fields (kept 3 planes), the xy part of the linear viscous term, and
    // the k = 1, 2 terms of the xz / yz stencils of outputs p -+ k.
    auto dd_put = [&](int f, T dx, T dy) {
        if constexpr (DDL) {
            dd2[(DS * 4 + f) * Sh::NT + threadIdx.x] = T2{dx, dy};
        } else {
            R.dd[DS][2 * f] = dx;
            R.dd[DS][2 * f + 1] = dy;
        }
    };
    T lx, ly, lz;  // xy parts of nu (lap u_i + (1/3) d_i div u) at plane p (19-point:
                   // of nu lap u_i)
    T zx[2], zy[2], zz[2];  // scaled k = 1, 2 differences feeding the xz / yz terms
    if constexpr (PIPE) {
        // lnrho
        auto c_lnrho = [&](const T* F) {
            dd_put(0,
                   cf.d1[0][0] * (F[1] - F[-1]) + cf.d1[0][1] * (F[2] - F[-2]) +
                       cf.d1[0][2] * (F[3] - F[-3]),
                   cf.d1[1][0] * (F[W] - F[-W]) + cf.d1[1][1] * (F[2 * W] - F[-2 * W]) +
                       cf.d1[1][2] * (F[3 * W] - F[-3 * W]));
        };
        // ux
        auto c_ux = [&](const T* F) {
            const T c = F[0];
            T a[3], b[3];
            T rx = T(0), ry = T(0), m = T(0);
    #pragma unroll
            for (int k = 1; k <= 3; ++k) {
                const T xp = F[k], xm = F[-k], yp = F[k * W], ym = F[-k * W];
                a[k - 1] = xp - xm;
                b[k - 1] = yp - ym;
                rx += w2[k - 1] * (xp + xm);
                ry += w2[k - 1] * (yp + ym);
                if constexpr (!P19) {
                    const T t = (F[k * W + k] - F[k * W - k]) + (F[-k * W - k] - F[-k * W + k]);
                    m += w2[k - 1] * t;
                }
            }
            dd_put(1, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            if constexpr (P19) {
                lx = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
                ly = T(0);
            } else {
                lx = cf.kxy[0] * c + cf.sg4[0] * rx + cf.sg[1] * ry;  // (4/3) D2x + D2y
                ly = cf.mu[0] * m;                                     // (1/3) Dxy ux
            }
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) zz[k] = cf.mu[1] * a[k];  // (1/3) Dxz ux
            }
        };
        // uy
        auto c_uy = [&](const T* F) {
            const T c = F[0];
            T a[3], b[3];
            T rx = T(0), ry = T(0), m = T(0);
    #pragma unroll
            for (int k = 1; k <= 3; ++k) {
                const T xp = F[k], xm = F[-k], yp = F[k * W], ym = F[-k * W];
                a[k - 1] = xp - xm;
                b[k - 1] = yp - ym;
                rx += w2[k - 1] * (xp + xm);
                ry += w2[k - 1] * (yp + ym);
                if constexpr (!P19) {
                    const T t = (F[k * W + k] - F[k * W - k]) + (F[-k * W - k] - F[-k * W + k]);
                    m += w2[k - 1] * t;
                }
            }
            dd_put(2, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            if constexpr (P19) {
                ly = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
            } else {
                ly += cf.kxy[1] * c + cf.sg[0] * rx + cf.sg4[1] * ry;  // D2x + (4/3) D2y
                lx += cf.mu[0] * m;                                     // (1/3) Dxy uy
            }
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) zz[k] += cf.mu[2] * b[k];  // (1/3) Dyz uy
            }
        };
        // uz
        auto c_uz = [&](const T* F) {
            const T c = F[0];
            T a[3], b[3];
            T rx = T(0), ry = T(0);
    #pragma unroll
            for (int k = 1; k <= 3; ++k) {
                const T xp = F[k], xm = F[-k], yp = F[k * W], ym = F[-k * W];
                a[k - 1] = xp - xm;
                b[k - 1] = yp - ym;
                rx += w2[k - 1] * (xp + xm);
                ry += w2[k - 1] * (yp + ym);
            }
            dd_put(3, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            lz = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) {
                    zx[k] = cf.mu[1] * a[k];  // (1/3) Dxz uz
                    zy[k] = cf.mu[2] * b[k];  // (1/3) Dyz uy
                }
            }
        };
        // stages: [next window, this field's arithmetic], pinned apart
        __builtin_amdgcn_sched_barrier(0);
        fill(wv[1], B1);
        c_lnrho(wv[0] + C0);
        __builtin_amdgcn_sched_barrier(0);
        fill(wv[2], B2);
        c_ux(wv[1] + C0);
        __builtin_amdgcn_sched_barrier(0);
        fill(wv[3], B3);
        c_uy(wv[2] + C0);
        __builtin_amdgcn_sched_barrier(0);
        c_uz(wv[3] + C0);
    } else {
        dd_put(0,
               cf.d1[0][0] * (B0[1] - B0[-1]) + cf.d1[0][1] * (B0[2] - B0[-2]) +
                   cf.d1[0][2] * (B0[3] - B0[-3]),
               cf.d1[1][0] * (B0[W] - B0[-W]) + cf.d1[1][1] * (B0[2 * W] - B0[-2 * W]) +
                   cf.d1[1][2] * (B0[3 * W] - B0[-3 * W]));
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
                if constexpr (!P19) {
                    const T t = (B1[k * W + k] - B1[k * W - k]) + (B1[-k * W - k] - B1[-k * W + k]);
                    m += w2[k - 1] * t;
                }
            }
            dd_put(1, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            if constexpr (P19) {
                lx = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
                ly = T(0);
            } else {
                lx = cf.kxy[0] * c + cf.sg4[0] * rx + cf.sg[1] * ry;  // (4/3) D2x + D2y
                ly = cf.mu[0] * m;                                     // (1/3) Dxy ux
            }
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) zz[k] = cf.mu[1] * a[k];  // (1/3) Dxz ux
            }
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
                if constexpr (!P19) {
                    const T t = (B2[k * W + k] - B2[k * W - k]) + (B2[-k * W - k] - B2[-k * W + k]);
                    m += w2[k - 1] * t;
                }
            }
            dd_put(2, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            if constexpr (P19) {
                ly = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
            } else {
                ly += cf.kxy[1] * c + cf.sg[0] * rx + cf.sg4[1] * ry;  // D2x + (4/3) D2y
                lx += cf.mu[0] * m;                                     // (1/3) Dxy uy
            }
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) zz[k] += cf.mu[2] * b[k];  // (1/3) Dyz uy
            }
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
            dd_put(3, cf.d1[0][0] * a[0] + cf.d1[0][1] * a[1] + cf.d1[0][2] * a[2],
                   cf.d1[1][0] * b[0] + cf.d1[1][1] * b[1] + cf.d1[1][2] * b[2]);
            lz = cf.kp * c + cf.sg[0] * rx + cf.sg[1] * ry;  // D2x + D2y
            if constexpr (!P19) {
    #pragma unroll
                for (int k = 0; k < 2; ++k) {
                    zx[k] = cf.mu[1] * a[k];  // (1/3) Dxz uz
                    zy[k] = cf.mu[2] * b[k];  // (1/3) Dyz uy
                }
            }
        }
    }

    // Scatter: the bidiagonal xz / yz stencil at output z is
    // sum_k c_k [A_k(z + k) - A_k(z - k)], so plane p adds +c_k A_k to the
    // pending output p - k and -c_k A_k to p + k (c = 270, -27, 2); the k = 3
    // terms were added in (A).
    if constexpr (P19) {
        R.L[0][sl8(PH)] = lx;
        R.L[1][sl8(PH)] = ly;
        R.L[2][sl8(PH)] = lz;
    } else {
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
// arguments.  P19: pass 1 of the 19-point method (dv receives the divergence).
// RED: also reduce the FP64 diagnostics of the output and store this
// workgroup's partial at part[blockIdx.x * kReduceSlots ...].
template <typename T, typename TW, int TX, int TY, int S, int PD, bool LD, bool NT, int VS,
          bool P19 = false, bool RED = false, bool FRC = false, bool DDL = false>
__device__ __forceinline__ void sweep_tile(const Geom& g, const Fields4<T>& in,
                                           const Fields4<T>& out, const Fields4<TW>& w, T* dv,
                                           const Coef<T>& cf, const RKCoef<TW>& rk, int x0,
                                           int y0, int zb, int ze, T* lds, lds_t<T> lds3,
                                           double* part = nullptr,
                                           ForceArgs<T> fa = ForceArgs<T>{nullptr, nullptr},
                                           T* ddl = nullptr) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr int NH = Sh::NH;
    SweepCtx<T, TX, TY, LD> X;
    static_assert(VS == 1 || !P19, "the 19-point passes use one array per field");
    sweep_ctx_init<T, TW, TX, TY, LD, VS>(X, g, x0, y0);

    SweepRegs<T, TW, NH> R;
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
#pragma unroll
    for (int i = 0; i < 4; ++i) R.red[i] = 0.0;
    R.bad = 0;
    if constexpr (DDL) {
#pragma unroll
        for (int s = 0; s < 32; ++s) ddl[s * Sh::NT + threadIdx.x] = T(0);
    }
    if constexpr (FRC) {
        const ForceDev<T>* fd = fa.dev;
        const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
        const double ang = fd->kx * ((x0 + tx) * fd->dx) + fd->ky * ((y0 + ty) * fd->dy);
        double sn, cs;
        sincos(ang, &sn, &cs);
        R.fc = T(cs);
        R.fs = T(sn);
#pragma unroll
        for (int i = 0; i < 3; ++i) R.fa[i] = fd->a[i];
    }

    const int nplanes = (ze - zb) + 2 * kR;
    if constexpr (LD) {
        sweep_dma<T, TX, TY>(X, in, plane_corner(g, zb - kR), lds3, X.plane_bytes);
    } else {
        sweep_prefetch<0, VS>(R, X, in, plane_corner(g, zb - kR), X.plane_bytes);
        if constexpr (PD >= 2)
            sweep_prefetch<1, VS>(R, X, in, plane_corner(g, zb - kR + 1), X.plane_bytes);
        if constexpr (PD == 4) {
            // a chunk sweeps at least 7 planes, so these exist
            sweep_prefetch<2, VS>(R, X, in, plane_corner(g, zb - kR + 2), X.plane_bytes);
            sweep_prefetch<3, VS>(R, X, in, plane_corner(g, zb - kR + 3), X.plane_bytes);
        }
    }
    for (int t0 = 0; t0 < nplanes; t0 += 8) {
        sweep_step<0, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<1, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<2, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<3, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<4, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<5, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<6, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
        sweep_step<7, S, PD, LD, NT, VS, P19, RED, FRC, 0, DDL>(
            t0, nplanes, zb, R, X, lds, lds3, g, in, out, w, dv, cf, rk, fa.tab, (T*)nullptr, (TW*)nullptr, ddl);
    }
    if constexpr (RED) red_store_n<SweepShape<T, TX, TY, LD>::NW>(R.red, R.bad, part);
}

// Where the x / y first derivatives wait for their output plane: LDS slots
// for the FP64 array-of-structures register sweeps of at most 256 threads,
// registers otherwise.  Those kernels need more than 256 registers and run
// one wave per SIMD; the slots take about 110 registers off the part kept in
// AGPRs and the copies between the two files.
#ifndef FD6_DD_LDS
#define FD6_DD_LDS 1
#endif
template <typename T, int TX, int TY, bool LD, int VS>
constexpr bool kDdInLds = FD6_DD_LDS && sizeof(T) == 8 && TX * TY <= 256 && !LD && VS == 4;

template <typename T, typename TW, int TX, int TY, int S, int PD, bool LD, bool NT, int VS,
          bool FRC>
__global__ __launch_bounds__(TX* TY)
void substep55_sweep(Geom g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, Coef<T> cf,
                     RKCoef<TW> rk, SweepGrid m, ForceArgs<T> fa) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr bool DDL = kDdInLds<T, TX, TY, LD, VS>;
    __shared__ T lds[2 * 4 * Sh::FS];
    __shared__ __attribute__((aligned(16))) T ddl[DDL ? 32 * TX * TY : 2];
    const TileXY t = sweep_tile_of(g, TX, TY, m);
    if (t.zb >= t.ze) return;
    sweep_tile<T, TW, TX, TY, S, PD, LD, NT, VS, false, false, FRC, DDL>(
        g, in, out, w, nullptr, cf, rk, t.tx, t.ty, t.zb, t.ze, lds, (lds_t<T>)lds, nullptr, fa,
        ddl);
}

// Substeps 1 and 2 of one step in one launch: the temporal blocking the
// paper's discussion of Sec. 7 proposes, in the z-sweep.  A workgroup of
// (TX + 6) x (TY + 6) threads owns a TX x TY output tile.
//  * Stage 1: the substep-1 sweep over the extended tile (the output tile
//    and a 3-column ring), one column per thread, loading the input state as
//    the plain sweep does.  Its new state does not go to memory: plane o1
//    goes into an LDS plane buffer laid out as the inner tile's sweep reads
//    its planes, and the RK3 register of the inner columns into an LDS ring
//    of 4 planes.
//  * Stage 2 (threads 0 .. TX TY - 1, whole waves): the substep-2 sweep of
//    the output tile with that buffer as its plane source, 3 planes behind
//    stage 1, storing the substep-2 state and RK3 register.
// The substep-1 state and register never reach HBM: substeps 1 and 2 move
// 16 + 32 bytes per point (FP32) instead of 48 + 64, at the price of
// substep 1 on (TX + 6)(TY + 6) / (TX TY) times the columns.  Per point the
// arithmetic is the plain sweep's, so the result is bit for bit that of two
// plain launches.  The loaded planes start 2 * kR further back (nplanes =
// chunk + 4 kR).
template <typename T, typename TW, int TX, int TY, int PD, bool NT, int VS>
__device__ __forceinline__ void fused12_tile(const Geom& g, const Fields4<T>& in,
                                             const Fields4<T>& out, const Fields4<TW>& w,
                                             const Coef<T>& cf, const RKCoef<TW>& rk1,
                                             const RKCoef<TW>& rk2, int x0, int y0, int zb,
                                             int ze, T* lds1, T* lds2, TW* ring) {
    constexpr int EX = TX + 2 * kR, EY = TY + 2 * kR;
    using Sh1 = SweepShape<T, EX, EY>;
    using Sh2 = SweepShape<T, TX, TY>;
    static_assert(Sh2::W == EX && Sh2::H == EY, "stage-2 planes are the stage-1 tile");
    static_assert((TX * TY) % 64 == 0, "stage 2 runs on whole waves");
    SweepCtx<T, EX, EY> X1;
    sweep_ctx_init<T, TW, EX, EY, false, VS, true>(X1, g, x0 - kR, y0 - kR);
    SweepCtx<T, TX, TY> X2;
    const bool inner = threadIdx.x < TX * TY;
    if (inner) sweep_ctx_init<T, TW, TX, TY, false, VS>(X2, g, x0, y0);
    SweepRegs<T, TW, Sh1::NH> R1;
    SweepRegs<T, TW, Sh2::NH> R2;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            R1.q[f][s] = R2.q[f][s] = T(0);
            R1.dd[s >> 1][(2 * f + (s & 1))] = R2.dd[s >> 1][(2 * f + (s & 1))] = T(0);
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int s = 0; s < 8; ++s) R1.L[i][s] = R2.L[i][s] = T(0);
    const int nplanes = (ze - zb) + 4 * kR;
    const int zb1 = zb - kR, zb2 = zb - 2 * kR;  // stage 1 outputs from zb - 3
    sweep_prefetch<0, VS>(R1, X1, in, plane_corner(g, zb1 - kR), X1.plane_bytes);
    if constexpr (PD >= 2)
        sweep_prefetch<1, VS>(R1, X1, in, plane_corner(g, zb1 - kR + 1), X1.plane_bytes);
    static_assert(PD == 1 || PD == 2, "prefetch depth of the fused sweep");
    const Fields4<T> none{{nullptr, nullptr, nullptr, nullptr}};
    for (int t0 = 0; t0 < nplanes; t0 += 8) {
#define FD6_FUSED_STEP(PH)                                                                      \
        sweep_step<PH, 1, PD, false, NT, VS, false, false, false, 1>(                            \
            t0, nplanes, zb1, R1, X1, lds1, (lds_t<T>)lds1, g, in, none, w, (T*)nullptr, cf,     \
            rk1, (const T*)nullptr, lds2, ring);                                                 \
        __syncthreads();                                                                         \
        if (inner)                                                                               \
            sweep_step<PH, 2, PD, false, NT, VS, false, false, false, 2>(                        \
                t0, nplanes, zb2, R2, X2, lds2, (lds_t<T>)lds2, g, in, out, w, (T*)nullptr, cf,  \
                rk2, (const T*)nullptr, (T*)nullptr, ring);
        FD6_FUSED_STEP(0)
        FD6_FUSED_STEP(1)
        FD6_FUSED_STEP(2)
        FD6_FUSED_STEP(3)
        FD6_FUSED_STEP(4)
        FD6_FUSED_STEP(5)
        FD6_FUSED_STEP(6)
        FD6_FUSED_STEP(7)
#undef FD6_FUSED_STEP
    }
}

template <typename T, typename TW, int TX, int TY, int PD, bool NT, int VS>
__global__ __launch_bounds__((TX + 2 * kR) * (TY + 2 * kR))
void substep55_fused12(Geom g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, Coef<T> cf,
                       RKCoef<TW> rk1, RKCoef<TW> rk2, SweepGrid m) {
    using Sh1 = SweepShape<T, TX + 2 * kR, TY + 2 * kR>;
    using Sh2 = SweepShape<T, TX, TY>;
    __shared__ T lds1[2 * 4 * Sh1::FS];
    __shared__ T lds2[2 * 4 * Sh2::FS];
    __shared__ TW ring[4 * 4 * TX * TY];
    const TileXY t = sweep_tile_of(g, TX, TY, m);
    if (t.zb >= t.ze) return;
    fused12_tile<T, TW, TX, TY, PD, NT, VS>(g, in, out, w, cf, rk1, rk2, t.tx, t.ty, t.zb, t.ze,
                                            lds1, lds2, ring);
}

// Substep 3 with the FP64 diagnostics of the new state fused in: one partial
// per workgroup (every workgroup of the grid has a non-empty chunk).
template <typename T, typename TW, int TX, int TY, int PD, bool LD, bool NT, int VS, bool FRC>
__global__ __launch_bounds__(TX* TY)
void substep55_sweep_red(Geom g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, Coef<T> cf,
                         RKCoef<TW> rk, SweepGrid m, double* part,
                         ForceArgs<T> fa) {
    using Sh = SweepShape<T, TX, TY, LD>;
    constexpr bool DDL = kDdInLds<T, TX, TY, LD, VS>;
    __shared__ T lds[2 * 4 * Sh::FS];
    __shared__ __attribute__((aligned(16))) T ddl[DDL ? 32 * TX * TY : 2];
    const TileXY t = sweep_tile_of(g, TX, TY, m);
    sweep_tile<T, TW, TX, TY, 3, PD, LD, NT, VS, false, true, FRC, DDL>(
        g, in, out, w, nullptr, cf, rk, t.tx, t.ty, t.zb, t.ze, lds, (lds_t<T>)lds, part, fa, ddl);
}

// Pass 1 of the 19-point method (Sec. 4.2, Algorithm 3): the same sweep
// without the mixed-derivative terms, with nu lap u in place of the viscous
// operator, and the divergence stored for pass 2.
template <typename T, typename TW, int TX, int TY, int S, int PD, bool LD, bool NT, bool FRC>
__global__ __launch_bounds__(TX* TY)
void substep19_pass1(Geom g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, T* dv, Coef<T> cf,
                     RKCoef<TW> rk, SweepGrid m, ForceArgs<T> fa) {
    using Sh = SweepShape<T, TX, TY, LD>;
    __shared__ T lds[2 * 4 * Sh::FS];
    const TileXY t = sweep_tile_of(g, TX, TY, m);
    if (t.zb >= t.ze) return;
    sweep_tile<T, TW, TX, TY, S, PD, LD, NT, 1, true, false, FRC>(
        g, in, out, w, dv, cf, rk, t.tx, t.ty, t.zb, t.ze, lds, (lds_t<T>)lds, nullptr, fa);
}

// Batched form: one persistent launch advances every box of an ensemble by
// one substep.  The host gives every workgroup its own list of tile-chunks
// (items wg_first[L] .. wg_first[L + 1] - 1), where L = remap(blockIdx) numbers
// the workgroups of one XCD contiguously, so that the host can hand one XCD
// neighbouring tiles of the same boxes and they share its L2.  Per-box
// geometry, pointers, coefficients and time step come from device memory, so
// a captured graph never needs re-capture when they change.  Per point the
// arithmetic is the single-box kernel's.
template <typename T, typename TW, int TX, int TY, int S, int PD, bool LD, bool NT, int VS>
__global__ __launch_bounds__(TX* TY)
void substep55_batch(const BatchBox<T, TW>* __restrict__ boxes,
                     const BatchItem* __restrict__ items, const int* __restrict__ wg_first,
                     int parity, TW alpha, TW beta) {
    using Sh = SweepShape<T, TX, TY, LD>;
    __shared__ T lds[2 * 4 * Sh::FS];
    const int G = gridDim.x;
    int b = blockIdx.x;
    if ((G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
    const int last = wg_first[b + 1];
    for (int it = wg_first[b]; it < last; ++it) {
        const BatchItem wi = items[it];
        const BatchBox<T, TW>* bx = boxes + wi.box;
        const Geom g = bx->g;
        const Coef<T> cf = bx->cf;
        const Fields4<T> in = bx->st[parity], out = bx->st[parity ^ 1];
        const Fields4<TW> w = bx->w;
        const RKCoef<TW> rk{alpha, beta, bx->dt};
        sweep_tile<T, TW, TX, TY, S, PD, LD, NT, VS>(g, in, out, w, nullptr, cf, rk, wi.x0, wi.y0,
                                             wi.zb, wi.ze, lds, (lds_t<T>)lds);
        __syncthreads();  // the next item's first LDS write must follow every read
    }
}

// Launch helpers: the substep index S is a template argument of every kernel.
template <template <int> class K, typename... A>
hipError_t launch_s(int s, dim3 grid, dim3 block, hipStream_t st, A... args) {
    switch (s) {
    case 1: hipLaunchKernelGGL(K<1>::fn, grid, block, 0, st, args...); break;
    case 2: hipLaunchKernelGGL(K<2>::fn, grid, block, 0, st, args...); break;
    default: hipLaunchKernelGGL(K<3>::fn, grid, block, 0, st, args...); break;
    }
    return hipGetLastError();
}

template <typename T, typename TW, int TX, int TY, int PD, bool LD, bool NT, int VS, bool FRC>
struct K55 {
    template <int S>
    struct at {
        static constexpr auto fn = substep55_sweep<T, TW, TX, TY, S, PD, LD, NT, VS, FRC>;
    };
};
template <typename T, typename TW, int TX, int TY, int PD, bool LD, bool NT, int VS, bool FRC>
struct KRed {
    static constexpr auto fn = substep55_sweep_red<T, TW, TX, TY, PD, LD, NT, VS, FRC>;
};
template <typename T, typename TW, int TX, int TY, int PD, bool LD, bool NT, bool FRC>
struct K19 {
    template <int S>
    struct at {
        static constexpr auto fn = substep19_pass1<T, TW, TX, TY, S, PD, LD, NT, FRC>;
    };
};
template <typename T, typename TW, int TX, int TY, int PD, bool LD, bool NT, int VS>
struct KBatch {
    template <int S>
    struct at {
        static constexpr auto fn = substep55_batch<T, TW, TX, TY, S, PD, LD, NT, VS>;
    };
};
template <typename T, typename TW, bool FRC>
struct KDirect {
    template <int S>
    struct at {
        static constexpr auto fn = substep55_direct<T, TW, S, FRC>;
    };
};

// VS = 1: one array per field; VS = 4: array of structures (register-loader
// z-sweep shapes only).
template <typename T, typename TW, int VS>
hipError_t launch_substep55_vs(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                               const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                               int zchunk, double* partials, int part_cap, int* nparts,
                               const ForceArgs<T>* frc, hipStream_t st) {
    if (nparts) *nparts = 0;
    if (g.vs != VS) return hipErrorInvalidValue;
    const ForceArgs<T> fa = frc ? *frc : ForceArgs<T>{nullptr, nullptr};
    auto go = [&](auto force) -> hipError_t {
        constexpr bool FRC = decltype(force)::value;
        return with_tile(tile, hipErrorInvalidValue, [&](auto I) -> hipError_t {
            constexpr TileCfg k = kTiles[decltype(I)::value];
            if constexpr (VS != 1 && (k.tx == 0 || k.ld)) {
                return hipErrorInvalidValue;
            } else if constexpr (k.tx == 0) {
                const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4),
                                (unsigned)g.nz);
                return launch_s<KDirect<T, TW, FRC>::template at>(s, grid, dim3(256), st, g, in,
                                                                  out, w, c, rk, fa);
            } else {
                using K = K55<T, TW, k.tx, k.ty, k.pd, k.ld, k.nt, VS, FRC>;
                using KR = KRed<T, TW, k.tx, k.ty, k.pd, k.ld, k.nt, VS, FRC>;
                const int res = resident_blocks<K::template at<2>::fn>(k.tx * k.ty);
                const SweepGrid sg = sweep_grid(g, k.tx, k.ty, zchunk, res);
                // fuse only where the extra accumulators cost no occupancy
                static const bool fuse_ok = [] {
                    int a = 0, b = 0;
                    const int blk = k.tx * k.ty;
                    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, KR::fn, blk, 0) !=
                            hipSuccess ||
                        hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &b, K::template at<3>::fn, blk, 0) != hipSuccess)
                        return false;
                    return a >= b && a > 0;
                }();
                if (s == 3 && partials && nparts && fuse_ok && sg.blocks <= part_cap) {
                    hipLaunchKernelGGL(KR::fn, dim3(sg.blocks), dim3(k.tx * k.ty), 0, st, g, in,
                                       out, w, c, rk, sg, partials, fa);
                    *nparts = sg.blocks;
                    return hipGetLastError();
                }
                return launch_s<K::template at>(s, dim3(sg.blocks), dim3(k.tx * k.ty), st, g, in,
                                                out, w, c, rk, sg, fa);
            }
        });
    };
    return frc ? go(std::true_type{}) : go(std::false_type{});
}

}  // namespace

template <typename T, typename TW>
hipError_t launch_substep55(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                            const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                            double* partials, int part_cap, int* nparts,
                            const ForceArgs<T>* frc, hipStream_t st) {
    return launch_substep55_vs<T, TW, 1>(g, in, out, w, c, rk, s, tile, zchunk, partials,
                                         part_cap, nparts, frc, st);
}

template <typename T, typename TW>
hipError_t launch_substep55_aos(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                                const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                                int zchunk, double* partials, int part_cap, int* nparts,
                                const ForceArgs<T>* frc, hipStream_t st) {
    return launch_substep55_vs<T, TW, 4>(g, in, out, w, c, rk, s, tile, zchunk, partials,
                                         part_cap, nparts, frc, st);
}

// Pass 1 of the 19-point method in a z-sweep shape (tile >= 1).
template <typename T, typename TW>
hipError_t launch_pass19a_sweep(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                                T* dv, const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                                int zchunk, const ForceArgs<T>* frc, hipStream_t st) {
    const ForceArgs<T> fa = frc ? *frc : ForceArgs<T>{nullptr, nullptr};
    auto go = [&](auto force) -> hipError_t {
        constexpr bool FRC = decltype(force)::value;
        return with_tile(tile, hipErrorInvalidValue, [&](auto I) -> hipError_t {
            constexpr TileCfg k = kTiles[decltype(I)::value];
            if constexpr (k.tx == 0) {
                return hipErrorInvalidValue;
            } else {
                using K = K19<T, TW, k.tx, k.ty, k.pd, k.ld, k.nt, FRC>;
                const int res = resident_blocks<K::template at<2>::fn>(k.tx * k.ty);
                const SweepGrid sg = sweep_grid(g, k.tx, k.ty, zchunk, res);
                return launch_s<K::template at>(s, dim3(sg.blocks), dim3(k.tx * k.ty), st, g, in,
                                                out, w, dv, c, rk, sg, fa);
            }
        });
    };
    return frc ? go(std::true_type{}) : go(std::false_type{});
}

namespace {

template <typename T, typename TW, int VS>
hipError_t launch_batch55_vs(const BatchBox<T, TW>* boxes, const BatchItem* items,
                             const int* wg_first, int grid, int parity, int s, int tile, TW alpha,
                             TW beta, hipStream_t st) {
    return with_tile(tile, hipErrorInvalidValue, [&](auto I) -> hipError_t {
        constexpr TileCfg k = kTiles[decltype(I)::value];
        if constexpr (k.tx == 0 || (VS != 1 && k.ld)) {
            return hipErrorInvalidValue;
        } else {
            return launch_s<KBatch<T, TW, k.tx, k.ty, k.pd, k.ld, k.nt, VS>::template at>(
                s, dim3(grid), dim3(k.tx * k.ty), st, boxes, items, wg_first, parity, alpha, beta);
        }
    });
}

template <typename T, typename TW, int VS>
int batch55_blocks_per_cu_vs(int tile) {
    return with_tile(tile, 1, [&](auto I) -> int {
        constexpr TileCfg k = kTiles[decltype(I)::value];
        if constexpr (k.tx == 0 || (VS != 1 && k.ld)) {
            return 1;
        } else {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, substep55_batch<T, TW, k.tx, k.ty, 2, k.pd, k.ld, k.nt, VS>, k.tx * k.ty,
                    0) != hipSuccess)
                return 1;
            return n > 0 ? n : 1;
        }
    });
}

}  // namespace

template <typename T, typename TW>
hipError_t launch_batch55(const BatchBox<T, TW>* boxes, const BatchItem* items,
                          const int* wg_first, int grid, int parity, int s, int tile, TW alpha,
                          TW beta, hipStream_t st) {
    return launch_batch55_vs<T, TW, 1>(boxes, items, wg_first, grid, parity, s, tile, alpha,
                                       beta, st);
}

template <typename T, typename TW>
hipError_t launch_batch55_aos(const BatchBox<T, TW>* boxes, const BatchItem* items,
                              const int* wg_first, int grid, int parity, int s, int tile,
                              TW alpha, TW beta, hipStream_t st) {
    return launch_batch55_vs<T, TW, 4>(boxes, items, wg_first, grid, parity, s, tile, alpha,
                                       beta, st);
}

template <typename T, typename TW>
int batch55_blocks_per_cu(int tile) {
    return batch55_blocks_per_cu_vs<T, TW, 1>(tile);
}

template <typename T, typename TW>
int batch55_blocks_per_cu_aos(int tile) {
    return batch55_blocks_per_cu_vs<T, TW, 4>(tile);
}

}  // namespace fd6
