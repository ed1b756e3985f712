// Building blocks shared by the z-sweep kernels of the 55-point and the
// 19-point methods: raw buffer access, tile geometry, plane addressing.
#pragma once

#include <cstdlib>
#include <type_traits>

#include "exp_fp64.hpp"
#include "fd6_internal.hpp"

namespace fd6 {
namespace {

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
// Cache policy of an access (the instruction's cache-policy field): 0 keeps
// the default, kNonTemporal marks a stream whose lines are not reused before
// eviction (the new state and the RK register: each is touched once per
// substep).
constexpr int kNonTemporal = 2;

template <int CP = 0>
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP));
}
template <int CP = 0>
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP));
}
template <int CP = 0>
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, CP);
}

// One grid point of the array-of-structures layout: the four fields in 16
// (FP32) or 32 (FP64) consecutive bytes, moved with 16-byte accesses.
// (Whole vectors are bit-cast: with this compiler a bit cast of a single
// element of the loaded vector shrank the access to one dword and gave wrong
// values for the other elements.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int CP = 0>
__device__ __forceinline__ void bload_point(float (&v)[4], __amdgpu_buffer_rsrc_t r,
                                            unsigned off) {
    const f32x4 a = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP));
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = a[i];
}
template <int CP = 0>
__device__ __forceinline__ void bload_point(double (&v)[4], __amdgpu_buffer_rsrc_t r,
                                            unsigned off) {
    // a dropped point (off = kDropOffset) stays beyond the range at off + 16
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, CP);
    v[0] = __builtin_bit_cast(double, u32x2{a[0], a[1]});
    v[1] = __builtin_bit_cast(double, u32x2{a[2], a[3]});
    v[2] = __builtin_bit_cast(double, u32x2{b[0], b[1]});
    v[3] = __builtin_bit_cast(double, u32x2{b[2], b[3]});
}
template <int CP = 0>
__device__ __forceinline__ void bstore_point(const float (&v)[4], __amdgpu_buffer_rsrc_t r,
                                             unsigned off) {
    const f32x4 a{v[0], v[1], v[2], v[3]};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, a), r, off, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bstore_point(const double (&v)[4], __amdgpu_buffer_rsrc_t r,
                                             unsigned off) {
    const u32x2 p0 = __builtin_bit_cast(u32x2, v[0]), p1 = __builtin_bit_cast(u32x2, v[1]);
    const u32x2 p2 = __builtin_bit_cast(u32x2, v[2]), p3 = __builtin_bit_cast(u32x2, v[3]);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{p0[0], p0[1], p1[0], p1[1]}, r, off, 0, CP);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{p2[0], p2[1], p3[0], p3[1]}, r, off + 16u, 0, CP);
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

// Element index of the ghost corner (-3, -3) of interior plane p mod nz.
__device__ __forceinline__ long long plane_corner(const Geom& g, int p) {
    const int pz = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
    return g.origin + (long long)pz * g.plane - kR * g.px - kR;
}

// LDS pointer in the local address space (required by the LDS copy).
template <typename T>
using lds_t = __attribute__((address_space(3))) T*;

// Workgroup-to-XCD remapping of tiles (FD6_XCD_REMAP=0 disables it).
inline int xcd_remap() {
    static const int v = [] {
        const char* e = getenv("FD6_XCD_REMAP");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    return v;
}

// Per-thread addressing of one tile: byte offsets, relative to the ghost
// corner (-3, -3) of a plane, of the cells this thread loads (beyond the
// plane's range the load returns 0; such cells are only read by threads whose
// outputs are dropped), LDS slots of its halo loads, and its output offsets.
template <typename T, int TX, int TY, bool LD = false>
struct SweepCtx {
    using Sh = SweepShape<T, TX, TY, LD>;
    unsigned doff[Sh::ND];  // LD: byte offset of each lane's dword of the plane tile
    unsigned goff_int;
    unsigned goff_h[Sh::NH];
    int loff_h[Sh::NH];   // LDS slot of each halo load (dummy cell if unused)
    unsigned lane_o;      // byte offset of the output point in a state plane
    unsigned lane_w;      // byte offset of the output point in a w plane
    unsigned plane_bytes, wplane_bytes;
};

// Addressing of the tile with corner (x0, y0).  The periodic boundary
// condition (Sec. 4) is resolved here: a halo cell outside the interior reads
// its periodic image, so the sweep kernels neither read nor need the ghost
// zone.  Cells beyond x < nx + 3, y < ny + 3 never feed a stored point and are
// dropped.
// VS: values per point in memory (1, or 4 for the array-of-structures
// layout); all byte offsets and plane sizes scale with it.  WRAP_ALL: every
// cell at any offset takes its periodic image and none is dropped (the
// extended tile of the substep-1+2 fusion, whose cells may lie a whole tile
// beyond the box).
template <typename T, typename TW, int TX, int TY, bool LD, int VS = 1, bool WRAP_ALL = false>
__device__ __forceinline__ void sweep_ctx_init(SweepCtx<T, TX, TY, LD>& X, const Geom& g, int x0,
                                               int y0) {
    using Sh = SweepShape<T, TX, TY, LD>;
    static_assert(VS == 1 || !LD, "the LDS-copy loader reads one array per field");
    constexpr int PT = VS * (int)sizeof(T), PW = VS * (int)sizeof(TW);  // bytes per point
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    X.plane_bytes = (unsigned)(g.plane * (long long)PT);
    X.wplane_bytes = (unsigned)(g.wplane * (long long)PW);
    auto wrapped_off = [&](int gx, int gy) -> unsigned {  // gx, gy in [-3, ...)
        if constexpr (WRAP_ALL) {
            const int ix = ((gx % g.nx) + g.nx) % g.nx, iy = ((gy % g.ny) + g.ny) % g.ny;
            return (unsigned)(((iy + kR) * g.px + (ix + kR)) * PT);
        }
        if (gx >= g.nx + kR || gy >= g.ny + kR) return kDropOffset;
        const int ix = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
        const int iy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
        return (unsigned)(((iy + kR) * g.px + (ix + kR)) * PT);
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
    for (int h = 0; h < Sh::NH; ++h) {
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
    const int xo = x0 + tx, yo = y0 + ty;
    const bool store = xo < g.nx && yo < g.ny;
    X.lane_o = store ? (unsigned)(((yo + kR) * g.px + (xo + kR)) * PT) : kDropOffset;
    X.lane_w = store ? (unsigned)((yo * g.wpx + xo) * PW) : kDropOffset;
}

// Workgroup index -> (tile x, tile y, z chunk).  Each XCD receives every 8th
// workgroup; with remap the grid is renumbered so that one XCD takes a
// contiguous range of tiles instead.  Within a z chunk the tiles are ordered
// in column blocks gx tiles wide (x fastest inside a block, then y, then the
// next block), so the tiles an XCD holds at once cover a near-square region
// and the halo rows and columns they read from outside it (from HBM rather
// than from that XCD's L2) are few.  gx >= ntx is plain row order.
struct SweepGrid {
    int ntx, nty, zlen, blocks;
    int gx;     // column-block width in tiles
    int remap;  // 1: contiguous tile ranges per XCD
};

// Column-block width that minimises the halo fraction of the region one XCD
// holds at once (per_xcd tiles of tx x ty; a region spanning a whole
// periodic axis reads no halo along it).  FD6_SWEEP_GX > 0 overrides it.
inline int sweep_block_width(int ntx, int nty, int tx, int ty, int per_xcd) {
    static const int forced = [] {
        const char* e = getenv("FD6_SWEEP_GX");
        return e ? atoi(e) : 0;
    }();
    if (forced > 0) return forced < ntx ? forced : ntx;
    int best = ntx;
    double best_cost = 1e30;
    for (int gx = ntx; gx >= 1; --gx) {
        const int rows = (per_xcd + gx - 1) / gx;
        const double xh = gx >= ntx ? 0.0 : 2.0 * kR / (gx * tx);
        const double yh = rows >= nty ? 0.0 : 2.0 * kR / ((double)rows * ty);
        if (xh + yh < best_cost - 1e-12) best_cost = xh + yh, best = gx;
    }
    return best;
}

// zchunk > 0 fixes the chunk length (planes); 0 chooses it.  resident: how
// many workgroups of the kernel the device holds at once.  The automatic
// choice minimises (rounds of resident workgroups) x (planes swept per chunk,
// including the 6 re-read planes), i.e. it prefers long chunks unless they
// leave compute units idle.
inline SweepGrid sweep_grid(const Geom& g, int tx, int ty, int zchunk, int resident) {
    SweepGrid s;
    s.ntx = (g.nx + tx - 1) / tx;
    s.nty = (g.ny + ty - 1) / ty;
    const long long tiles = (long long)s.ntx * s.nty;
    int nch = 1;
    if (zchunk > 0) {
        nch = (g.nz + zchunk - 1) / zchunk;
    } else {
        const long long res = resident > 0 ? resident : 1;
        long long best = -1;
        for (int c = 1; c <= (g.nz + 7) / 8; ++c) {
            const long long len = (g.nz + c - 1) / c;
            const long long cost = ((tiles * c + res - 1) / res) * (len + 2 * kR);
            if (best < 0 || cost < best) best = cost, nch = c;
        }
    }
    s.zlen = (g.nz + nch - 1) / nch;
    nch = (g.nz + s.zlen - 1) / s.zlen;
    s.blocks = (int)(tiles * nch);
    s.remap = xcd_remap();
    s.gx = s.remap ? sweep_block_width(s.ntx, s.nty, tx, ty, resident > 8 ? resident / 8 : 1)
                   : s.ntx;
    return s;
}

// Workgroups of Kernel (block threads) the current device holds at once
// (the per-CU occupancy is queried once per kernel).
template <auto Kernel>
int resident_blocks(int block) {
    static const int per_cu = [&] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, Kernel, block, 0) != hipSuccess)
            n = 1;
        return n > 0 ? n : 1;
    }();
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    return per_cu * cus;
}

struct TileXY {
    int tx, ty, zb, ze;
};

__device__ __forceinline__ TileXY sweep_tile_of(const Geom& g, int TX, int TY,
                                                const SweepGrid& m) {
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if (m.remap && (nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int per = m.ntx * m.nty;
    const int ch = b / per;
    int l = b - ch * per;                     // tile within the chunk
    const int blk = l / (m.gx * m.nty);       // column block
    const int bx0 = blk * m.gx;
    const int bw = min(m.gx, m.ntx - bx0);    // the last block may be narrower
    l -= blk * m.gx * m.nty;
    const int tiy = l / bw;
    const int tix = bx0 + (l - tiy * bw);
    const int zb = ch * m.zlen;
    return TileXY{tix * TX, tiy * TY, zb, min(zb + m.zlen, g.nz)};
}

// FP64 diagnostics of one point of the new state (the quantities of the
// standalone reduction): per thread, red = {sum rho, sum rho |u|^2, sum
// lnrho, max |u|^2} and bad = points holding a non-finite value.  The caller
// skips points that are not outputs (branches, not selects, so the skipped
// steps and lanes cost no FP64 instructions).  The kinetic energy's factor
// 1/2 is applied once per workgroup (exact).  Non-finite values are found by
// class checks of the stored values; the mass and kinetic-energy terms of
// such a point are meaningless and the final combination reports them as
// NaN whenever bad > 0.
template <typename T>
__device__ __forceinline__ void red_point(double red[4], int& bad, T lr, T ux, T uy, T uz) {
    const bool finite = __builtin_isfinite(lr) && __builtin_isfinite(ux) &&
                        __builtin_isfinite(uy) && __builtin_isfinite(uz);
    bad += finite ? 0 : 1;
    const double l = (double)lr, a = (double)ux, b = (double)uy, c = (double)uz;
    const double rho = exp_fp64(l);
    const double u2 = a * a + b * b + c * c;
    red[0] += rho;
    red[1] += rho * u2;
    red[2] += l;
    red[3] = __builtin_fmax(red[3], u2);
}

// Combines the per-thread diagnostics of a workgroup in a fixed order (xor
// tree within each wave, then waves in order) and stores the partial:
// sums for slots 0-2 and 4, the maximum for slot 3.
template <int NW>
__device__ __forceinline__ void red_store_n(const double red[4], int bad, double* part) {
    double v[5] = {red[0], 0.5 * red[1], red[2], red[3], (double)bad};
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double o = __shfl_xor(v[i], off, 64);
            v[i] = i == 3 ? (o > v[i] ? o : v[i]) : v[i] + o;
        }
    }
    __shared__ double sw[NW][5];
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 5; ++i) sw[wv][i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < NW; ++k)
#pragma unroll
            for (int i = 0; i < 5; ++i)
                a[i] = i == 3 ? (sw[k][i] > a[i] ? sw[k][i] : a[i]) : a[i] + sw[k][i];
        double* p = part + (size_t)blockIdx.x * kReduceSlots;
        p[0] = a[0];
        p[1] = a[1];
        p[2] = a[2];
        p[3] = sqrt(a[3]);  // max |u| = sqrt(max |u|^2): sqrt is monotonic
        p[4] = a[4];
    }
}

// Kernel shapes of the z-sweep substeps.  Index 0 is the direct kernel (one
// thread per point, taps from the ghost zone); the others are (TX, TY) column
// tiles.  pd: how many planes ahead the register loader fetches (1, 2 or 4;
// 2 and 4 also load the RK3 register one step early); ld: the LDS-copy loader
// instead.
struct TileCfg {
    int tx, ty, pd;
    bool ld;
    bool nt;  // new state and RK register streamed past the caches
};
constexpr TileCfg kTiles[] = {
    {0, 0, 1, false, false},  {64, 4, 1, false, true},  {64, 8, 1, false, true},
    {128, 4, 1, false, true}, {32, 8, 1, false, true},  {64, 4, 2, false, true},
    {64, 8, 2, false, true},  {128, 4, 2, false, true}, {32, 8, 2, false, true},
    {64, 8, 1, true, true},   {64, 8, 4, false, true},  {64, 8, 1, false, false},
    {64, 8, 2, false, false}, {32, 8, 2, false, false}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// Calls f(std::integral_constant<int, tile>) so that f can use kTiles[tile]
// as template arguments; returns `bad` for an out-of-range tile.
template <int I = 0, typename R, typename F>
R with_tile(int tile, R bad, F&& f) {
    if constexpr (I < kNumTiles) {
        if (tile == I) return f(std::integral_constant<int, I>{});
        return with_tile<I + 1>(tile, bad, f);
    } else {
        return bad;
    }
}

}  // namespace
}  // namespace fd6
