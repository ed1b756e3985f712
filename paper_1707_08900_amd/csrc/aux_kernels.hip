// Auxiliary kernels: periodic ghost fill, FP64 import/export of the state,
// and the deterministic FP64 global reductions.
#include "exp_fp64.hpp"
#include "fd6_internal.hpp"

namespace fd6 {
namespace {

__device__ inline int wrap_index(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Periodic boundary condition of Sec. 4 (the boundary step of Algorithms
// 1-3): every ghost cell (i, j, k) in [-3, n+3)^3 \ [0, n)^3 takes
// the value of its periodic image (i mod nx, j mod ny, k mod nz).  The image
// is always an interior cell (n >= 6 > R), so all ghost cells are independent.
// The ghost cells are enumerated region by region so that consecutive threads
// touch consecutive x wherever a region has a full row:
//   Z: 6 ghost planes, full (nx+6)(ny+6) rows
//   Y: interior planes, 6 ghost rows each of nx+6 cells
//   X: interior rows, the 3 + 3 cells at the row ends
template <typename T>
__global__ __launch_bounds__(256) void ghost_fill_kernel(Geom g, Fields4<T> f, int nfields,
                                                         long long nz_cells, long long ny_cells,
                                                         long long total) {
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int wx = g.nx + 2 * kR;
    for (long long e = e0; e < total; e += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        if (e < nz_cells) {
            long long r = e / wx;
            i = (int)(e - r * wx) - kR;
            int row = (int)(r % (g.ny + 2 * kR));
            int pl = (int)(r / (g.ny + 2 * kR));
            j = row - kR;
            k = pl < kR ? pl - kR : g.nz + (pl - kR);
        } else if (e < nz_cells + ny_cells) {
            long long e1 = e - nz_cells;
            long long r = e1 / wx;
            i = (int)(e1 - r * wx) - kR;
            int row = (int)(r % (2 * kR));
            k = (int)(r / (2 * kR));
            j = row < kR ? row - kR : g.ny + (row - kR);
        } else {
            long long e2 = e - nz_cells - ny_cells;
            long long r = e2 / (2 * kR);
            int c = (int)(e2 - r * (2 * kR));
            i = c < kR ? c - kR : g.nx + (c - kR);
            j = (int)(r % g.ny);
            k = (int)(r / g.ny);
        }
        const long long dst = g.origin + (long long)k * g.plane + (long long)j * g.px + i;
        const long long src = g.origin + (long long)wrap_index(k, g.nz) * g.plane +
                              (long long)wrap_index(j, g.ny) * g.px + wrap_index(i, g.nx);
        for (int q = 0; q < nfields; ++q) f.f[q][dst] = f.f[q][src];
    }
}

// Compact FP64 planes [zbeg, zbeg + nplanes) -> interior of a state field,
// rounding to T (round to nearest even for float).
template <typename T>
__global__ __launch_bounds__(256) void import_kernel(Geom g, const double* __restrict__ src,
                                                     T* __restrict__ dst, long long zbeg,
                                                     long long count) {
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long e = e0; e < count; e += (long long)gridDim.x * blockDim.x) {
        long long r = e / g.nx;
        int i = (int)(e - r * g.nx);
        int j = (int)(r % g.ny);
        long long k = zbeg + r / g.ny;
        dst[(g.origin + k * g.plane + (long long)j * g.px + i) * g.vs] = (T)src[e];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void export_kernel(Geom g, const T* __restrict__ src,
                                                     double* __restrict__ dst, long long zbeg,
                                                     long long count) {
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long e = e0; e < count; e += (long long)gridDim.x * blockDim.x) {
        long long r = e / g.nx;
        int i = (int)(e - r * g.nx);
        int j = (int)(r % g.ny);
        long long k = zbeg + r / g.ny;
        dst[e] = (double)src[(g.origin + k * g.plane + (long long)j * g.px + i) * g.vs];
    }
}

template <typename TW>
__global__ __launch_bounds__(256) void export_w_kernel(Geom g, const TW* __restrict__ src,
                                                       double* __restrict__ dst, long long count) {
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long e = e0; e < count; e += (long long)gridDim.x * blockDim.x) {
        long long r = e / g.nx;
        int i = (int)(e - r * g.nx);
        int j = (int)(r % g.ny);
        long long k = r / g.ny;
        dst[e] = (double)src[(k * g.wplane + (long long)j * g.wpx + i) * g.vs];
    }
}

template <typename TW>
__global__ __launch_bounds__(256) void zero_w_kernel(Fields4<TW> w, long long n, int vs) {
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long e = e0; e < n; e += (long long)gridDim.x * blockDim.x)
        for (int q = 0; q < 4; ++q) w.f[q][e * vs] = TW(0);
}

// ---------------------------------------------------------------------------
// Reductions.  Each block accumulates a fixed, grid-size-determined subset of
// the interior points in FP64, reduces it with a fixed tree in LDS and writes
// one partial; a single block then combines the partials in a fixed tree.
// The result is therefore bitwise reproducible run to run.
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

struct RedAcc {
    double mass, ke, slr, umax, bad;
};

__device__ inline void red_combine(RedAcc& a, const RedAcc& b) {
    a.mass += b.mass;
    a.ke += b.ke;
    a.slr += b.slr;
    a.umax = fmax(a.umax, b.umax);
    a.bad += b.bad;
}

__device__ inline void block_reduce_store(RedAcc acc, double* out) {
    __shared__ RedAcc sh[kRedThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            RedAcc a = sh[threadIdx.x];
            red_combine(a, sh[threadIdx.x + s]);
            sh[threadIdx.x] = a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0].mass;
        out[1] = sh[0].ke;
        out[2] = sh[0].slr;
        out[3] = sh[0].umax;
        out[4] = sh[0].bad;
    }
}

// Each block takes whole x rows (row r = blockIdx.x, blockIdx.x + gridDim.x,
// ...), threads stride along the row: coalesced loads, one division per row.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void reduce_partials_kernel(Geom g, Fields4<T> f,
                                                                      double* partials,
                                                                      long long count) {
    (void)count;
    RedAcc acc{0.0, 0.0, 0.0, 0.0, 0.0};
    const int rows = g.ny * g.nz;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int k = r / g.ny, j = r - k * g.ny;
        const long long base = g.origin + (long long)k * g.plane + (long long)j * g.px;
        for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
            const long long c = (base + i) * g.vs;
            const double lr = (double)f.f[0][c], ux = (double)f.f[1][c], uy = (double)f.f[2][c],
                         uz = (double)f.f[3][c];
            // the per-point quantities of the fused diagnostics (red_point)
            const double rho = exp_fp64(lr);
            const double u2 = ux * ux + uy * uy + uz * uz;
            acc.mass += rho;
            acc.ke += 0.5 * (rho * u2);
            acc.slr += lr;
            const double um = sqrt(u2);
            acc.umax = um > acc.umax ? um : acc.umax;
            const bool finite = isfinite(lr) && isfinite(ux) && isfinite(uy) && isfinite(uz);
            acc.bad += finite ? 0.0 : 1.0;
        }
    }
    block_reduce_store(acc, partials + (size_t)blockIdx.x * kReduceSlots);
}

__global__ __launch_bounds__(kRedThreads) void reduce_final_kernel(const double* partials,
                                                                   int nparts, double* result,
                                                                   double dV) {
    RedAcc acc{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        const double* p = partials + (size_t)b * kReduceSlots;
        RedAcc o{p[0], p[1], p[2], p[3], p[4]};
        red_combine(acc, o);
    }
    __shared__ double out[kReduceSlots];
    block_reduce_store(acc, out);
    if (threadIdx.x == 0) {
        // with a non-finite value anywhere, mass and kinetic energy are
        // reported as NaN (the clamped exponential would otherwise turn a
        // NaN lnrho into a large finite term)
        const bool bad = out[4] > 0.0;
        result[0] = bad ? __builtin_nan("") : out[0] * dV;
        result[1] = bad ? __builtin_nan("") : out[1] * dV;
        result[2] = out[2];
        result[3] = out[3];
        result[4] = out[4];
    }
}

unsigned grid_for(long long n, int threads, int maxblocks = 65536) {
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > maxblocks) b = maxblocks;
    return (unsigned)b;
}

}  // namespace

template <typename T>
hipError_t launch_ghost_fill(const Geom& g, Fields4<T> f, int nfields, hipStream_t s) {
    if (g.vs != 1) return hipErrorInvalidValue;  // only the sweep shapes take other layouts
    const long long wx = g.nx + 2 * kR, wy = g.ny + 2 * kR;
    const long long nzc = 2LL * kR * wy * wx;
    const long long nyc = (long long)g.nz * 2 * kR * wx;
    const long long nxc = (long long)g.nz * g.ny * 2 * kR;
    const long long total = nzc + nyc + nxc;
    hipLaunchKernelGGL(ghost_fill_kernel<T>, dim3(grid_for(total, 256)), dim3(256), 0, s, g, f,
                       nfields, nzc, nyc, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_import(const Geom& g, const double* src, T* dst, long long zbeg, int nplanes,
                         hipStream_t s) {
    const long long n = (long long)g.nx * g.ny * nplanes;
    hipLaunchKernelGGL(import_kernel<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, g, src, dst,
                       zbeg, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const Geom& g, const T* src, double* dst, long long zbeg, int nplanes,
                         hipStream_t s) {
    const long long n = (long long)g.nx * g.ny * nplanes;
    hipLaunchKernelGGL(export_kernel<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, g, src, dst,
                       zbeg, n);
    return hipGetLastError();
}

template <typename TW>
hipError_t launch_export_w(const Geom& g, const TW* src, double* dst, int z0, int nplanes,
                           hipStream_t s) {
    // planes [z0, z0 + nplanes) of the compact register, to dst[0 ..)
    const long long n = (long long)g.nx * g.ny * nplanes;
    hipLaunchKernelGGL(export_w_kernel<TW>, dim3(grid_for(n, 256)), dim3(256), 0, s, g,
                       src + (long long)z0 * g.wplane * g.vs, dst, n);
    return hipGetLastError();
}

template <typename TW>
hipError_t launch_zero_w(const Geom& g, Fields4<TW> w, hipStream_t s) {
    hipLaunchKernelGGL(zero_w_kernel<TW>, dim3(grid_for(g.wfelems, 256)), dim3(256), 0, s, w,
                       g.wfelems, g.vs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const Geom& g, Fields4<T> f, double* partials, double* result, double dV,
                         hipStream_t s) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(reduce_partials_kernel<T>, dim3(kReduceBlocks), dim3(kRedThreads), 0, s, g,
                       f, partials, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kRedThreads), 0, s, partials,
                       kReduceBlocks, result, dV);
    return hipGetLastError();
}

namespace {
// Writes the force descriptor and the per-plane factors of eq. (forcing).
template <typename T>
__global__ __launch_bounds__(256) void force_table_kernel(int nz, ForceDev<T>* dev, T* tab,
                                                          double kx, double ky, double kz,
                                                          double phase, double dx, double dy,
                                                          double dz, double a0, double a1,
                                                          double a2) {
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        double sn, cs;
        sincos(kz * (k * dz) + phase, &sn, &cs);
        tab[2 * k] = T(cs);
        tab[2 * k + 1] = T(sn);
    }
    if (threadIdx.x == 0) {
        ForceDev<T> d;
        d.kx = kx;
        d.ky = ky;
        d.kz = kz;
        d.phase = phase;
        d.dx = dx;
        d.dy = dy;
        d.dz = dz;
        d.a[0] = T(a0);
        d.a[1] = T(a1);
        d.a[2] = T(a2);
        *dev = d;
    }
}
}  // namespace

template <typename T>
hipError_t launch_force_table(const Geom& g, ForceDev<T>* dev, T* tab, const double k[3],
                              double phase, const double h[3], const double a[3],
                              hipStream_t s) {
    hipLaunchKernelGGL(force_table_kernel<T>, dim3(1), dim3(256), 0, s, g.nz, dev, tab, k[0], k[1],
                       k[2], phase, h[0], h[1], h[2], a[0], a[1], a[2]);
    return hipGetLastError();
}
template hipError_t launch_force_table<float>(const Geom&, ForceDev<float>*, float*,
                                              const double*, double, const double*, const double*,
                                              hipStream_t);
template hipError_t launch_force_table<double>(const Geom&, ForceDev<double>*, double*,
                                               const double*, double, const double*,
                                               const double*, hipStream_t);

hipError_t launch_reduce_final(const double* partials, int nparts, double* result, double dV,
                               hipStream_t s) {
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, nparts,
                       result, dV);
    return hipGetLastError();
}

#define FD6_INST_T(T)                                                                        \
    template hipError_t launch_ghost_fill<T>(const Geom&, Fields4<T>, int, hipStream_t);    \
    template hipError_t launch_import<T>(const Geom&, const double*, T*, long long, int,    \
                                         hipStream_t);                                     \
    template hipError_t launch_export<T>(const Geom&, const T*, double*, long long, int,    \
                                         hipStream_t);                                     \
    template hipError_t launch_export_w<T>(const Geom&, const T*, double*, int, int,        \
                                           hipStream_t);                                \
    template hipError_t launch_zero_w<T>(const Geom&, Fields4<T>, hipStream_t);            \
    template hipError_t launch_reduce<T>(const Geom&, Fields4<T>, double*, double*, double, \
                                         hipStream_t);
FD6_INST_T(float)
FD6_INST_T(double)

}  // namespace fd6
