// FP64 diagnostics of caller-owned device fields without any allocation:
// fd6_reduce_fields_static (declared in include/fd6.h) runs the kernels of
// fd6_reduce_device over four compact arrays, with the per-block partials in
// a file-scope device array instead of a box workspace.
#include <cmath>
#include <mutex>

#include "../../include/fd6.h"
#include "fd6_internal.hpp"

using namespace fd6;

// Partials of the two-level reduction: one slot group per block of the first
// level (kReduceBlocks x kReduceSlots doubles, 64 KiB).  Every device the
// library runs on holds its own copy until the process ends.  Each call
// writes every slot it reads, so nothing has to start at zero.
constexpr int kScratchDoubles = kReduceBlocks * kReduceSlots;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of `scratch` on each device.  In host code the array's name
// is only a host-side stand-in, so kernels receive this address instead.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Looks the address up once per device, with that device current.
int scratch_on_current_device(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FD6_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FD6_EHIP;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return FD6_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename T>
int reduce_compact(int nx, int ny, int nz, const void* const f[4], double dV, hipStream_t st,
                   double* d_out5) {
    double* part = nullptr;
    int rc = scratch_on_current_device(&part);
    if (rc) return rc;
    // compact [z][y][x] arrays: rows of nx points, no ghost zone
    Geom g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.px = nx;
    g.plane = (long long)nx * ny;
    g.origin = 0;
    g.vs = 1;
    Fields4<T> fl;
    for (int q = 0; q < 4; ++q) fl.f[q] = static_cast<T*>(const_cast<void*>(f[q]));
    return launch_reduce<T>(g, fl, part, d_out5, dV, st) == hipSuccess ? FD6_OK : FD6_EHIP;
}

}  // namespace

extern "C" int fd6_reduce_fields_static(int32_t nx, int32_t ny, int32_t nz, int32_t precision,
                                        const void* lnrho, const void* ux, const void* uy,
                                        const void* uz, double dx, double dy, double dz,
                                        void* stream, double* d_out5) {
    if (!lnrho || !ux || !uy || !uz || !d_out5) return FD6_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096) return FD6_EINVAL;
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz)) return FD6_EINVAL;
    const void* f[4] = {lnrho, ux, uy, uz};
    const double dV = dx * dy * dz;
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (precision) {
    case FD6_FP64: return reduce_compact<double>(nx, ny, nz, f, dV, st, d_out5);
    case FD6_FP32:
    case FD6_FP32_ACC64: return reduce_compact<float>(nx, ny, nz, f, dV, st, d_out5);
    default: return FD6_EINVAL;
    }
}
