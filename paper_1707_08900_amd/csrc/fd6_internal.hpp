// Internal definitions shared by the HIP kernels and the host runtime of the
// fd6 library (sixth-order finite-difference RK3 substep for isothermal
// compressible hydrodynamics, Pekkila et al. 2017).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fd6 {

constexpr int kR = 3;  // stencil radius: sixth order, n = 2R (Sec. 2.3)

// Storage geometry of one box.
//
// A state field is a ghosted array: interior (i, j, k), 0 <= i < nx, lives at
// element  origin + k * plane + j * px + i,  for -3 <= i < nx + 3 likewise.
// Rows are padded so that every row starts on a 128-byte boundary and the
// interior point i = 0 of every row is 128-byte aligned (the ghost cells
// i = -3..-1 sit at the end of the preceding 128-byte line).
//
// The RK3 register w has no ghost zone: (i, j, k) lives at
// k * wplane + j * wpx + i, rows 128-byte aligned.
struct Geom {
    int nx, ny, nz;
    int px;                // elements per state row
    long long plane;       // elements per state plane = px * (ny + 6)
    long long origin;      // element of interior (0, 0, 0)
    long long felems;      // elements per state field (multiple of 256 B)
    int wpx;               // elements per w row
    long long wplane;      // wpx * ny
    long long wfelems;     // elements per w field (multiple of 256 B)
    // Values per grid point in memory: 1 = one array per field; 4 = the four
    // fields of a point adjacent (array of structures).  Element indices above
    // count points; field q of point e is at f[q][e * vs], with f[q] = f[0] + q
    // when vs = 4 (the same holds for w).
    int vs = 1;
};

// Four state fields (lnrho, ux, uy, uz) and four w fields.
template <typename T>
struct Fields4 {
    T* f[4];
};

// RK3 substep constants (eq. 2N-RK_scheme): w <- alpha w + dt r,
// out <- in + beta w.
template <typename TW>
struct RKCoef {
    TW alpha, beta, dt;
};

// Finite-difference weights with the grid spacings folded in (Sec. 2.3).
//   d1[a][k-1]  = {45, -9, 1}[k-1] / (60 h_a)          first derivative
//   d2[a][k]    = {-490, 270, -27, 2}[k] / (180 h_a^2)  second derivative
//   mx[p][k-1]  = {270, -27, 2}[k-1] / (720 h_a h_b)    mixed, p = xy, xz, yz
// The fused kernel also uses combinations of these; the host precomputes
// them in FP64 and rounds once to the working precision.
template <typename T>
struct Coef {
    T d1[3][3];
    T d2[3][4];
    T mx[3][3];
    T nu, cs2;
    // Linear viscous part of the momentum equation for component i:
    //   L_i = lap u_i + (1/3) d_i div u
    //       = sum_a (1 + delta_ia / 3) D2_a u_i + (1/3) sum_{j != i} D_ij u_j
    // lw[i][a][k]: weight of the second-derivative tap k along axis a in L_i
    // (nu folded in), mw[p][k-1]: mixed weights / 3 (nu folded in).
    T lw[3][3][4];
    T mw[3][3];
    // 19-point method: nu-scaled plain second-derivative weights (nu lap u)
    // and nu / 3 in FP64 for the pass-2 factor dt (nu / 3).
    T lp[3][4];
    double nu3;
    // Scale factors for stencils written with their integer weights
    // (second derivative 2, -27, 270, -490; mixed 270, -27, 2):
    //   sg[a]  = nu / (180 h_a^2),  sg4[a] = (4/3) sg[a]
    //   kxy[i] = -490 (s_ix + s_iy), s_ia = (a == i ? sg4 : sg)[a]
    //   mu[p]  = nu / (3 * 720 h_a h_b), p = xy, xz, yz
    //   kp     = -490 (sg[x] + sg[y])  (centre weight of nu (D2x + D2y))
    T sg[3], sg4[3], kxy[3], mu[3], kp;
};

// External force of the momentum equation, one Fourier mode of eq. (forcing)
// (Sec. 6): f(x) = a cos(k.x + phase), a = N f_k, with grid point (i, j, k)
// at x = (i dx, j dy, k dz).  Lives in device memory so that a captured step
// reads the force of the current time step.  The sweep kernels form
// cos(k.x + phase) = cos(A) cos(B) - sin(A) sin(B) with A = kx x + ky y per
// column (once per tile) and B = kz z + phase per plane from tab:
// tab[2 k] = cos(kz k dz + phase), tab[2 k + 1] = sin(...), 0 <= k < nz.
template <typename T>
struct ForceDev {
    double kx, ky, kz, phase;
    double dx, dy, dz;
    T a[3];
};
template <typename T>
struct ForceArgs {
    const ForceDev<T>* dev;
    const T* tab;
};

// Host-side launchers (implemented in the .hip files).
template <typename T>
hipError_t launch_force_table(const Geom& g, ForceDev<T>* dev, T* tab, const double k[3],
                              double phase, const double h[3], const double a[3],
                              hipStream_t s);
template <typename T>
hipError_t launch_ghost_fill(const Geom& g, Fields4<T> f, int nfields, hipStream_t s);

template <typename T>
hipError_t launch_import(const Geom& g, const double* src, T* dst, long long zbeg, int nplanes,
                         hipStream_t s);
template <typename T>
hipError_t launch_export(const Geom& g, const T* src, double* dst, long long zbeg, int nplanes,
                         hipStream_t s);
template <typename TW>
hipError_t launch_export_w(const Geom& g, const TW* src, double* dst, int z0, int nplanes,
                           hipStream_t s);
template <typename TW>
hipError_t launch_zero_w(const Geom& g, Fields4<TW> w, hipStream_t s);

// 55-point fused right-hand side + RK3 update for substep s (1, 2, 3) with
// kernel shape `tile` and z-chunk length `zchunk` (0: chosen by the launcher).
// With partials != nullptr, substep 3 of a z-sweep shape whose grid has at
// most part_cap workgroups also writes one FP64 diagnostics partial per
// workgroup (kReduceSlots doubles each) and sets *nparts to their number;
// otherwise *nparts = 0 and the caller reduces separately.
// frc != nullptr adds the external force to the momentum right-hand side.
template <typename T, typename TW>
hipError_t launch_substep55(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                            const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                            double* partials, int part_cap, int* nparts,
                            const ForceArgs<T>* frc, hipStream_t st);
// The same substep for the array-of-structures layout (vs = 4): each loaded
// or stored point is one 16-byte (FP32) or two 16-byte (FP64) accesses
// instead of one access per field.  Register-loader z-sweep shapes only
// (substep55_aos_tile_ok).
template <typename T, typename TW>
hipError_t launch_substep55_aos(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                                const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                                int zchunk, double* partials, int part_cap, int* nparts,
                                const ForceArgs<T>* frc, hipStream_t st);
bool substep55_aos_tile_ok(int tile);
// Substeps 1 and 2 of one step in a single launch (FP32 state and register,
// either layout): in -> out after both substeps, w holding the substep-2
// register.  rk1, rk2: the two substeps' coefficients.
template <typename T, typename TW>
hipError_t launch_fused12(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                          const Coef<T>& c, const RKCoef<TW>& rk1, const RKCoef<TW>& rk2,
                          int zchunk, hipStream_t st);
// Whether a kernel shape reads the ghost zone of its input (the z-sweep
// shapes resolve the periodic images in their loader instead).
bool substep55_reads_ghosts(int tile);

// Batched ensemble: per-box descriptor (device resident) and one tile-chunk
// work item.
template <typename T, typename TW>
struct BatchBox {
    Geom g;
    Fields4<T> st[2];  // the two state sets; st[parity] is the substep input
    Fields4<TW> w;
    Coef<T> cf;
    TW dt;
};
struct BatchItem {
    int box, x0, y0, zb, ze;
};
// Workgroups of a batched launch: the persistent grid never exceeds this, so
// the per-workgroup list offsets fit a fixed slot in the workspace.
constexpr int kMaxBatchGrid = 65536;
// Tile extents of a z-sweep kernel shape (tile >= 1); -1 for other shapes.
int substep55_tile_dims(int tile, int* tx, int* ty);
template <typename T, typename TW>
hipError_t launch_batch55(const BatchBox<T, TW>* boxes, const BatchItem* items,
                          const int* wg_first, int grid, int parity, int s, int tile, TW alpha,
                          TW beta, hipStream_t st);
template <typename T, typename TW>
int batch55_blocks_per_cu(int tile);
// The same for ensembles whose boxes all use the array-of-structures layout.
template <typename T, typename TW>
hipError_t launch_batch55_aos(const BatchBox<T, TW>* boxes, const BatchItem* items,
                              const int* wg_first, int grid, int parity, int s, int tile,
                              TW alpha, TW beta, hipStream_t st);
template <typename T, typename TW>
int batch55_blocks_per_cu_aos(int tile);

// 19-point method: pass 1 (divergence, partial update) and pass 2 (the
// (nu/3) grad div u term).  tile 0 runs the direct kernels, which read the
// ghost zones of the state (pass 1) and of the divergence (pass 2); the
// z-sweep shapes resolve periodic images themselves.
template <typename T, typename TW>
hipError_t launch_pass19a(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w, T* div,
                          const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                          const ForceArgs<T>* frc, hipStream_t st);
template <typename T, typename TW>
hipError_t launch_pass19a_sweep(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                                T* div, const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile,
                                int zchunk, const ForceArgs<T>* frc, hipStream_t st);
// With partials != nullptr, substep 3 of a z-sweep shape also writes the FP64
// diagnostics partials of the new state (as launch_substep55 does).
template <typename T, typename TW>
hipError_t launch_pass19b(const Geom& g, const T* div, Fields4<T> out, Fields4<TW> w,
                          const Coef<T>& c, const RKCoef<TW>& rk, int s, int tile, int zchunk,
                          double* partials, int part_cap, int* nparts, hipStream_t st);

// FP64 reductions: per-block partials then one fixed-order final block.
constexpr int kReduceBlocks = 1024;
constexpr int kFusedPartials = 8192;  // partial slots for diagnostics fused into substep 3
constexpr int kReduceSlots = 8;  // mass, ke, sum lnrho, umax, nonfinite, pad
template <typename T>
hipError_t launch_reduce(const Geom& g, Fields4<T> f, double* partials, double* result,
                         double dV, hipStream_t s);
// Final fixed-order combination of nparts partials into result.
hipError_t launch_reduce_final(const double* partials, int nparts, double* result, double dV,
                               hipStream_t s);


int substep55_tile_count();

}  // namespace fd6
