// Substeps 1 and 2 fused in one launch (temporal blocking, discussion of
// Sec. 7), FP32 state and register, either state layout: the launcher of
// substep55_fused12 (16 x 16 output tiles, 22 x 22 threads).
#include "sweep_substep.hpp"

namespace fd6 {

namespace {
template <typename T, typename TW, int VS>
hipError_t launch_fused12_vs(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                             const Coef<T>& c, const RKCoef<TW>& rk1, const RKCoef<TW>& rk2,
                             int zchunk, hipStream_t st) {
    constexpr int TX = 16, TY = 16, PD = 2;
    constexpr int NT = (TX + 2 * kR) * (TY + 2 * kR);
    constexpr auto kern = substep55_fused12<T, TW, TX, TY, PD, true, VS>;
    const int res = resident_blocks<kern>(NT);
    const SweepGrid sg = sweep_grid(g, TX, TY, zchunk, res);
    hipLaunchKernelGGL(kern, dim3(sg.blocks), dim3(NT), 0, st, g, in, out, w, c, rk1, rk2, sg);
    return hipGetLastError();
}
}  // namespace

template <typename T, typename TW>
hipError_t launch_fused12(const Geom& g, Fields4<T> in, Fields4<T> out, Fields4<TW> w,
                          const Coef<T>& c, const RKCoef<TW>& rk1, const RKCoef<TW>& rk2,
                          int zchunk, hipStream_t st) {
    return g.vs == 4 ? launch_fused12_vs<T, TW, 4>(g, in, out, w, c, rk1, rk2, zchunk, st)
                     : launch_fused12_vs<T, TW, 1>(g, in, out, w, c, rk1, rk2, zchunk, st);
}

template hipError_t launch_fused12<float, float>(const Geom&, Fields4<float>, Fields4<float>,
                                                 Fields4<float>, const Coef<float>&,
                                                 const RKCoef<float>&, const RKCoef<float>&, int,
                                                 hipStream_t);

}  // namespace fd6
