// Instantiations of the 55-point z-sweep substep (single box and ensemble)
// for the array-of-structures state layout, state type float and RK3 register
// type float (a translation unit of its own keeps the build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55_aos<float, float>(const Geom&, Fields4<float>, Fields4<float>,
                                                   Fields4<float>, const Coef<float>&,
                                                   const RKCoef<float>&, int, int, int, double*,
                                                   int, int*, const ForceArgs<float>*,
                                                   hipStream_t);
template hipError_t launch_batch55_aos<float, float>(const BatchBox<float, float>*,
                                                 const BatchItem*, const int*, int, int, int, int,
                                                 float, float, hipStream_t);
template int batch55_blocks_per_cu_aos<float, float>(int);

bool substep55_aos_tile_ok(int tile) {
    return tile > 0 && tile < kNumTiles && !kTiles[tile].ld;
}

}  // namespace fd6
