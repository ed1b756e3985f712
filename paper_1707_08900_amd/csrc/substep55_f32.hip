// Instantiations of the z-sweep substep kernels (55-point single box and
// batch, 19-point pass 1) for state type float and RK3
// register type float (one translation unit per precision form keeps the
// build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55<float, float>(const Geom&, Fields4<float>, Fields4<float>,
                                              Fields4<float>, const Coef<float>&,
                                              const RKCoef<float>&, int, int, int, double*, int,
                                              int*, const ForceArgs<float>*, hipStream_t);
template hipError_t launch_batch55<float, float>(const BatchBox<float, float>*, const BatchItem*, const int*,
                                            int, int, int, int, float, float, hipStream_t);
template int batch55_blocks_per_cu<float, float>(int);
template hipError_t launch_pass19a_sweep<float, float>(const Geom&, Fields4<float>, Fields4<float>,
                                                  Fields4<float>, float*, const Coef<float>&,
                                                  const RKCoef<float>&, int, int, int,
                                                  const ForceArgs<float>*, hipStream_t);

int substep55_tile_count() { return kNumTiles; }

bool substep55_reads_ghosts(int tile) { return tile == 0; }

int substep55_tile_dims(int tile, int* tx, int* ty) {
    if (tile <= 0 || tile >= kNumTiles) return -1;
    *tx = kTiles[tile].tx;
    *ty = kTiles[tile].ty;
    return 0;
}

}  // namespace fd6
