// Instantiations of the z-sweep substep kernels (55-point single box and
// batch, 19-point pass 1) for state type double and RK3
// register type double (one translation unit per precision form keeps the
// build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55<double, double>(const Geom&, Fields4<double>, Fields4<double>,
                                              Fields4<double>, const Coef<double>&,
                                              const RKCoef<double>&, int, int, int, double*, int,
                                              int*, const ForceArgs<double>*, hipStream_t);
template hipError_t launch_batch55<double, double>(const BatchBox<double, double>*, const BatchItem*, const int*,
                                            int, int, int, int, double, double, hipStream_t);
template int batch55_blocks_per_cu<double, double>(int);
template hipError_t launch_pass19a_sweep<double, double>(const Geom&, Fields4<double>, Fields4<double>,
                                                  Fields4<double>, double*, const Coef<double>&,
                                                  const RKCoef<double>&, int, int, int,
                                                  const ForceArgs<double>*, hipStream_t);

}  // namespace fd6
