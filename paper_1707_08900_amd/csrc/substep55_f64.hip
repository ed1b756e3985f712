// Instantiations of the 55-point substep kernels for state type double and RK3
// register type double (one translation unit per precision form keeps the
// build parallel).
#include "substep55_impl.hpp"

namespace fd6 {

template hipError_t launch_substep55<double, double>(const Geom&, Fields4<double>, Fields4<double>,
                                              Fields4<double>, const Coef<double>&,
                                              const RKCoef<double>&, int, int, hipStream_t);
template hipError_t launch_batch55<double, double>(const BatchBox<double, double>*, const BatchItem*, int,
                                            int, int, int, int, double, double, hipStream_t);
template int batch55_blocks_per_cu<double, double>(int);

}  // namespace fd6
