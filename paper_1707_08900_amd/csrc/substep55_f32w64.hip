// Instantiations of the 55-point substep kernels for state type float and RK3
// register type double (one translation unit per precision form keeps the
// build parallel).
#include "substep55_impl.hpp"

namespace fd6 {

template hipError_t launch_substep55<float, double>(const Geom&, Fields4<float>, Fields4<float>,
                                              Fields4<double>, const Coef<float>&,
                                              const RKCoef<double>&, int, int, hipStream_t);
template hipError_t launch_batch55<float, double>(const BatchBox<float, double>*, const BatchItem*, int,
                                            int, int, int, int, double, double, hipStream_t);
template int batch55_blocks_per_cu<float, double>(int);

}  // namespace fd6
