// Instantiations of the 55-point z-sweep substep (single box and ensemble)
// for the array-of-structures state layout, state type float and RK3 register
// type double (a translation unit of its own keeps the build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55_aos<float, double>(const Geom&, Fields4<float>, Fields4<float>,
                                                   Fields4<double>, const Coef<float>&,
                                                   const RKCoef<double>&, int, int, int, double*,
                                                   int, int*, const ForceArgs<float>*,
                                                   hipStream_t);
template hipError_t launch_batch55_aos<float, double>(const BatchBox<float, double>*,
                                                 const BatchItem*, const int*, int, int, int, int,
                                                 double, double, hipStream_t);
template int batch55_blocks_per_cu_aos<float, double>(int);

}  // namespace fd6
