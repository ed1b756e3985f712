// Instantiations of the 55-point z-sweep substep (single box and ensemble)
// for the array-of-structures state layout, state type double and RK3 register
// type double (a translation unit of its own keeps the build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55_aos<double, double>(const Geom&, Fields4<double>, Fields4<double>,
                                                   Fields4<double>, const Coef<double>&,
                                                   const RKCoef<double>&, int, int, int, double*,
                                                   int, int*, const ForceArgs<double>*,
                                                   hipStream_t);
template hipError_t launch_batch55_aos<double, double>(const BatchBox<double, double>*,
                                                 const BatchItem*, const int*, int, int, int, int,
                                                 double, double, hipStream_t);
template int batch55_blocks_per_cu_aos<double, double>(int);

}  // namespace fd6
