// Instantiations of the 55-point z-sweep substep for the array-of-structures
// state layout, state type float and RK3 register type double (a translation
// unit of its own keeps the build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55_aos<float, double>(const Geom&, Fields4<float>, Fields4<float>,
                                                  Fields4<double>, const Coef<float>&,
                                                  const RKCoef<double>&, int, int, int, double*,
                                                  int, int*, const ForceArgs<float>*, hipStream_t);

}  // namespace fd6
