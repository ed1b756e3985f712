// Instantiations of the 55-point z-sweep substep for the array-of-structures
// state layout, state type double and RK3 register type double (a translation
// unit of its own keeps the build parallel).
#include "sweep_substep.hpp"

namespace fd6 {

template hipError_t launch_substep55_aos<double, double>(const Geom&, Fields4<double>, Fields4<double>,
                                                  Fields4<double>, const Coef<double>&,
                                                  const RKCoef<double>&, int, int, int, double*,
                                                  int, int*, const ForceArgs<double>*, hipStream_t);

}  // namespace fd6
