// Solver instantiation: lattice D2Q9, storage double.
#include "msc_solver_impl.h"

namespace msc {
SolverBase* make_solver_d2_fp64(const msc_params& p, const Geometry& g, hipStream_t s) {
  return new Solver<D2Q9, double>(p, g, s);
}
}  // namespace msc
