// Solver instantiation: lattice D2Q9, storage float.
#include "msc_solver_impl.h"

namespace msc {
SolverBase* make_solver_d2_fp32(const msc_params& p, const Geometry& g, hipStream_t s) {
  return new Solver<D2Q9, float>(p, g, s);
}
}  // namespace msc
