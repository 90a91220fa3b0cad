// Solver instantiation: lattice D3Q19, storage float.
#include "msc_solver_impl.h"

namespace msc {
SolverBase* make_solver_d3_fp32(const msc_params& p, const Geometry& g, hipStream_t s) {
  return new Solver<D3Q19, float>(p, g, s);
}
}  // namespace msc
