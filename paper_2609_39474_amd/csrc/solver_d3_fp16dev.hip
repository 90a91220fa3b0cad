// Solver instantiation: lattice D3Q19, FP16 deviation-from-equilibrium storage.
#include "msc_solver_impl.h"

namespace msc {
SolverBase* make_solver_d3_fp16dev(const msc_params& p, const Geometry& g, hipStream_t s) {
  return new Solver<D3Q19, _Float16>(p, g, s);
}
}  // namespace msc
