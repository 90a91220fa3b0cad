// Solver instantiation: lattice D2Q9, FP16 deviation-from-equilibrium storage.
#include "msc_solver_impl.h"

namespace msc {
SolverBase* make_solver_d2_fp16dev(const msc_params& p, const Geometry& g, hipStream_t s) {
  return new Solver<D2Q9, _Float16>(p, g, s);
}
}  // namespace msc
