// FP32 instantiations of the fused low stage for general local settings (one 2x2
// matrix per setting and qubit), see qst_stages.hpp.  States of one chunk (the input
// is the atoms) are instantiated in qst_lo_gen_whole.hip.
#include "qst_stages.hpp"

namespace qst {

hipError_t launch_stage_lo_gen_whole(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
int lo_occupancy_gen_whole(const Geometry& g);

hipError_t launch_stage_lo_gen(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  if (g.n_hi == 0) return launch_stage_lo_gen_whole(g, m, adjoint, st);
  switch (g.n_lo) {
    case 6: return launch_lo_n<float, 6, false, false, true>(g, m, adjoint, st);
    case 7: return launch_lo_n<float, 7, false, false, true>(g, m, adjoint, st);
    case 8: return launch_lo_n<float, 8, false, false, true>(g, m, adjoint, st);
    case 9: return launch_lo_n<float, 9, false, false, true>(g, m, adjoint, st);
    case 10: return launch_lo_n<float, 10, false, false, true>(g, m, adjoint, st);
    case 11: return launch_lo_n<float, 11, false, false, true>(g, m, adjoint, st);
    case 12: return launch_lo_n<float, 12, false, false, true>(g, m, adjoint, st);
    case 13: return launch_lo_n<float, 13, false, false, true>(g, m, adjoint, st);
    case 14: return launch_lo_n<float, 14, false, false, true>(g, m, adjoint, st);
  }
  return hipErrorInvalidValue;
}

int lo_occupancy_gen(const Geometry& g) {
  if (g.n_hi == 0) return lo_occupancy_gen_whole(g);
  switch (g.n_lo) {
    case 6: return lo_occupancy_n<float, 6, false, false, true>(g);
    case 7: return lo_occupancy_n<float, 7, false, false, true>(g);
    case 8: return lo_occupancy_n<float, 8, false, false, true>(g);
    case 9: return lo_occupancy_n<float, 9, false, false, true>(g);
    case 10: return lo_occupancy_n<float, 10, false, false, true>(g);
    case 11: return lo_occupancy_n<float, 11, false, false, true>(g);
    case 12: return lo_occupancy_n<float, 12, false, false, true>(g);
    case 13: return lo_occupancy_n<float, 13, false, false, true>(g);
    case 14: return lo_occupancy_n<float, 14, false, false, true>(g);
  }
  return 1;
}

}  // namespace qst
