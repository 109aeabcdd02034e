// Instantiations of the high-bit tile stages A (forward) and C (adjoint and
// gradient accumulation), see qst_stages.hpp.
#include "qst_stages.hpp"

namespace qst {

// Supported (tile bits, high bits) pairs of the FP32 path: n in 11..20 with the
// low-stage sizes chosen by the host (n_lo >= 10).
hipError_t launch_stage_hi_gen(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st);

hipError_t launch_stage_hi(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st) {
  if (g.elem != 4 || a.nsplit < 1 || a.nsplit > a.S) return hipErrorInvalidValue;
  if (g.gen) return g.h16 ? hipErrorInvalidValue : launch_stage_hi_gen(g, a, adjoint, st);
#define QST_HI(TBv, NHv)                                                       \
  if (g.t == TBv && g.n_hi == NHv)                                             \
    return g.h16 ? launch_hi_n<TBv, NHv, true>(g, a, adjoint, st)              \
                 : launch_hi_n<TBv, NHv, false>(g, a, adjoint, st);
  QST_HI(14, 1) QST_HI(14, 2) QST_HI(14, 3) QST_HI(14, 4) QST_HI(14, 5)
  QST_HI(14, 6) QST_HI(14, 7) QST_HI(14, 8) QST_HI(14, 9) QST_HI(14, 10)
  QST_HI(13, 1) QST_HI(13, 2) QST_HI(13, 3) QST_HI(12, 1) QST_HI(12, 2) QST_HI(11, 1)
#undef QST_HI
  return hipErrorInvalidValue;
}

}  // namespace qst
