// Instantiations of the high-bit tile stages for general local settings (one 2x2
// matrix per setting and qubit), see qst_stages.hpp.
#include "qst_stages.hpp"

namespace qst {

hipError_t launch_stage_hi_gen(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st) {
  if (g.elem != 4 || g.h16 || !g.gen || a.um == nullptr || a.nsplit < 1 || a.nsplit > a.S) return hipErrorInvalidValue;
#define QST_HI(TBv, NHv) \
  if (g.t == TBv && g.n_hi == NHv) return launch_hi_n<TBv, NHv, false, true>(g, a, adjoint, st);
  QST_HI(14, 1) QST_HI(14, 2) QST_HI(14, 3) QST_HI(14, 4) QST_HI(14, 5)
  QST_HI(14, 6) QST_HI(14, 7) QST_HI(14, 8) QST_HI(14, 9) QST_HI(14, 10)
  QST_HI(13, 1) QST_HI(13, 2) QST_HI(13, 3) QST_HI(12, 1) QST_HI(12, 2) QST_HI(11, 1)
#undef QST_HI
  return hipErrorInvalidValue;
}

}  // namespace qst
