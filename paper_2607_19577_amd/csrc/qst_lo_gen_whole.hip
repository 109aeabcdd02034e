// FP32 instantiations of the fused low stage for general local settings when the
// state is one chunk (the input is the atoms), see qst_stages.hpp.
#include "qst_stages.hpp"

namespace qst {

#define QST_LO_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t launch_stage_lo_gen_whole(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  switch (g.n_lo) {
#define QST_P(N) \
  case N: return launch_lo_n<float, N, true, false, true>(g, m, adjoint, st);
    QST_LO_CASES(QST_P)
#undef QST_P
  }
  return hipErrorInvalidValue;
}

int lo_occupancy_gen_whole(const Geometry& g) {
  switch (g.n_lo) {
#define QST_P(N) \
  case N: return lo_occupancy_n<float, N, true, false, true>(g);
    QST_LO_CASES(QST_P)
#undef QST_P
  }
  return 1;
}

}  // namespace qst
