// FP64 instantiations of the fused low stage (see qst_stages.hpp).  The FP64
// path keeps the whole state in one chunk (R * 2^n <= 8192), so the stage
// always applies the Y phases itself.
#include "qst_stages.hpp"

namespace qst {

#define QST_LO64_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)

hipError_t launch_stage_lo_f64(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  if (g.n_hi != 0) return hipErrorInvalidValue;
  switch (g.n_lo) {
#define QST_P(N) \
  case N: return launch_lo_n<double, N, true, false>(g, m, adjoint, st);
    QST_LO64_CASES(QST_P)
#undef QST_P
  }
  return hipErrorInvalidValue;
}

int lo_occupancy_f64(const Geometry& g) {
  switch (g.n_lo) {
#define QST_P(N) \
  case N: return lo_occupancy_n<double, N, true, false>(g);
    QST_LO64_CASES(QST_P)
#undef QST_P
  }
  return 1;
}

}  // namespace qst
