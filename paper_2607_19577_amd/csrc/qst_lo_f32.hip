// FP32 instantiations of the fused low stage (see qst_stages.hpp).  Compiled
// twice: intermediates in FP32, and (QST_LO_H16) in BF16.
#include "qst_stages.hpp"

#ifndef QST_LO_H16
#define QST_LO_H16 false
#define QST_LO_SUFFIX(name) name##_f32
#endif

namespace qst {

#define QST_LO_CASES(X)                                                                                      \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t QST_LO_SUFFIX(launch_stage_lo)(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  if (g.n_hi == 0) {  // the state is one chunk: this stage applies the Y phases itself
    switch (g.n_lo) {
#define QST_P(N) \
  case N: return launch_lo_n<float, N, true, QST_LO_H16>(g, m, adjoint, st);
      QST_LO_CASES(QST_P)
#undef QST_P
    }
    return hipErrorInvalidValue;
  }
  switch (g.n_lo) {
    case 6: return launch_lo_n<float, 6, false, QST_LO_H16>(g, m, adjoint, st);
    case 7: return launch_lo_n<float, 7, false, QST_LO_H16>(g, m, adjoint, st);
    case 8: return launch_lo_n<float, 8, false, QST_LO_H16>(g, m, adjoint, st);
    case 9: return launch_lo_n<float, 9, false, QST_LO_H16>(g, m, adjoint, st);
    case 10: return launch_lo_n<float, 10, false, QST_LO_H16>(g, m, adjoint, st);
    case 11: return launch_lo_n<float, 11, false, QST_LO_H16>(g, m, adjoint, st);
    case 12: return launch_lo_n<float, 12, false, QST_LO_H16>(g, m, adjoint, st);
    case 13: return launch_lo_n<float, 13, false, QST_LO_H16>(g, m, adjoint, st);
    case 14: return launch_lo_n<float, 14, false, QST_LO_H16>(g, m, adjoint, st);
  }
  return hipErrorInvalidValue;
}

int QST_LO_SUFFIX(lo_occupancy)(const Geometry& g) {
  if (g.n_hi == 0) {
    switch (g.n_lo) {
#define QST_P(N) \
  case N: return lo_occupancy_n<float, N, true, QST_LO_H16>(g);
      QST_LO_CASES(QST_P)
#undef QST_P
    }
    return 1;
  }
  switch (g.n_lo) {
    case 6: return lo_occupancy_n<float, 6, false, QST_LO_H16>(g);
    case 7: return lo_occupancy_n<float, 7, false, QST_LO_H16>(g);
    case 8: return lo_occupancy_n<float, 8, false, QST_LO_H16>(g);
    case 9: return lo_occupancy_n<float, 9, false, QST_LO_H16>(g);
    case 10: return lo_occupancy_n<float, 10, false, QST_LO_H16>(g);
    case 11: return lo_occupancy_n<float, 11, false, QST_LO_H16>(g);
    case 12: return lo_occupancy_n<float, 12, false, QST_LO_H16>(g);
    case 13: return lo_occupancy_n<float, 13, false, QST_LO_H16>(g);
    case 14: return lo_occupancy_n<float, 14, false, QST_LO_H16>(g);
  }
  return 1;
}

}  // namespace qst
