// MFMA tile path: fused 4-qubit 16x16 Kronecker tiles (placeholder until the
// tile kernels land; the API reports QST_ERR_UNSUPPORTED for these paths).
#include "qst_internal.hpp"

namespace qst {

hipError_t launch_tile_lo(const Geometry&, const LoArgs&, int, bool, bool, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_tile_hi(const Geometry&, const HiArgs&, bool, bool, hipStream_t) { return hipErrorNotSupported; }

}  // namespace qst
