// Fused low stage with BF16 intermediates (FP32 arithmetic); same source as qst_lo_f32.hip.
#define QST_LO_H16 true
#define QST_LO_SUFFIX(name) name##_h16
#include "qst_lo_f32.hip"
