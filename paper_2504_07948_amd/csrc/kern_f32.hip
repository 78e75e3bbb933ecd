// FP32 working precision (the mixed form): every NOB-templated kernel but the
// sweep (sweep_f32_*.hip) and its launcher.
#include "kern_impl.h"

namespace dmcx {
template struct NobLaunch<float>;
}
