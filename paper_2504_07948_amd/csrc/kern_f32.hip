// FP32 working precision (the mixed form): every NOB-templated kernel and
// its launcher.
#include "kern_impl.h"

namespace dmcx {
template struct NobLaunch<float>;
}
