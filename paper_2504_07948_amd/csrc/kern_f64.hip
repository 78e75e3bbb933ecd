// FP64 working precision: every NOB-templated kernel but the sweep (sweep_f64.hip)
// and its launcher.
#include "kern_impl.h"

namespace dmcx {
template struct NobLaunch<double>;
}
