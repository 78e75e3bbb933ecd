// FP32 single-determinant sweep (the mixed form), deep stages.
#include "sweep_impl.h"

namespace dmcx {
template struct SweepLaunch<float, SHAPE_DEEP>;
}
