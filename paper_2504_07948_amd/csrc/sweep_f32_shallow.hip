// FP32 single-determinant sweep (the mixed form), shallow stages.
#include "sweep_impl.h"

namespace dmcx {
template struct SweepLaunch<float, SHAPE_SHALLOW>;
}
