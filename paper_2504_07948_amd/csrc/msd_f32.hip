// FP32 (mixed form) multideterminant sweep kernels and launcher.
#include "msd_impl.h"

namespace dmcx {
template struct MsdLaunch<float>;
}
