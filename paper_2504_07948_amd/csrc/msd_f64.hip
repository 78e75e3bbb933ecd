// FP64 multideterminant sweep kernels and launcher.
#include "msd_impl.h"

namespace dmcx {
template struct MsdLaunch<double>;
}
