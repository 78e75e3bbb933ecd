// Wave inverse instantiation for padded width 64 (float, double).
#include "inverse.h"

namespace dmcx {
template void launch_inverse_nr<float, double, 64>(const DevCtx &, const double *, int, double *, int,
                                             hipStream_t);
}  // namespace dmcx
