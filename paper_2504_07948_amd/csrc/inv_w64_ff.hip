// Wave inverse instantiation for padded width 64 (float, float).
#include "inverse.h"

namespace dmcx {
template void launch_inverse_nr<float, float, 64>(const DevCtx &, const float *, int, double *, int,
                                             hipStream_t);
}  // namespace dmcx
