// Wave inverse instantiation for padded width 64 (double, double).
#include "inverse.h"

namespace dmcx {
template void launch_inverse_nr<double, double, 64>(const DevCtx &, const double *, int, double *, int,
                                             hipStream_t);
}  // namespace dmcx
