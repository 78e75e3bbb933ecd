// Wave inverse instantiations for padded widths 16, 32 and 48.
#include "inverse.h"

namespace dmcx {
#define DMCX_INV(T, S, NR) \
  template void launch_inverse_nr<T, S, NR>(const DevCtx &, const S *, int, double *, int, hipStream_t);
DMCX_INV(double, double, 16) DMCX_INV(double, double, 32) DMCX_INV(double, double, 48)
DMCX_INV(float, float, 16) DMCX_INV(float, float, 32) DMCX_INV(float, float, 48)
DMCX_INV(float, double, 16) DMCX_INV(float, double, 32) DMCX_INV(float, double, 48)
#undef DMCX_INV
}  // namespace dmcx
