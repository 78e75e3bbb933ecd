// FP64 single-determinant sweep (deep stages).
#include "sweep_impl.h"

namespace dmcx {
template struct SweepLaunch<double, SHAPE_DEEP>;
}

#ifdef DMCX_PHASE_TIMING
// Profiling builds only: read and clear the sweep's per-phase cycle totals.
extern "C" void dmcx_debug_phase_cycles(unsigned long long out[16]) {
  (void)hipMemcpyFromSymbol(out, HIP_SYMBOL(dmcx::g_phase_cycles), 16 * sizeof(unsigned long long));
  unsigned long long z[16] = {0};
  (void)hipMemcpyToSymbol(HIP_SYMBOL(dmcx::g_phase_cycles), z, sizeof(z));
}
#endif
