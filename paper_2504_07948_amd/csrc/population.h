// Population control: comb reconfiguration of one system's walkers at fixed
// population (the DMC weights of Eq. 1 decide the copies; the paper does not
// fix the control scheme, this is the published systematic-resampling form).
#pragma once
#include "kernels.h"

namespace dmcx {

// Device scratch of one system's reconfiguration ([Wpad] each unless noted).
struct PopScratch {
  double *w;      // weights, then their cumulative sums
  int *copies;    // copies of each walker in the next population
  int *dead;      // walkers without a copy, lowest first
  int *ex;        // inclusive prefix of the extra copies
  int2 *pairs;    // (destination, source) of every extra copy
  int *n_pairs;   // [1]
  double *lwbar;  // [1] log of the mean weight (NaN: no positive weight)
};

// Select (one workgroup), copy the per-walker state of every pair and give
// every walker the mean weight.  es: bytes per working-precision element.
hipError_t launch_reconfigure(const DevCtx &c, size_t es, double u, const PopScratch &p,
                              hipStream_t s);

}  // namespace dmcx
