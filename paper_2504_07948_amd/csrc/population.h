// Population control of one system's walkers (the DMC weights of Eq. 1
// decide the copies; the paper does not fix the control scheme): comb
// reconfiguration at fixed population (the published systematic-resampling
// form) and birth/death branching with a varying walker count.
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
  int *n_pairs;   // [2] pairs of the copy; of the padding copy (branching)
  double *lwbar;  // [1] log of the mean weight (NaN: no positive weight)
  int *alive;     // branching: inclusive prefix of the walkers with a copy
  int *info;      // branching, [4]: status (0 or 5), W', main pairs, padding pairs
};

// Select (one workgroup), copy the per-walker state of every pair and give
// every walker the mean weight.  es: bytes per working-precision element.
hipError_t launch_reconfigure(const DevCtx &c, size_t es, double u, const PopScratch &p,
                              hipStream_t s);

// Branching, first half: walker j of c.W gets M_j = floor(w_j + u_j) copies
// (w_j = exp(log w_j), 0 for a non-finite log w or a flagged walker; u_j the
// first uniform of Philox draw 5 of (electron 0, walker j, step)); writes
// copies and the (destination, source) pairs of the new population of
// W' = sum M_j walkers, and info = {0 or 5, W', main pairs, padding pairs}.
// Status 5 (W' < 1 or W' > cap; W' then reads min(sum, cap + 1)): nothing
// else is written.  Slot rule: a walker with a copy keeps its slot; the extra
// copies, walkers in order, fill the slots of the walkers without a copy,
// lowest first, then the slots W, W + 1, ...; walkers left in slots >= W'
// move into the empty slots below W', both in slot order.  The padding
// slots W'..ceil(W'/tw)*tw - 1 then receive walker 0.
hipError_t launch_branch_select(const DevCtx &c, uint64_t step, int cap, int tw,
                                const PopScratch &p, hipStream_t s);
// Second half, after the host has read info: the copies (main pairs, then
// the padding pairs from slot 0) and log w = 0 on the new padded range.
// c carries the new W' and its padded size.
hipError_t launch_branch_copy(const DevCtx &c, size_t es, int n_main, int n_pad,
                              const PopScratch &p, hipStream_t s);

}  // namespace dmcx
