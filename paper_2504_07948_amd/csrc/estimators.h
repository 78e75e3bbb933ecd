// Weighted walker estimators of one system, in FP64 (the walker weights of
// Eq. 1: omega_w = exp(log w_w - m) with m the largest log-weight, so the
// sums stay finite however far the log-weights drift).
//
// Two passes over the walkers: blocks of EST_NB walkers write one partial
// record each (their own shift m_b, shifted sums, centred second moment,
// extremes, move counters) into a scratch buffer; one thread then merges the
// records in block order (log-sum-exp rescaling exp(m_b - m) and the
// pairwise update of the centred moment), so the result does not depend on
// the launch and the variance never forms <E^2> - <E>^2.
//
// A walker counts when its log-weight and E_L are finite and its status flags
// are clear (the comb of population control gives such walkers weight zero
// too).  The per-walker move counters (moves proposed and accepted since the
// previous call) are read by every real walker and cleared in the same pass.
#pragma once
#include "kernels.h"

namespace dmcx {

constexpr int EST_NB = 256;   // walkers (threads) per block of the first pass
constexpr int EST_PART = 10;  // doubles per block record
constexpr int EST_OUT = 11;   // doubles per system (DMCX_N_ESTIMATORS)

__device__ __forceinline__ double max64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double min64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide reduction of one value over EST_NB threads (4 waves): the wave
// results meet in LDS and every thread gets the total.  op: 0 sum, 1 max, 2 min.
template <int OP>
__device__ __forceinline__ double block_reduce(double v, double *red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = OP == 0 ? sum64(v) : (OP == 1 ? max64(v) : min64(v));
  __syncthreads();  // red is reused by consecutive calls
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int q = 1; q < EST_NB / 64; ++q)
    r = OP == 0 ? r + red[q] : (OP == 1 ? fmax(r, red[q]) : fmin(r, red[q]));
  return r;
}

// Inputs of the first pass: one system's per-walker arrays (device
// pointers).  F is the element type of the status flags (the context's own
// flags are 32-bit; an array from dmcx_walker_flags is 8-bit).  flags may be
// null (no walker flagged); nacc and nprop are both given or both null (no
// move counters: nothing accepted, nothing proposed).
template <typename F>
struct EstIn {
  int W;
  const double *logw, *eloc;
  const F *flags;
  unsigned *nacc, *nprop;
};

// Record of block b: {m_b, S0, S1, S2, Q, M2, n, min log w, accepted, proposed}
// with S0 = sum omega, S1 = sum omega E, S2 = sum omega E^2, Q = sum omega^2,
// M2 = sum omega (E - S1/S0)^2, omega = exp(log w - m_b).
template <typename F>
__global__ __launch_bounds__(EST_NB) void k_est_partial(EstIn<F> in, double *part) {
  __shared__ double red[EST_NB / 64];
  const int w = blockIdx.x * EST_NB + threadIdx.x;
  const bool real = w < in.W;
  const double lw_in = real ? in.logw[w] : 0.0, e_in = real ? in.eloc[w] : 0.0;
  const bool clear = !real || !in.flags || in.flags[w] == (F)0;
  const bool ok = real && clear && isfinite(lw_in) && isfinite(e_in);
  // excluded walkers enter every sum as exact zeros (0 * NaN would not be)
  const double lw = ok ? lw_in : 0.0, e = ok ? e_in : 0.0;
  double na = 0.0, np = 0.0;
  if (real && in.nacc) {
    na = (double)in.nacc[w];
    np = (double)in.nprop[w];
    in.nacc[w] = 0u;
    in.nprop[w] = 0u;
  }
  const double mb = block_reduce<1>(ok ? lw : -INFINITY, red);
  const double lmin = block_reduce<2>(ok ? lw : INFINITY, red);
  const double om = ok ? exp(lw - mb) : 0.0;
  const double s0 = block_reduce<0>(om, red);
  const double s1 = block_reduce<0>(om * e, red);
  const double s2 = block_reduce<0>(om * e * e, red);
  const double q = block_reduce<0>(om * om, red);
  const double n = block_reduce<0>(ok ? 1.0 : 0.0, red);
  const double mu = s0 > 0.0 ? s1 / s0 : 0.0;
  const double m2 = block_reduce<0>(ok ? om * (e - mu) * (e - mu) : 0.0, red);
  const double acc = block_reduce<0>(na, red);
  const double prop = block_reduce<0>(np, red);
  if (threadIdx.x == 0) {
    double *r = part + (size_t)blockIdx.x * EST_PART;
    r[0] = mb; r[1] = s0; r[2] = s1; r[3] = s2; r[4] = q;
    r[5] = m2; r[6] = n; r[7] = lmin; r[8] = acc; r[9] = prop;
  }
}

// Merge the nblk records (block order) into out[EST_OUT]:
//   0 walkers counted, 1 m = max log w, 2 S0, 3 S1, 4 S2, 5 Q (all shifted by
//   m), 6 <E_L>_w = S1/S0, 7 weighted variance M2/S0, 8 min log w,
//   9 acceptance ratio (accepted / proposed moves since the previous call;
//   NaN when no move was proposed), 10 moves proposed.
// With no walker counted, 1..8 are NaN.
__device__ inline void est_merge(int nblk, const double *part, double *out) {
  double m = -INFINITY, lmin = INFINITY, n = 0.0, acc = 0.0, prop = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double *r = part + (size_t)b * EST_PART;
    if (r[6] > 0.0) {
      m = fmax(m, r[0]);
      lmin = fmin(lmin, r[7]);
    }
    n += r[6];
    acc += r[8];
    prop += r[9];
  }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, q = 0.0, mu = 0.0, m2 = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double *r = part + (size_t)b * EST_PART;
    if (!(r[6] > 0.0)) continue;
    const double f = exp(r[0] - m);
    const double w0 = f * r[1];
    const double mub = r[2] / r[1];
    // pairwise merge of (weight, mean, centred moment)
    const double tot = s0 + w0;
    const double d = mub - mu;
    m2 += f * r[5] + d * d * s0 * w0 / tot;
    mu += d * w0 / tot;
    s0 = tot;
    s1 += f * r[2];
    s2 += f * r[3];
    q += f * f * r[4];
  }
  const bool any = n > 0.0;
  const double nan = __builtin_nan("");
  out[0] = n;
  out[1] = any ? m : nan;
  out[2] = any ? s0 : nan;
  out[3] = any ? s1 : nan;
  out[4] = any ? s2 : nan;
  out[5] = any ? q : nan;
  out[6] = any ? s1 / s0 : nan;
  out[7] = any ? m2 / s0 : nan;
  out[8] = any ? lmin : nan;
  out[9] = prop > 0.0 ? acc / prop : nan;
  out[10] = prop;
}
__global__ void k_est_final(int nblk, const double *part, double *out) {
  if (threadIdx.x == 0) est_merge(nblk, part, out);
}

// E_T feedback after a DMC step (population control of the projection of
// Eq. 1):  E_T <- <E_L>_w - (gain / tau) ln(W_tot / W), with the weighted
// mean energy and ln W_tot = m + ln S0 from the merged block records.  Left
// unchanged in VMC steps and when no walker counts.
__global__ void k_et_feedback(int nblk, const double *part, RunState *run, double gain,
                              double tau, int W) {
  if (threadIdx.x != 0 || run->mode != 1) return;
  double r[EST_OUT];
  est_merge(nblk, part, r);
  if (r[0] > 0.0) run->e_trial = r[6] - gain / tau * (r[1] + log(r[2]) - log((double)W));
}

inline int est_blocks(int W) { return (W + EST_NB - 1) / EST_NB; }

// The first-pass inputs of a context: its own walker arrays and counters.
inline EstIn<unsigned> est_in(const DevCtx &c) {
  return EstIn<unsigned>{c.W, c.logw, c.eloc, c.flags, c.nacc, c.nprop};
}

}  // namespace dmcx
