// Comb reconfiguration at fixed population.
//
// Walker j of W has weight w_j = exp(log_w_j - m), m the largest finite
// log-weight (a non-finite log-weight is weight 0).  C_j = w_0 + ... + w_j is
// summed in walker order by one thread (the order fixes the rounding), S is
// the total.  Tooth k = 0..W-1 of the comb sits at t_k = (k + u) (S / W) and
// selects the first walker with t_k < C_j (binary search; the last walker of
// positive weight if rounding leaves none).  The slots of walkers without a
// copy receive the extra copies, lowest slot first, sources in walker order
// (integer scans, exact in any order), and every walker then carries the
// mean weight S / W (times e^m).
//
// Birth/death branching (the second half of this file) turns the weights
// into integer multiplicities M_j = floor(w_j + u_j), so the walker count
// changes; the host reads the new count between the selection and the
// copies (the launches after it size their grids by it).
#include "population.h"

namespace dmcx {
namespace {

constexpr int NT_SEL = 1024;
constexpr int NT_COPY = 256;
constexpr int COPY_SPLIT = 8;  // workgroups sharing one walker's copy

// Block-wide inclusive scan of one int per thread (NT_SEL threads): a scan
// within each wave, then wave 0 scans the wave totals (three barriers).
__device__ int block_scan_incl(int v, int *sh) {
  constexpr int NWV = NT_SEL / 64;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) sh[wv] = v;
  __syncthreads();
  if (wv == 0) {
    int x = lane < NWV ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < NWV; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane < NWV) sh[lane] = x;
  }
  __syncthreads();
  const int r = v + (wv > 0 ? sh[wv - 1] : 0);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(NT_SEL) void k_pop_select(DevCtx c, double u, PopScratch p) {
  __shared__ int sh[NT_SEL / 64];
  __shared__ double cw[NT_SEL];  // one chunk of weights, then of cumulative sums
  __shared__ double red[NT_SEL / 64];
  __shared__ double s_m, s_S;
  __shared__ int s_last, s_carry[2];
  const int W = c.W, t = threadIdx.x;
  // largest finite log-weight (a max is exact in any order)
  double m = -INFINITY;
  for (int j = t; j < W; j += NT_SEL) {
    const double x = c.logw[j];
    if (isfinite(x) && x > m) m = x;
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((t & 63) == 0) red[t >> 6] = m;
  __syncthreads();
  if (t == 0) {
    double mm = red[0];
    for (int i = 1; i < NT_SEL / 64; ++i) mm = fmax(mm, red[i]);
    s_m = mm;
    s_S = 0.0;
    s_last = 0;
    s_carry[0] = 0;
    s_carry[1] = 0;
  }
  __syncthreads();
  m = s_m;
  if (!isfinite(m)) {  // no positive weight: the population stays as it is
    for (int j = t; j < W; j += NT_SEL) p.copies[j] = 1;
    if (t == 0) {
      *p.n_pairs = 0;
      *p.lwbar = NAN;
    }
    return;
  }
  // cumulative weights chunk by chunk: the chunk's weights go to LDS and one
  // thread adds them in walker order (the order fixes the rounding)
  for (int j0 = 0; j0 < W; j0 += NT_SEL) {
    const int j = j0 + t;
    double w = 0.0;
    if (j < W) {
      const double x = c.logw[j];
      w = isfinite(x) ? exp(x - m) : 0.0;
      p.copies[j] = 0;
    }
    cw[t] = w;
    __syncthreads();
    if (t == 0) {
      double acc = s_S;
      int last = s_last;
      // groups of 16: the reads go out together, the adds stay in walker
      // order; entries past W hold 0.0, and acc + 0.0 == acc exactly
      const int n = min(NT_SEL, W - j0);
      for (int q0 = 0; q0 < n; q0 += 16) {
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = cw[q0 + r];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (x[r] > 0.0) last = j0 + q0 + r;
          acc += x[r];
          cw[q0 + r] = acc;
        }
      }
      s_S = acc;
      s_last = last;
    }
    __syncthreads();
    if (j < W) p.w[j] = cw[t];
    __syncthreads();
  }
  const double S = s_S, step = S / (double)W;
  const int last = s_last;
  for (int k = t; k < W; k += NT_SEL) {
    const double tk = ((double)k + u) * step;
    int lo = 0, hi = W;  // first j with tk < C_j
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (tk < p.w[mid]) hi = mid; else lo = mid + 1;
    }
    atomicAdd(&p.copies[lo < W ? lo : last], 1);
  }
  __syncthreads();
  // dead slots in order (dead[r] = r-th walker without a copy) and the
  // inclusive prefix of the extra copies (ex[j] = extras of walkers <= j)
  for (int j0 = 0; j0 < W; j0 += NT_SEL) {
    const int j = j0 + t;
    const int cj = j < W ? p.copies[j] : 1;
    const int d = cj == 0 ? 1 : 0;
    const int e = cj > 1 ? cj - 1 : 0;
    const int di = block_scan_incl(d, sh);
    const int ei = block_scan_incl(e, sh);
    if (d) p.dead[s_carry[0] + di - 1] = j;
    if (j < W) p.ex[j] = s_carry[1] + ei;
    __syncthreads();
    if (t == NT_SEL - 1) {
      s_carry[0] += di;
      s_carry[1] += ei;
    }
    __syncthreads();
  }
  // extra copy r (walkers in order) -> the r-th dead slot; its source is the
  // first walker whose inclusive extra count exceeds r
  const int np = s_carry[1];
  for (int r = t; r < np; r += NT_SEL) {
    int lo = 0, hi = W - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (p.ex[mid] > r) hi = mid; else lo = mid + 1;
    }
    p.pairs[r] = make_int2(p.dead[r], lo);
  }
  if (t == 0) {
    *p.n_pairs = np;
    *p.lwbar = m + log(S / (double)W);
  }
}

// Copy nbytes between two walker slots of one array with the lanes of the
// COPY_SPLIT workgroups of a pair (16-byte words when both ends and the size
// allow it).
__device__ __forceinline__ void slot_copy(void *dst, const void *src, size_t nbytes) {
  const size_t t = threadIdx.x + (size_t)blockIdx.y * NT_COPY, nt = (size_t)NT_COPY * COPY_SPLIT;
  const uintptr_t a = (uintptr_t)dst | (uintptr_t)src | (uintptr_t)nbytes;
  if ((a & 15) == 0) {
    uint4 *d = (uint4 *)dst;
    const uint4 *s = (const uint4 *)src;
    for (size_t i = t; i < nbytes / 16; i += nt) d[i] = s[i];
  } else if ((a & 7) == 0) {
    uint2 *d = (uint2 *)dst;
    const uint2 *s = (const uint2 *)src;
    for (size_t i = t; i < nbytes / 8; i += nt) d[i] = s[i];
  } else {
    unsigned *d = (unsigned *)dst;
    const unsigned *s = (const unsigned *)src;
    for (size_t i = t; i < nbytes / 4; i += nt) d[i] = s[i];
  }
}

// Every state a walker carries from one step to the next: positions, cached
// orbital VGL rows, inverses, log|D| and signs, E_L, log|Psi|, V, flags and,
// with a multideterminant expansion, its table, minors and S.  (The block
// buffers of the delayed update are empty between steps.)
__global__ __launch_bounds__(NT_COPY) void k_pop_copy(DevCtx c, size_t es, PopScratch p) {
  const int b = blockIdx.x;
  if (b >= *p.n_pairs) return;
  const int2 pr = p.pairs[b];
  const size_t dst = (size_t)pr.x, src = (size_t)pr.y;
  const size_t ne = (size_t)c.ne, NP = (size_t)c.NP;
  const size_t r = ne * 3 * sizeof(double);
  slot_copy((char *)c.R + dst * r, (const char *)c.R + src * r, r);
  const size_t v = ne * 5 * NP * es;
  slot_copy((char *)c.vglc + dst * v, (const char *)c.vglc + src * v, v);
  const size_t g = 2 * NP * NP * es;
  slot_copy((char *)c.GT + dst * g, (const char *)c.GT + src * g, g);
  if (c.M.on) {
    const size_t tt = 2 * NP * (size_t)c.M.ldt * es;
    slot_copy((char *)c.M.Tt + dst * tt, (const char *)c.M.Tt + src * tt, tt);
    const size_t rd = 2 * (size_t)c.M.n_det * sizeof(double);
    slot_copy((char *)c.M.Rdet + dst * rd, (const char *)c.M.Rdet + src * rd, rd);
  }
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    c.logdet[2 * dst] = c.logdet[2 * src];
    c.logdet[2 * dst + 1] = c.logdet[2 * src + 1];
    c.sgn[2 * dst] = c.sgn[2 * src];
    c.sgn[2 * dst + 1] = c.sgn[2 * src + 1];
    c.eloc[dst] = c.eloc[src];
    c.logpsi[dst] = c.logpsi[src];
    c.vpot[dst] = c.vpot[src];
    c.flags[dst] = c.flags[src];
    if (c.M.on) c.M.S[dst] = c.M.S[src];
  }
}

__global__ void k_pop_finish(DevCtx c, PopScratch p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const double lw = *p.lwbar;
  if (j < c.W && isfinite(lw)) c.logw[j] = lw;
}

// Branching selection (one workgroup; see launch_branch_select).
__global__ __launch_bounds__(NT_SEL) void k_branch_select(DevCtx c, uint64_t step, int cap, int tw,
                                                          PopScratch p) {
  __shared__ int sh[NT_SEL / 64];
  __shared__ double red[NT_SEL / 64];
  __shared__ int s_carry[3];
  const int W = c.W, t = threadIdx.x;
  // multiplicities (clamped at cap + 1: any larger total is refused anyway);
  // their total as a double is exact while below 2^53 and above cap beyond
  double tot = 0.0;
  for (int j = t; j < W; j += NT_SEL) {
    double u0, u1;
    uniform_pair(c.seed, (uint32_t)step, (uint32_t)j, 0u, 5u, u0, u1);
    const double x = c.logw[j];
    const double m = (isfinite(x) && c.flags[j] == 0u) ? floor(exp(x) + u0) : 0.0;
    const int mj = m > (double)cap ? cap + 1 : (int)m;
    p.copies[j] = mj;
    tot += (double)mj;
  }
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  if ((t & 63) == 0) red[t >> 6] = tot;
  if (t < 3) s_carry[t] = 0;
  __syncthreads();
  tot = 0.0;
  for (int i = 0; i < NT_SEL / 64; ++i) tot += red[i];
  if (tot < 1.0 || tot > (double)cap) {
    if (t == 0) {
      p.info[0] = 5;
      p.info[1] = tot > (double)cap ? cap + 1 : (int)tot;
      p.info[2] = 0;
      p.info[3] = 0;
    }
    return;
  }
  const int Wn = (int)tot;
  // dead slots in order, the inclusive prefixes of the extra copies and of
  // the walkers with a copy (all counts <= cap now)
  for (int j0 = 0; j0 < W; j0 += NT_SEL) {
    const int j = j0 + t;
    const int cj = j < W ? p.copies[j] : 1;
    const int d = cj == 0 ? 1 : 0;
    const int e = cj > 1 ? cj - 1 : 0;
    const int a = (j < W && cj > 0) ? 1 : 0;
    const int di = block_scan_incl(d, sh);
    const int ei = block_scan_incl(e, sh);
    const int ai = block_scan_incl(a, sh);
    if (d && j < W) p.dead[s_carry[0] + di - 1] = j;
    if (j < W) {
      p.ex[j] = s_carry[1] + ei;
      p.alive[j] = s_carry[2] + ai;
    }
    __syncthreads();
    if (t == NT_SEL - 1) {
      s_carry[0] += di;
      s_carry[1] += ei;
      s_carry[2] += ai;
    }
    __syncthreads();
  }
  const int nd = s_carry[0], E = s_carry[1];
  // extra copy r (walkers in order): the r-th dead slot, then the new slots
  for (int r = t; r < E; r += NT_SEL) {
    int lo = 0, hi = W - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (p.ex[mid] > r) hi = mid; else lo = mid + 1;
    }
    p.pairs[r] = make_int2(r < nd ? p.dead[r] : W + (r - nd), lo);
  }
  // walkers in slots >= W' (in order) -> the dead slots after the extras'
  // (these lie below W': as many empty slots below W' remain as there are
  // walkers with a copy at or above W')
  const int base = Wn < W ? p.alive[Wn - 1] : 0;
  for (int j = Wn + t; j < W; j += NT_SEL)
    if (p.copies[j] > 0) {
      const int k = p.alive[j] - base - 1;
      p.pairs[E + k] = make_int2(p.dead[E + k], j);
    }
  const int nmove = Wn < W ? p.alive[W - 1] - base : 0;
  const int np = E + nmove;
  const int Wnp = (Wn + tw - 1) / tw * tw;
  for (int i = t; i < Wnp - Wn; i += NT_SEL) p.pairs[np + i] = make_int2(Wn + i, 0);
  if (t == 0) {
    p.n_pairs[0] = np;
    p.n_pairs[1] = Wnp - Wn;
    p.info[0] = 0;
    p.info[1] = Wn;
    p.info[2] = np;
    p.info[3] = Wnp - Wn;
  }
}

__global__ void k_branch_finish(DevCtx c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < c.Wpad) c.logw[j] = 0.0;
}

}  // namespace

hipError_t launch_branch_select(const DevCtx &c, uint64_t step, int cap, int tw,
                                const PopScratch &p, hipStream_t s) {
  hipLaunchKernelGGL(k_branch_select, dim3(1), dim3(NT_SEL), 0, s, c, step, cap, tw, p);
  return hipGetLastError();
}

hipError_t launch_branch_copy(const DevCtx &c, size_t es, int n_main, int n_pad,
                              const PopScratch &p, hipStream_t s) {
  // every destination is an empty slot and every source a surviving walker's
  // own slot, so the main copies are independent; the padding copies read
  // slot 0 after them
  if (n_main > 0)
    hipLaunchKernelGGL(k_pop_copy, dim3(n_main, COPY_SPLIT), dim3(NT_COPY), 0, s, c, es, p);
  if (n_pad > 0) {
    PopScratch q = p;
    q.pairs = p.pairs + n_main;
    q.n_pairs = p.n_pairs + 1;
    hipLaunchKernelGGL(k_pop_copy, dim3(n_pad, COPY_SPLIT), dim3(NT_COPY), 0, s, c, es, q);
  }
  hipLaunchKernelGGL(k_branch_finish, dim3((c.Wpad + 255) / 256), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_reconfigure(const DevCtx &c, size_t es, double u, const PopScratch &p,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pop_select, dim3(1), dim3(NT_SEL), 0, s, c, u, p);
  // at most W - 1 pairs; blocks past the selected count return at once
  hipLaunchKernelGGL(k_pop_copy, dim3(c.W, COPY_SPLIT), dim3(NT_COPY), 0, s, c, es, p);
  hipLaunchKernelGGL(k_pop_finish, dim3((c.W + 255) / 256), dim3(256), 0, s, c, p);
  return hipGetLastError();
}

}  // namespace dmcx
