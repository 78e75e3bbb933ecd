// FP64 inverse of the Slater matrices A_ij = phi_j(r_i) (the periodic
// recompute, and the per-step FP64 energy of the mixed form), one 64-lane
// wave per matrix with the matrix in registers.
//
// Gauss-Jordan elimination in place with partial pivoting: lane r holds row r
// of A (NR >= n registers, NR = the padded orbital count).  Rows are never
// exchanged.  At step k the pivot is the largest |A[r][k]| over the rows not
// yet used as pivots (lowest row on ties), the pivot row p_k is normalised
// and broadcast through LDS, and every other row subtracts its multiple of it:
//   pivot row:  A[p][j] <- A[p][j] / a (j != k),  A[p][k] <- 1 / a,
//   other rows: A[r][j] <- A[r][j] - A[r][k] A[p][j] / a (j != k),
//               A[r][k] <- -A[r][k] / a.
// With pos[r] the step at which row r was the pivot, the finished registers
// hold (A^{-1})[pos[r]][p_m] in lane r, register m, so the inverse column b
// (row b of GT, GT[b][j] = (A^{-1})[j][b]) receives GT[p_m][pos[r]] from lane
// r, register m.  det A = sign(p) prod(pivots), sign(p) the parity of the
// pivot order.  Register indices must be constants (a dynamic index sends the
// row to scratch memory), so the kernel is instantiated per padded width and
// the steps are unrolled in blocks of eight (gj_eliminate).
#pragma once
#include "kernels.h"

namespace dmcx {

constexpr int INV_WAVES = 4;  // matrices (waves) per workgroup

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Largest value over the 64 lanes (wave-uniform), the sum64 pattern with max:
// quad permutations and row rotations inside each 16-lane row, then the four
// row results.  Every lane must be active.
__device__ __forceinline__ double max64_dpp(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x124>(v));
  v = fmax(v, dpp_f64<0x128>(v));
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Per-wave elimination state (wave-uniform except used and pos).
struct GJState {
  bool used;      // this lane's row has been a pivot
  int pos;        // the step at which it was
  double mant;    // prod |pivot| = mant 2^expo, mant in [0.5, 1)
  int expo;
  bool neg;       // odd number of negative pivots
  bool sing;      // a zero pivot was met
};

// The elimination in blocks of eight pivot columns.  The loop over blocks
// stays rolled (the whole elimination unrolled is hundreds of KB of code that
// streams through the instruction cache); inside a block the eight steps are
// unrolled against a working copy w of the block's columns, so every
// register index is a constant.  Each step updates every column of the row
// (the block's columns too, with the same arithmetic as w) and w; the pivot
// columns of the block, whose update differs, are taken back from w at the
// block end.
template <int NR>
__device__ __forceinline__ void gj_eliminate(double (&a)[NR], GJState &st, int n, int lane,
                                             double *prow, int *piv) {
  constexpr int NB = NR / 8;
  for (int kb = 0; kb < NB; ++kb) {
    if (kb * 8 >= n || st.sing) break;
    double w[8];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
      if (jb == kb) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) w[jj] = a[jb * 8 + jj];
      }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = kb * 8 + kk;
      if (k >= n || st.sing) break;
      // pivot: largest |A[r][k]| over unused rows, lowest row on ties (a NaN
      // entry counts as infinite, so the wave agrees on a pivot and the NaN
      // reaches log|det| and the walker's flags)
      const double ak = w[kk];
      const double v = st.used ? -1.0 : (ak != ak ? INFINITY : fabs(ak));
      const double vmax = max64_dpp(v);
      const int p = (int)__builtin_ctzll(__ballot(v == vmax));  // lowest such row
      const double ap = readlane_f64(ak, p);
      if (ap == 0.0) {
        st.sing = true;
        break;
      }
      // |det| as mantissa x 2^exponent, one log at the end
      int ex;
      st.mant = frexp(st.mant * fabs(ap), &ex);
      st.expo += ex;
      st.neg ^= ap < 0.0;
      const double ainv = 1.0 / ap;
      const bool isp = lane == p;
      if (isp) {
        // normalised pivot row; the block's entries come from w
#pragma unroll
        for (int j = 0; j < NR; ++j) prow[j] = a[j] * ainv;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) prow[kb * 8 + jj] = jj == kk ? ainv : w[jj] * ainv;
        piv[k] = p;
        st.pos = k;
        st.used = true;
      }
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const double sj = prow[j];
        a[j] = isp ? sj : fma(-ak, sj, a[j]);
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const double sj = prow[kb * 8 + jj];
        if (jj == kk)
          w[jj] = isp ? ainv : -ak * ainv;
        else
          w[jj] = isp ? sj : fma(-ak, sj, w[jj]);
      }
      wave_lds_sync();  // prow is rewritten by the next step's pivot lane
    }
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
      if (jb == kb) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) a[jb * 8 + jj] = w[jj];
      }
  }
}

// Rows come from `rows` (walker w, electron e at rows + (w ne + e) rs); the
// inverse goes to GT (precision T, transposed and zero padded to NP x NP) and,
// if G64 is not null, to G64 in FP64 with the same layout.  grid:
// ceil(2 Wpad / INV_WAVES) workgroups of INV_WAVES waves; matrix q = (walker
// q / 2, spin q % 2).  periodic != 0: only at steps s = 0 (mod P) of the
// device step counter.
template <typename T, typename S, int NR>
__global__ __launch_bounds__(64 * INV_WAVES) void k_inverse_w(DevCtx c, const S *rows, int rs,
                                                              double *G64, int periodic) {
  __shared__ __align__(16) double prow_all[INV_WAVES][NR];
  __shared__ int piv_all[INV_WAVES][NR];
  __shared__ __align__(16) double stage_all[INV_WAVES][64 * 8];  // 8 columns of 64 rows
  if (periodic && (c.run->step % (unsigned long long)c.P) != 0ull) return;
  const int wv = wave_id(), lane = threadIdx.x & 63;
  const int q = blockIdx.x * INV_WAVES + wv;
  if (q >= 2 * c.Wpad) return;  // whole wave; the kernel has no workgroup barrier
  const int w = q >> 1, sp = q & 1;
  const int n = sp == 0 ? c.n_up : c.n_dn;
  const int NP = c.NP;
  const int e0 = sp == 0 ? 0 : c.n_up;
  double *prow = prow_all[wv];
  int *piv = piv_all[wv];
  T *GT = (T *)c.GT + gt_off(c, w, sp);
  double *G6 = G64 ? G64 + gt_off(c, w, sp) : nullptr;
  if (n == 0) {
    for (int i = lane; i < NP * NP; i += 64) {
      GT[i] = (T)0;
      if (G6) G6[i] = 0.0;
    }
    if (lane == 0) {
      c.logdet[w * 2 + sp] = 0.0;
      c.sgn[w * 2 + sp] = 1.0;
    }
    return;
  }
  // lane r < n: row r; lanes past n hold zeros and are never pivots
  // Rows are read eight columns at a time: each load instruction covers
  // eight rows' 8-column segments (64 consecutive bytes per row, so eight
  // cache lines instead of one line per lane), staged in LDS, from which
  // every lane takes its own row's eight entries.
  double a[NR];
  {
    double *stg = stage_all[wv];
    const S *base = rows + ((size_t)w * c.ne + e0) * rs;
#pragma unroll
    for (int j0 = 0; j0 < NR; j0 += 8) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = 8 * k + (lane >> 3), j = j0 + (lane & 7);
        const double v = (double)base[(size_t)min(r, n - 1) * rs + j];
        stg[r * 8 + (lane & 7)] = (r < n && j < n) ? v : 0.0;
      }
      wave_lds_sync();
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) a[j0 + jj] = stg[lane * 8 + jj];
      wave_lds_sync();  // the next columns are staged in the same place
    }
  }
  GJState st{lane >= n, 0, 1.0, 0, false, false};
  gj_eliminate<NR>(a, st, n, lane, prow, piv);
  const bool sing = st.sing;
  const int pos = st.pos;
  const double logdet = log(st.mant) + st.expo * 0.69314718055994530942;
  const bool neg = st.neg;
  if (sing) {
    if (lane == 0) {
      c.logdet[w * 2 + sp] = -INFINITY;
      c.sgn[w * 2 + sp] = 0.0;
      c.flags[w] |= 2u;
    }
    return;
  }
  // GT[p_m][pos[r]] = register m of lane r; padding (columns and rows past n) zero
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    if (m >= n) continue;
    const int b = piv[m];
    const int col = lane < n ? pos : lane;
    const double val = lane < n ? a[m] : 0.0;
    if (lane < NP) {
      GT[(size_t)b * NP + col] = (T)val;
      if (G6) G6[(size_t)b * NP + col] = val;
    }
  }
  for (int b = n; b < NP; ++b)
    if (lane < NP) {
      GT[(size_t)b * NP + lane] = (T)0;
      if (G6) G6[(size_t)b * NP + lane] = 0.0;
    }
  if (lane == 0) {
    // parity of the pivot order k -> p_k from its cycles
    unsigned long long seen = 0ull;
    int cycles = 0;
    for (int i = 0; i < n; ++i) {
      if ((seen >> i) & 1ull) continue;
      ++cycles;
      for (int j = i; !((seen >> j) & 1ull); j = piv[j]) seen |= 1ull << j;
    }
    const bool odd = ((n - cycles) & 1) != 0;
    c.logdet[w * 2 + sp] = logdet;
    c.sgn[w * 2 + sp] = (neg != odd) ? -1.0 : 1.0;
  }
}

template <typename T, typename S, int NR>
void launch_inverse_nr(const DevCtx &c, const S *rows, int rs, double *G64, int periodic,
                       hipStream_t s) {
  const dim3 grid((2 * c.Wpad + INV_WAVES - 1) / INV_WAVES), block(64 * INV_WAVES);
  k_inverse_w<T, S, NR><<<grid, block, 0, s>>>(c, rows, rs, G64, periodic);
}

}  // namespace dmcx
