// Residual of the stored inverses (a diagnostic of the delayed updates and
// of the periodic FP64 recompute): for walker w and spin s,
//   r = max_ij |sum_k A_ik (A^{-1})_kj - delta_ij|
// over the spin's n x n Slater matrix A_ik = phi_k(r_i) (the cached value
// rows of the current positions) and the stored inverse (GT row j holds
// column j of A^{-1}, so the sum is a dot product of two contiguous rows),
// products and sums in FP64 whatever the working precision.  A NaN anywhere
// gives NaN; an empty spin gives 0.
#pragma once
#include "kernels.h"

namespace dmcx {

template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_inv_residual(DevCtx c, double *res) {
  __shared__ double s_max[NT_AUX / 64];
  __shared__ int s_nan[NT_AUX / 64];
  const int w = blockIdx.x, sp = blockIdx.y, tid = threadIdx.x;
  const int n = sp == 0 ? c.n_up : c.n_dn, e0 = sp == 0 ? 0 : c.n_up;
  const T *GT = (const T *)c.GT + gt_off(c, w, sp);
  double m = 0.0;
  int bad = 0;
  for (int q = tid; q < n * n; q += NT_AUX) {
    const int i = q / n, j = q - i * n;
    const T *a = (const T *)c.vglc + vglc_off(c, w, e0 + i);
    const T *g = GT + (size_t)j * c.NP;
    double s0 = 0.0, s1 = 0.0;
    int k = 0;
    for (; k + 1 < n; k += 2) {
      s0 += (double)a[k] * (double)g[k];
      s1 += (double)a[k + 1] * (double)g[k + 1];
    }
    if (k < n) s0 += (double)a[k] * (double)g[k];
    const double d = fabs(s0 + s1 - (i == j ? 1.0 : 0.0));
    bad |= isnan(d) ? 1 : 0;
    m = fmax(m, d);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if ((tid & 63) == 0) {
    s_max[tid >> 6] = m;
    s_nan[tid >> 6] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    int b = 0;
    for (int i = 0; i < NT_AUX / 64; ++i) {
      r = fmax(r, s_max[i]);
      b |= s_nan[i];
    }
    res[2 * w + sp] = b ? __builtin_nan("") : r;
  }
}

}  // namespace dmcx
