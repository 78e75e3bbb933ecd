// Multideterminant expansion (Eq. 2 with M > 1) by the table method: the
// table T = A^{-1} M and the excited-determinant ratios rebuilt from
// scratch (at walker set-up and at every FP64 inverse recompute).
#pragma once
#include "kernels.h"

namespace dmcx {

// T[j][v] = sum_i (A^{-1})_{j i} M_{i v} = sum_i GT[i][j] phi_{vcol[v]}(r_i)
// for occupied j < n_sigma and virtual v < nv.  grid (Wpad, 2).
// periodic != 0: only at steps s = 0 (mod P) of the device step counter.
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_msd_table(DevCtx c, int periodic) {
  if (periodic && (c.run->step % (unsigned long long)c.P) != 0ull) return;
  const int w = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? c.n_up : c.n_dn, e0 = sp == 0 ? 0 : c.n_up;
  const int NP = c.NP, nv = c.M.nv, ldt = c.M.ldt;
  const T *GT = (const T *)c.GT + gt_off(c, w, sp);
  T *Tw = (T *)c.M.Tt + ((size_t)w * 2 + sp) * NP * ldt;
  for (int idx = threadIdx.x; idx < n * nv; idx += NT_AUX) {
    const int j = idx / nv, v = idx - j * nv;
    const int cv = c.M.vcol[v];
    double s = 0.0;
    for (int i = 0; i < n; ++i)
      s += (double)GT[(size_t)i * NP + j] * (double)((const T *)c.vglc)[vglc_off(c, w, e0 + i) + cv];
    Tw[(size_t)j * ldt + v] = (T)s;
  }
}

// R_d^s for every determinant and spin from the table, and
// S = sum_d c_d R_d^up R_d^dn.  grid Wpad, block NT_AUX.
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_msd_dets(DevCtx c, int periodic) {
  if (periodic && (c.run->step % (unsigned long long)c.P) != 0ull) return;
  __shared__ double part[NT_AUX / 64];
  const int w = blockIdx.x, tid = threadIdx.x;
  const DevMsd &M = c.M;
  double s = 0.0;
  for (int d = tid; d < M.n_det; d += NT_AUX) {
    double r[2];
    for (int sp = 0; sp < 2; ++sp) {
      const T *Tw = (const T *)M.Tt + ((size_t)w * 2 + sp) * c.NP * M.ldt;
      const int4 e = M.dexc[2 * d + sp];
      const int n = e.x, h0 = e.y & 0xffff, h1 = (unsigned)e.y >> 16, v0 = e.z & 0xffff,
                v1 = (unsigned)e.z >> 16;
      if (n == 0) {
        r[sp] = 1.0;
      } else if (n == 1) {
        r[sp] = (double)Tw[(size_t)h0 * M.ldt + v0];
      } else {
        r[sp] = (double)Tw[(size_t)h0 * M.ldt + v0] * (double)Tw[(size_t)h1 * M.ldt + v1] -
                (double)Tw[(size_t)h0 * M.ldt + v1] * (double)Tw[(size_t)h1 * M.ldt + v0];
      }
      M.Rdet[((size_t)w * 2 + sp) * M.n_det + d] = r[sp];
    }
    s += M.coef[d] * r[0] * r[1];
  }
  s = sum64(s);
  if ((tid & 63) == 0) part[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double S = 0.0;
    for (int q = 0; q < NT_AUX / 64; ++q) S += part[q];
    M.S[w] = S;
    if (!(S != 0.0) || !isfinite(S)) c.flags[w] |= 1u;
  }
}

// Orbital-space weights of the ion-force adjoint with the expansion.  With
// S = sum_d c_d R_d^up R_d^dn and dT = A^{-1} (dM - dA T) for a change of
// the orbitals,
//   d ln S = sum_i [ sum_v X_iv dM_iv - sum_j Y_ij dA_ij ],
//   Gamma_hv = d ln S / dT_hv = sum_d c_d R_d^other dR_d/dT_hv / S,
//   X = A^{-T} Gamma (X_iv = sum_h G_hi Gamma_hv),  Y = X T^T,
// so the reference determinant's weights g_i (row i of GT) become
//   W[i][j] = g_i[j] - Y_ij (occupied j),  W[i][vcol[v]] = X_iv,
// and the same contraction with the basis gradients (forces.h) gives
// d ln|D_0 S| / dR.  grid (Wpad, 2), dynamic LDS 2 n_sigma nv doubles.
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_msd_force_weights(DevCtx c, T *WT) {
  extern __shared__ double gx[];  // Gamma [n][nv], then X [n][nv]
  const int w = blockIdx.x, sp = blockIdx.y, tid = threadIdx.x;
  const DevMsd &M = c.M;
  const int n = sp == 0 ? c.n_up : c.n_dn, NP = c.NP, nv = M.nv, ldt = M.ldt;
  double *Gam = gx, *X = gx + (size_t)n * nv;
  const T *GT = (const T *)c.GT + gt_off(c, w, sp);
  const T *Tw = (const T *)M.Tt + ((size_t)w * 2 + sp) * NP * ldt;
  const double *Ro = M.Rdet + ((size_t)w * 2 + (1 - sp)) * M.n_det;
  T *Wo = WT + gt_off(c, w, sp);
  const double iS = 1.0 / M.S[w];
  // each entry sums its own contributions in determinant order (no atomics,
  // so the result does not depend on how the threads were scheduled)
  const int *gptr = M.gptr[sp];
  const int4 *gcon = M.gcon[sp];
  for (int q = tid; q < n * nv; q += NT_AUX) {
    double g = 0.0;
    for (int k = gptr[q]; k < gptr[q + 1]; ++k) {
      const int4 e = gcon[k];
      const double cr = M.lcoef[sp][e.x] * Ro[M.lst[sp][e.x].x];
      const double f = e.y < 0 ? 1.0 : (double)Tw[(size_t)e.y * ldt + e.z];
      g += (double)e.w * cr * f;
    }
    Gam[q] = g * iS;
  }
  __syncthreads();
  for (int q = tid; q < n * nv; q += NT_AUX) {
    const int i = q / nv, v = q - i * nv;
    double x = 0.0;
    for (int h = 0; h < n; ++h) x += (double)GT[(size_t)i * NP + h] * Gam[h * nv + v];
    X[q] = x;
  }
  __syncthreads();
  for (int q = tid; q < NP * NP; q += NT_AUX) {
    const int i = q / NP, j = q - i * NP;
    double wv = 0.0;
    if (i < n && j < n) {
      wv = (double)GT[(size_t)i * NP + j];
      for (int v = 0; v < nv; ++v) wv -= X[i * nv + v] * (double)Tw[(size_t)j * ldt + v];
    }
    Wo[q] = (T)wv;
  }
  __syncthreads();
  for (int q = tid; q < n * nv; q += NT_AUX) {
    const int i = q / nv, v = q - i * nv;
    Wo[(size_t)i * NP + M.vcol[v]] = (T)X[q];
  }
}

template <typename T>
struct MsdLaunch {
  static void sweep(int nob, const DevCtx &c, uint8_t *acc, long long acc_ss, int acc_ws,
                    size_t lds, hipStream_t s);
  static size_t sweep_lds(int nob);
  static void sweep_multi(int nob, const DevCtx *cs, const int2 *tiles, int ntiles,
                          const SweepLog *logs, size_t lds, hipStream_t s);
};

}  // namespace dmcx
