// Per-walker finishing of the ion derivatives, walker VJPs and the force
// estimator (host-launched from the runtime only).
#pragma once
#include "forces.h"

namespace dmcx {

// Per walker: d ln|Psi| / dR_A = -(sum of tile partials) - sum_i u_A'(r_iA) (r_i - R_A)/r_iA,
// dV/dR_A = -Z_A sum_i (r_i - R_A)/r_iA^3 - sum_{B != A} Z_A Z_B (R_A - R_B)/R_AB^3.
// grid Wpad, block 64 (atoms over threads).
__global__ void k_ion_grad_finalize(DevCtx c, const double *partial, double *dlogpsi, double *dv) {
  const int w = blockIdx.x;
  const int ntile = (c.ne + FPTS - 1) / FPTS;
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  for (int A = threadIdx.x; A < c.n_atom; A += blockDim.x) {
    const double *RA = c.ion + 3 * A;
    double g[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < ntile; ++t)
      for (int x = 0; x < 3; ++x) g[x] -= partial[((size_t)w * ntile + t) * c.n_atom * 3 + A * 3 + x];
    for (int i = 0; i < c.ne; ++i) {
      const double d[3] = {Rw[3 * i] - RA[0], Rw[3 * i + 1] - RA[1], Rw[3 * i + 2] - RA[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const Pade pd = pade(c.jen_a[A], c.jen_b, r);
      const double fj = pd.d1 / r, fv = c.Z[A] / (r * r * r);
      for (int x = 0; x < 3; ++x) {
        g[x] -= fj * d[x];
        v[x] -= fv * d[x];
      }
    }
    for (int B = 0; B < c.n_atom; ++B) {
      if (B == A) continue;
      const double *RB = c.ion + 3 * B;
      const double d[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double f = c.Z[A] * c.Z[B] / (r * r * r);
      for (int x = 0; x < 3; ++x) v[x] -= f * d[x];
    }
    for (int x = 0; x < 3; ++x) {
      dlogpsi[((size_t)w * c.n_atom + A) * 3 + x] = g[x];
      dv[((size_t)w * c.n_atom + A) * 3 + x] = v[x];
    }
  }
}

// out[k] = sum_{w < W} gbar[w] d[w][k], k over n_atom*3 components; one
// block per component.
__global__ void k_walker_vjp(const double *d, const double *gbar, int W, int ncomp, double *out) {
  __shared__ double part[256];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int w = threadIdx.x; w < W; w += blockDim.x) s += gbar[w] * d[(size_t)w * ncomp + k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = part[0];
}

// Force estimate with weights omega_w = exp(log w_w - max log w):
//   F = -<dV> - 2 (<E_L dlnPsi> - <E_L><dlnPsi>),  <x> = sum omega x / sum omega.
// A walker with a status flag, or a non-finite log-weight or E_L, has weight
// zero (as in the comb of population control); with no such walker left the
// result is NaN.  One block (256 threads) per component.
__device__ __forceinline__ bool est_walker_ok(const DevCtx &c, int w) {
  return c.flags[w] == 0u && isfinite(c.logw[w]) && isfinite(c.eloc[w]);
}
__global__ void k_force_estimator(DevCtx c, const double *dl, const double *dv, double *F) {
  __shared__ double part[5][256];
  __shared__ double s_max;
  const int k = blockIdx.x, ncomp = c.n_atom * 3;
  double m = -INFINITY;
  for (int w = threadIdx.x; w < c.W; w += blockDim.x)
    if (est_walker_ok(c, w)) m = fmax(m, c.logw[w]);
  part[0][threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[0][threadIdx.x] = fmax(part[0][threadIdx.x], part[0][threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) s_max = part[0][0];
  __syncthreads();
  double sw = 0.0, se = 0.0, sd = 0.0, sed = 0.0, sv = 0.0;
  for (int w = threadIdx.x; w < c.W; w += blockDim.x) {
    if (!est_walker_ok(c, w)) continue;
    const double om = exp(c.logw[w] - s_max), e = c.eloc[w];
    const double d = dl[(size_t)w * ncomp + k];
    sw += om;
    se += om * e;
    sd += om * d;
    sed += om * e * d;
    sv += om * dv[(size_t)w * ncomp + k];
  }
  part[0][threadIdx.x] = sw; part[1][threadIdx.x] = se; part[2][threadIdx.x] = sd;
  part[3][threadIdx.x] = sed; part[4][threadIdx.x] = sv;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 5; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double W = part[0][0];
    const double E = part[1][0] / W, D = part[2][0] / W, ED = part[3][0] / W, V = part[4][0] / W;
    F[k] = -V - 2.0 * (ED - E * D);
  }
}

}  // namespace dmcx
