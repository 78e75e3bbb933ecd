// Per-walker finishing of the ion derivatives, walker VJPs and the force
// estimator (host-launched from the runtime only).
#pragma once
#include "forces.h"
#include "zv.h"

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

// Per walker and ion coordinate: the warped (warp != 0) or plain derivatives
//   dE_L   = 1/2 sum_tiles zpart + djv + dV + warp sum_i omega_a(r_i) (gjv_i - 1/2 zs_i)
//   dlnPsi = dl + warp sum_i omega_a(r_i) (c_i + g_i)
//   dlnJ   = warp sum_i d omega_a(r_i) / dr_i
// from dl = d ln|Psi|/dR and dV = dV/dR of the Eq. 3 pass.  Block 64 per walker.
__global__ void k_zv_finalize(DevCtx c, int warp, const double *zpart, const double *zs,
                              const double *cg, const double *gjv, const double *djv,
                              const double *dl, const double *dv, double *dEL, double *dLP,
                              double *dJ) {
  extern __shared__ double s_wf[];  // [ne][4]: sum_b F_b and its gradient
  const int w = blockIdx.x;
  const int ntile = (c.ne + FPTS - 1) / FPTS;
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  if (warp) {
    for (int i = threadIdx.x; i < c.ne; i += blockDim.x) {
      double S = 0.0, dS[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < c.n_atom; ++b) {
        const double d[3] = {Rw[3 * i] - c.ion[3 * b], Rw[3 * i + 1] - c.ion[3 * b + 1],
                             Rw[3 * i + 2] - c.ion[3 * b + 2]};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double F = 1.0 / (r2 * r2);
        S += F;
        for (int x = 0; x < 3; ++x) dS[x] -= 4.0 * F / r2 * d[x];
      }
      s_wf[4 * i] = S;
      for (int x = 0; x < 3; ++x) s_wf[4 * i + 1 + x] = dS[x];
    }
    __syncthreads();
  }
  for (int A = threadIdx.x; A < c.n_atom; A += blockDim.x) {
    double e[3], l[3], j[3] = {0.0, 0.0, 0.0};
    const size_t o = ((size_t)w * c.n_atom + A) * 3;
    for (int x = 0; x < 3; ++x) {
      double p = 0.0;
      for (int t = 0; t < ntile; ++t) p += zpart[((size_t)w * ntile + t) * c.n_atom * 3 + A * 3 + x];
      e[x] = 0.5 * p + djv[o + x] + dv[o + x];
      l[x] = dl[o + x];
    }
    if (warp) {
      for (int i = 0; i < c.ne; ++i) {
        const double d[3] = {Rw[3 * i] - c.ion[3 * A], Rw[3 * i + 1] - c.ion[3 * A + 1],
                             Rw[3 * i + 2] - c.ion[3 * A + 2]};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double F = 1.0 / (r2 * r2), S = s_wf[4 * i];
        const double om = F / S;
        const double *cgi = cg + ((size_t)w * c.ne + i) * 6;
        const double *gi = gjv + ((size_t)w * c.ne + i) * 3;
        const double *zi = zs + ((size_t)w * c.ne + i) * 3;
        for (int x = 0; x < 3; ++x) {
          e[x] += om * (gi[x] - 0.5 * zi[x]);
          l[x] += om * (cgi[x] + cgi[3 + x]);
          const double dF = -4.0 * F / r2 * d[x];
          j[x] += (dF * S - F * s_wf[4 * i + 1 + x]) / (S * S);
        }
      }
    }
    for (int x = 0; x < 3; ++x) {
      dEL[o + x] = e[x];
      dLP[o + x] = l[x];
      dJ[o + x] = j[x];
    }
  }
}

// Zero-variance force estimate, weights omega_w = exp(log w - max) (walkers
// with a status flag or a non-finite log w / E_L have weight zero):
//   F = -<dE_L> - (<E_L q> - <E_L><q>),  q = 2 dlnPsi + dlnJ.
// One block (256 threads) per component.
__global__ void k_zv_force_estimator(DevCtx c, const double *dEL, const double *dLP,
                                     const double *dJ, double *F) {
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
  double sw = 0.0, se = 0.0, sd = 0.0, sq = 0.0, seq = 0.0;
  for (int w = threadIdx.x; w < c.W; w += blockDim.x) {
    if (!est_walker_ok(c, w)) continue;
    const double om = exp(c.logw[w] - s_max), e = c.eloc[w];
    const size_t o = (size_t)w * ncomp + k;
    const double q = 2.0 * dLP[o] + dJ[o];
    sw += om;
    se += om * e;
    sd += om * dEL[o];
    sq += om * q;
    seq += om * e * q;
  }
  part[0][threadIdx.x] = sw; part[1][threadIdx.x] = se; part[2][threadIdx.x] = sd;
  part[3][threadIdx.x] = sq; part[4][threadIdx.x] = seq;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 5; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double W = part[0][0];
    const double E = part[1][0] / W, D = part[2][0] / W, Q = part[3][0] / W, EQ = part[4][0] / W;
    F[k] = -D - (EQ - E * Q);
  }
}

}  // namespace dmcx
