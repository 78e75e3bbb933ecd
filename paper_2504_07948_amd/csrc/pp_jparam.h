// Derivatives of the non-local pseudopotential energy with respect to the
// eight Jastrow-parameter directions (the e-e and e-n Pade b, six three-body
// coefficients at zero): the non-local part of dE_L/dp that the linear
// method needs when the trial function carries a pseudopotential.
//
// Each quadrature ratio Psi(R_q)/Psi(R) carries exp(J(R_q) - J(R)), so at
// fixed rotations
//   dV_NL/dp = sum_{e,A,q} (1/12) f_q rho_q (O_p(R_q) - O_p(R)),
// with O_p the parameter directions of J.  R_q moves electron e only, so
// the difference keeps the terms of e: sum_{j != e} dU_ee/db(r_ej),
// sum_A dU_en/db(r_eA) and sum_A sum_{j != e} (x^l y^m + x^m y^l) z^n with
// x = s(r_eA), y = s(r_jA), z = s(r_ej), s(r) = r / (1 + r).
#pragma once
#include "jparams.h"
#include "pp.h"

namespace dmcx {

// The terms of the eight directions that involve electron e placed at pos
// (the other electrons at s_r).  s_y: [ne][na] table of s(|r_j - R_A|), or
// null to compute it in place.
__device__ inline void pp_dir_terms(const DevCtx &c, const double *s_r, const double *s_y, int e,
                                    const double pos[3], double o[8]) {
  const int ne = c.ne, na = c.n_atom;
  const bool up = e < c.n_up;
  for (int k = 0; k < 8; ++k) o[k] = 0.0;
  double h, h1, h2;
  for (int j = 0; j < ne; ++j) {
    if (j == e) continue;
    const double dx = pos[0] - s_r[3 * j], dy = pos[1] - s_r[3 * j + 1], dz = pos[2] - s_r[3 * j + 2];
    pade_db(((j < c.n_up) == up) ? c.jee_para : c.jee_anti, c.jee_b,
            sqrt(dx * dx + dy * dy + dz * dz), h, h1, h2);
    o[0] += h;
  }
  for (int A = 0; A < na; ++A) {
    const double *RA = c.ion + 3 * A;
    const double dx = pos[0] - RA[0], dy = pos[1] - RA[1], dz = pos[2] - RA[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    pade_db(c.jen_a[A], c.jen_b, r, h, h1, h2);
    o[1] += h;
    const double x = r / (1.0 + r), x2 = x * x;
    for (int j = 0; j < ne; ++j) {
      if (j == e) continue;
      double y;
      if (s_y) {
        y = s_y[j * na + A];
      } else {
        const double ax = s_r[3 * j] - RA[0], ay = s_r[3 * j + 1] - RA[1], az = s_r[3 * j + 2] - RA[2];
        const double ry = sqrt(ax * ax + ay * ay + az * az);
        y = ry / (1.0 + ry);
      }
      const double bx = pos[0] - s_r[3 * j], by = pos[1] - s_r[3 * j + 1], bz = pos[2] - s_r[3 * j + 2];
      const double rz = sqrt(bx * bx + by * by + bz * bz);
      const double z = rz / (1.0 + rz);
      // (l, m, n) = (1,1,0), (1,0,1), (1,1,1), (2,1,0), (2,0,1), (1,0,2)
      const double xy = x * y, xpy = x + y;
      o[2] += 2.0 * xy;
      o[3] += xpy * z;
      o[4] += 2.0 * xy * z;
      o[5] += xy * xpy;
      o[6] += (x2 + y * y) * z;
      o[7] += xpy * z * z;
    }
  }
}

inline size_t pp_jp_lds_bytes(int ne, int n_nl, int na, bool tab) {
  const int cap = ne * (n_nl < PP_MAXA ? n_nl : PP_MAXA);
  return (size_t)ne * 13 * sizeof(double) + (size_t)((cap + 1) / 2) * sizeof(double) +
         (size_t)ne * 8 * sizeof(double) + (tab ? (size_t)ne * na * sizeof(double) : 0);
}

// grid W, block NT_AUX (>= ne), dynamic LDS pp_jp_lds_bytes(ne, n_nl, na, tab).
// Adds dV_NL/dp into D[w][8]; a walker whose pairs exceed the list gets NaN.
// Sums in a fixed order (per lane over its points, then the waves in order).
__global__ __launch_bounds__(NT_AUX) void k_pp_jparam(DevCtx c, const double *Y, int ldy, int tab,
                                                     double *D) {
  extern __shared__ double sm[];
  __shared__ int s_cnt[NT_AUX];
  __shared__ double red[NT_AUX / 64][8];
  const int ne = c.ne, na = c.n_atom, w = blockIdx.x, tid = threadIdx.x;
  const double *s_r = sm, *s_rot = sm + 3 * ne, *s_J = sm + 12 * ne;
  const int *s_pair = (const int *)(sm + 13 * ne);
  const int cap = ne * (c.pp_nl < PP_MAXA ? c.pp_nl : PP_MAXA);
  double *s_old = sm + 13 * ne + (cap + 1) / 2;  // [ne][8] each electron's terms where it is
  double *s_y = tab ? s_old + 8 * ne : nullptr;  // [ne][na]
  bool over;
  double e_unused;
  const int npair = pp_setup(c, w, sm, s_cnt, over, e_unused);
  if (s_y)
    for (int i = tid; i < ne * na; i += NT_AUX) {
      const int j = i / na, A = i - j * na;
      const double *RA = c.ion + 3 * A;
      const double ax = s_r[3 * j] - RA[0], ay = s_r[3 * j + 1] - RA[1], az = s_r[3 * j + 2] - RA[2];
      const double r = sqrt(ax * ax + ay * ay + az * az);
      s_y[i] = r / (1.0 + r);
    }
  __syncthreads();
  if (tid < ne && !over) {
    // electrons with listed pairs only (the others are not moved)
    const bool has = (tid == 0 ? s_cnt[0] : s_cnt[tid] - s_cnt[tid - 1]) > 0;
    if (has) pp_dir_terms(c, s_r, s_y, tid, s_r + 3 * tid, s_old + 8 * tid);
  }
  __syncthreads();
  double acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (!over) {
    for (int p = tid; p < npair * 12; p += NT_AUX) {
      const PPPoint P = pp_point(c, s_r, s_rot, s_pair[p / 12], p % 12);
      const double rdet = basis_dot(c.B, P.p, Y + ((size_t)w * ne + P.e) * ldy);
      const double ratio = rdet * exp(jastrow_at(c, s_r, P.e, P.p) - s_J[P.e]);
      double vl[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < c.pp_n; ++t) {
        const int4 tt = c.pp_t[t];
        if (tt.x == P.A && tt.y >= 0) vl[tt.y] += pp_term(tt.z, c.pp_ba[t].x, c.pp_ba[t].y, P.r);
      }
      double f = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) f += vl[l] * (2 * l + 1) * legendre_pl(l, P.cth);
      const double wt = f * ratio * (1.0 / 12.0);
      double o[8];
      pp_dir_terms(c, s_r, s_y, P.e, P.p, o);
      for (int k = 0; k < 8; ++k) acc[k] += wt * (o[k] - s_old[8 * P.e + k]);
    }
  }
  for (int k = 0; k < 8; ++k) {
    const double v = sum64(acc[k]);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid < 8) {
    double t = 0.0;
    for (int q = 0; q < NT_AUX / 64; ++q) t += red[q][tid];
    D[(size_t)w * 8 + tid] += over ? __builtin_nan("") : t;
  }
}

}  // namespace dmcx
