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

// The Pade directions' terms of electron e placed at pos (the other
// electrons at s_r): sum_{j != e} dU_ee/db and sum_A dU_en/db.
__device__ inline void pp_dir_pade(const DevCtx &c, const double *s_r, int e, const double pos[3],
                                   double &o0, double &o1) {
  const bool up = e < c.n_up;
  double h, h1, h2;
  o0 = o1 = 0.0;
  for (int j = 0; j < c.ne; ++j) {
    if (j == e) continue;
    const double dx = pos[0] - s_r[3 * j], dy = pos[1] - s_r[3 * j + 1], dz = pos[2] - s_r[3 * j + 2];
    pade_db(((j < c.n_up) == up) ? c.jee_para : c.jee_anti, c.jee_b,
            sqrt(dx * dx + dy * dy + dz * dz), h, h1, h2);
    o0 += h;
  }
  for (int A = 0; A < c.n_atom; ++A) {
    const double *RA = c.ion + 3 * A;
    const double dx = pos[0] - RA[0], dy = pos[1] - RA[1], dz = pos[2] - RA[2];
    pade_db(c.jen_a[A], c.jen_b, sqrt(dx * dx + dy * dy + dz * dz), h, h1, h2);
    o1 += h;
  }
}

// s(|r_j - R_A|) from the LDS table (atom-major, so the lanes of a wave, one
// per electron j, read consecutive entries), or computed in place without one.
__device__ __forceinline__ double pp_sy(const DevCtx &c, const double *s_r, const double *s_y,
                                        int j, int A) {
  if (s_y) return s_y[A * c.ne + j];
  const double *RA = c.ion + 3 * A;
  const double ax = s_r[3 * j] - RA[0], ay = s_r[3 * j + 1] - RA[1], az = s_r[3 * j + 2] - RA[2];
  const double r = sqrt(ax * ax + ay * ay + az * az);
  return r / (1.0 + r);
}

// The six three-body terms (l, m, n) = (1,1,0), (1,0,1), (1,1,1), (2,1,0),
// (2,0,1), (1,0,2) of one (x, y, z), added with weight wt.
__device__ __forceinline__ void pp_j3_add(double x, double y, double z, double wt, double a[6]) {
  const double xy = x * y, xpy = x + y, wz = wt * z;
  a[0] += wt * 2.0 * xy;
  a[1] += wz * xpy;
  a[2] += wz * 2.0 * xy;
  a[3] += wt * xy * xpy;
  a[4] += wz * (x * x + y * y);
  a[5] += wz * z * xpy;
}

constexpr int PPJ_CHUNK = 16;  // pairs per round (their 192 points, one per lane)

// Dynamic LDS: the set-up block (positions, rotations, J sums, pair list),
// each electron's own terms [ne][8], the round's points and weights
// [PPJ_CHUNK * 12][4], each wave's s(|p_q - R_A|) [12][na] and point sums
// [12][2], and the table s(|r_j - R_A|) [na][ne] when tab.
inline size_t pp_jp_lds_bytes(int ne, int n_nl, int na, bool tab) {
  const int cap = ne * (n_nl < PP_MAXA ? n_nl : PP_MAXA);
  return ((size_t)ne * 13 + (size_t)(cap + 1) / 2 + (size_t)ne * 8 + PPJ_CHUNK * 12 * 4 +
          (size_t)(NT_AUX / 64) * (12 * na + 24) + (tab ? (size_t)ne * na : 0)) * sizeof(double);
}

// grid W, block NT_AUX (>= ne), dynamic LDS pp_jp_lds_bytes(ne, n_nl, na, tab).
// Adds dV_NL/dp into D[w][8]; a walker whose pairs exceed the list gets NaN.
// Rounds of PPJ_CHUNK pairs: one lane per point forms its weight
// f rho / 12 (the quadrature ratio as k_pp) and the Pade directions' change;
// then each wave takes whole pairs, one lane per other electron j, and sums
// the three-body terms of the pair's 12 points over the atoms, factored into
// sums of one point, of one electron and three cross sums (the points' atom
// distances staged per wave in LDS).  Each electron's own three-body
// terms are formed once, a wave per electron and a lane per other electron.
// Sums in a fixed order (each lane
// over its terms, then the lanes of a wave, then the waves in order).
__global__ __launch_bounds__(NT_AUX) void k_pp_jparam(DevCtx c, const double *Y, int ldy, int tab,
                                                     double *D) {
  extern __shared__ double sm[];
  __shared__ int s_cnt[NT_AUX];
  __shared__ double red[NT_AUX / 64][8];
  const int ne = c.ne, na = c.n_atom, w = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const double *s_r = sm, *s_rot = sm + 3 * ne, *s_J = sm + 12 * ne;
  const int *s_pair = (const int *)(sm + 13 * ne);
  const int cap = ne * (c.pp_nl < PP_MAXA ? c.pp_nl : PP_MAXA);
  double *s_old = sm + 13 * ne + (cap + 1) / 2;  // [ne][8]: Pade (0, 1), three-body (2..7)
  double *s_pw = s_old + 8 * ne;                 // [PPJ_CHUNK * 12][4]: point, weight
  double *s_xa = s_pw + PPJ_CHUNK * 12 * 4;      // [waves][12 na + 24]
  double *s_y = tab ? s_xa + (NT_AUX / 64) * (12 * na + 24) : nullptr;  // [na][ne]
  bool over;
  double e_unused;
  const int npair = pp_setup(c, w, sm, s_cnt, over, e_unused);
  if (s_y)
    for (int i = tid; i < ne * na; i += NT_AUX) {
      const int A = i / ne, j = i - A * ne;
      const double *RA = c.ion + 3 * A;
      const double ax = s_r[3 * j] - RA[0], ay = s_r[3 * j + 1] - RA[1], az = s_r[3 * j + 2] - RA[2];
      const double r = sqrt(ax * ax + ay * ay + az * az);
      s_y[i] = r / (1.0 + r);
    }
  __syncthreads();
  double acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (!over) {
    // each electron's own terms where it is (electrons with listed pairs)
    if (tid < ne && (tid == 0 ? s_cnt[0] : s_cnt[tid] - s_cnt[tid - 1]) > 0)
      pp_dir_pade(c, s_r, tid, s_r + 3 * tid, s_old[8 * tid], s_old[8 * tid + 1]);
    for (int e = wv; e < ne; e += NT_AUX / 64) {
      if ((e == 0 ? s_cnt[0] : s_cnt[e] - s_cnt[e - 1]) == 0) continue;  // wave-uniform
      double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int j = lane; j < ne; j += 64) {
        if (j == e) continue;
        const double bx = s_r[3 * e] - s_r[3 * j], by = s_r[3 * e + 1] - s_r[3 * j + 1],
                     bz = s_r[3 * e + 2] - s_r[3 * j + 2];
        const double rz = sqrt(bx * bx + by * by + bz * bz), z = rz / (1.0 + rz);
        for (int A = 0; A < na; ++A)
          pp_j3_add(pp_sy(c, s_r, s_y, e, A), pp_sy(c, s_r, s_y, j, A), z, 1.0, a);
      }
      for (int k = 0; k < 6; ++k) {
        const double t = sum64(a[k]);
        if (lane == 0) s_old[8 * e + 2 + k] = t;
      }
    }
  }
  __syncthreads();
  if (!over) {
    for (int p0 = 0; p0 < npair; p0 += PPJ_CHUNK) {
      const int np = min(PPJ_CHUNK, npair - p0);
      // one lane per point: its weight, the Pade change, minus the
      // electron's own three-body terms times the weight
      if (tid < np * 12) {
        const PPPoint P = pp_point(c, s_r, s_rot, s_pair[p0 + tid / 12], tid % 12);
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
        double o0, o1;
        pp_dir_pade(c, s_r, P.e, P.p, o0, o1);
        acc[0] += wt * (o0 - s_old[8 * P.e]);
        acc[1] += wt * (o1 - s_old[8 * P.e + 1]);
        for (int k = 0; k < 6; ++k) acc[2 + k] -= wt * s_old[8 * P.e + 2 + k];
        for (int x = 0; x < 3; ++x) s_pw[4 * tid + x] = P.p[x];
        s_pw[4 * tid + 3] = wt;
      }
      __syncthreads();
      // one wave per pair, one lane per other electron.  Over the atoms the
      // six terms factor into sums of one point (S1_q = sum_A x, S2_q =
      // sum_A x^2), of one electron (Y1 = sum_A y, Y2 = sum_A y^2) and the
      // cross sums C^{ab}_q = sum_A x^a y^b, (a, b) = (1,1), (2,1), (1,2):
      //   2xy -> 2 C11, (x+y)z -> z (S1 + Y1), 2xyz -> 2 z C11,
      //   x^2 y + x y^2 -> C21 + C12, (x^2+y^2)z -> z (S2 + Y2),
      //   (x+y)z^2 -> z^2 (S1 + Y1).
      double *xa = s_xa + (size_t)wv * (12 * na + 24);
      double *s12 = xa + 12 * na;  // [12][2]: S1_q, S2_q
      for (int pl = wv; pl < np; pl += NT_AUX / 64) {
        const int e = s_pair[p0 + pl] & 0xffff;
        const double *pw = s_pw + 4 * 12 * pl;
        for (int i = lane; i < 12 * na; i += 64) {
          const int q = i / na, A = i - q * na;
          const double *RA = c.ion + 3 * A;
          const double dx = pw[4 * q] - RA[0], dy = pw[4 * q + 1] - RA[1], dz = pw[4 * q + 2] - RA[2];
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          xa[i] = r / (1.0 + r);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xC07F);  // this wave's LDS writes are visible to its lanes
        if (lane < 12) {
          double a1 = 0.0, a2 = 0.0;
          for (int A = 0; A < na; ++A) {
            const double x = xa[lane * na + A];
            a1 += x;
            a2 += x * x;
          }
          s12[2 * lane] = a1;
          s12[2 * lane + 1] = a2;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xC07F);
        for (int j = lane; j < ne; j += 64) {
          if (j == e) continue;
          double c11[12], c21[12], c12[12];
#pragma unroll
          for (int q = 0; q < 12; ++q) c11[q] = c21[q] = c12[q] = 0.0;
          double y1 = 0.0, y2 = 0.0;
          for (int A = 0; A < na; ++A) {
            const double y = pp_sy(c, s_r, s_y, j, A), yy = y * y;
            y1 += y;
            y2 += yy;
#pragma unroll
            for (int q = 0; q < 12; ++q) {
              const double x = xa[q * na + A], xy = x * y;
              c11[q] += xy;
              c21[q] += x * xy;
              c12[q] += x * yy;
            }
          }
#pragma unroll
          for (int q = 0; q < 12; ++q) {
            const double bx = pw[4 * q] - s_r[3 * j], by = pw[4 * q + 1] - s_r[3 * j + 1],
                         bz = pw[4 * q + 2] - s_r[3 * j + 2];
            const double rz = sqrt(bx * bx + by * by + bz * bz), z = rz / (1.0 + rz);
            const double wt = pw[4 * q + 3], wz = wt * z;
            const double sy1 = s12[2 * q] + y1, sy2 = s12[2 * q + 1] + y2;
            acc[2] += wt * 2.0 * c11[q];
            acc[3] += wz * sy1;
            acc[4] += wz * 2.0 * c11[q];
            acc[5] += wt * (c21[q] + c12[q]);
            acc[6] += wz * sy2;
            acc[7] += wz * z * sy1;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      __syncthreads();
    }
  }
  for (int k = 0; k < 8; ++k) {
    const double v = sum64(acc[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (tid < 8) {
    double t = 0.0;
    for (int q = 0; q < NT_AUX / 64; ++q) t += red[q][tid];
    D[(size_t)w * 8 + tid] += over ? __builtin_nan("") : t;
  }
}

}  // namespace dmcx
