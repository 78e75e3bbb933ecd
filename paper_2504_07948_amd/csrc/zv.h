// Zero-variance force terms (Single Determinant QMC Forces, Eq. 4) and the
// space-warp transformation, by a hand-written reverse-mode adjoint.
//
// With B the one-body operator matrix of a spin (electron row i, orbital j),
//   B_ij = lap phi_j(r_i) + 2 grad_i J . grad phi_j(r_i),
// the local energy is E_L = -1/2 sum_spin tr(A^{-1} B)
// - 1/2 sum_i [lap_i J + |grad_i J|^2] + V, and along any direction lambda of
// the ions and electrons Eq. 4 gives d tr(A^{-1} B) = tr(A^{-1} dB - X dA),
// X = A^{-1} B A^{-1}.  Contracting the orbital index first, the determinant
// part of dE_L is a weighted sum over basis functions l and electrons i of
//   q_i^x(l) = y1_i[l] (d_x lap Phi_l + 2 sum_y (d_y J)_i d_x d_y Phi_l)
//              - y2_i[l] d_x Phi_l,
//   y1_i = C g_i (g_i = column i of A^{-1}),  y2_i = C x_i (x_i = column i of X),
// evaluated at r_i: moving ion a by e_x moves the functions of atom a, so
// d_{a,x} E_L(det) = +1/2 sum_i sum_{l on a} q_i^x(l); moving electron i by
// e_x gives d_{i,x} E_L(det) = -1/2 sum_l q_i^x(l).  The Jastrow part (with
// the determinant's g_i held fixed) and V are differentiated pair by pair.
//
// Space warp (Filippi and Umrigar): moving ion a by dR also moves every
// electron by omega_a(r_i) dR, omega_a(r) = F(|r - R_a|) / sum_b F(|r - R_b|),
// F(d) = d^-4; the warped derivative is d_a + sum_i omega_a(r_i) d_i and the
// sampled density gains the Jacobian, d ln J / dR_{a,x} = sum_i d omega_a(r_i)/dr_{i,x}.
#pragma once
#include "forces.h"

namespace dmcx {

// Per walker: Jastrow gradient c_i and determinant drift g_i of every
// electron (cg [Wpad][ne][6]); the electron gradient of the Jastrow part of
// E_L plus V, with g held fixed (gjv [Wpad][ne][3]); and its direct ion
// derivative without V (djv [Wpad][n_atom][3]).  One workgroup per walker.
//   E_J = -1/2 sum_i [lap_i J + |c_i|^2 + 2 c_i . g_i]
//   d E_J / d r_k = -H_k (c_k + g_k) + sum_{i != k} H(r_k - r_i)(c_i + g_i)
//                   - 1/2 sum_q glap(r_k - x_q) - 1/2 sum_{i != k} glap(r_k - r_i)
// (H = Hessian, glap = gradient of the Laplacian of one Pade pair term, H_k
// the sum of H over all partners q of electron k), and for an ion a
//   d E_J / d R_a = sum_i [H_a(r_i - R_a)(c_i + g_i) + 1/2 glap_a(r_i - R_a)].
struct PadeD {
  double g[3], H[6], glap[3];  // H: xx, xy, xz, yy, yz, zz
};
__device__ __forceinline__ PadeD pade_d3(double a, double b, const double d[3]) {
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double r = sqrt(r2), ir = 1.0 / r;
  const double q = 1.0 / (1.0 + b * r);
  const double u1 = a * q * q, u2 = -2.0 * a * b * q * q * q, u3 = 6.0 * a * b * b * q * q * q * q;
  const double n[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  const double t = u1 * ir, gl = u3 + 2.0 * u2 * ir - 2.0 * u1 * ir * ir;
  PadeD p;
  const int hx[6] = {0, 0, 0, 1, 1, 2}, hy[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    p.g[x] = u1 * n[x];
    p.glap[x] = gl * n[x];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k)
    p.H[k] = (u2 - t) * n[hx[k]] * n[hy[k]] + (hx[k] == hy[k] ? t : 0.0);
  return p;
}
__device__ __forceinline__ void hmul(const double H[6], const double v[3], double o[3]) {
  o[0] = H[0] * v[0] + H[1] * v[1] + H[2] * v[2];
  o[1] = H[1] * v[0] + H[3] * v[1] + H[4] * v[2];
  o[2] = H[2] * v[0] + H[4] * v[1] + H[5] * v[2];
}

// Jastrow gradient c_i and determinant drift g_i = sum_j grad phi_j(r_i)
// (A^{-1})_{ji} of electron i of walker w, computed by the calling 64-lane
// wave; every lane receives o = (c_i, g_i).
template <typename T>
__device__ __forceinline__ void electron_cg(const DevCtx &c, const double *Rw, int w, int i,
                                            int lane, double o[6]) {
  const int NP = c.NP;
  const int sp = i < c.n_up ? 0 : 1, ii = i - sp * c.n_up;
  const T *row = (const T *)c.vglc + vglc_off(c, w, i);
  const T *gcol = (const T *)c.GT + gt_off(c, w, sp) + (size_t)ii * NP;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int j = lane; j < NP; j += 64) {
    const double gj = (double)gcol[j];
    g0 += (double)row[NP + j] * gj;
    g1 += (double)row[2 * NP + j] * gj;
    g2 += (double)row[3 * NP + j] * gj;
  }
  double u = 0.0, cj[3] = {0.0, 0.0, 0.0};
  const double ri[3] = {Rw[3 * i], Rw[3 * i + 1], Rw[3 * i + 2]};
  jastrow_one_partial(c, Rw, i, ri, lane, 64, u, cj);
  o[3] = sum64(g0); o[4] = sum64(g1); o[5] = sum64(g2);
  o[0] = sum64(cj[0]); o[1] = sum64(cj[1]); o[2] = sum64(cj[2]);
}

template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_zv_prep(DevCtx c, double *cg, double *gjv,
                                                   double *djv) {
  extern __shared__ double s_cg[];  // [ne][6]: c_i, g_i
  const int w = blockIdx.x;
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  constexpr int NWV = NT_AUX / 64;
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  // c_i and g_i, one wave per electron
  for (int i = wid; i < c.ne; i += NWV) {
    double o[6];
    electron_cg<T>(c, Rw, w, i, lane, o);
    if (lane == 0) {
      double *go = cg + ((size_t)w * c.ne + i) * 6;
      for (int q = 0; q < 6; ++q) {
        s_cg[6 * i + q] = o[q];
        go[q] = o[q];
      }
    }
  }
  __syncthreads();
  // electron gradient of E_J + V, one wave per electron k
  for (int k = wid; k < c.ne; k += NWV) {
    const int sk = k < c.n_up ? 0 : 1;
    const double rk[3] = {Rw[3 * k], Rw[3 * k + 1], Rw[3 * k + 2]};
    const double vk[3] = {s_cg[6 * k] + s_cg[6 * k + 3], s_cg[6 * k + 1] + s_cg[6 * k + 4],
                          s_cg[6 * k + 2] + s_cg[6 * k + 5]};
    double Hk[6] = {0, 0, 0, 0, 0, 0}, acc[3] = {0.0, 0.0, 0.0};
    for (int q = lane; q < c.ne + c.n_atom; q += 64) {
      if (q == k) continue;
      double d[3], a, b;
      const bool el = q < c.ne;
      if (el) {
        for (int x = 0; x < 3; ++x) d[x] = rk[x] - Rw[3 * q + x];
        a = ((q < c.n_up ? 0 : 1) == sk) ? c.jee_para : c.jee_anti;
        b = c.jee_b;
      } else {
        const int A = q - c.ne;
        for (int x = 0; x < 3; ++x) d[x] = rk[x] - c.ion[3 * A + x];
        a = c.jen_a[A];
        b = c.jen_b;
      }
      const PadeD p = pade_d3(a, b, d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double ir3 = 1.0 / (r2 * sqrt(r2));
      for (int m = 0; m < 6; ++m) Hk[m] += p.H[m];
      for (int x = 0; x < 3; ++x) acc[x] -= 0.5 * p.glap[x];
      if (el) {
        const double vi[3] = {s_cg[6 * q] + s_cg[6 * q + 3], s_cg[6 * q + 1] + s_cg[6 * q + 4],
                              s_cg[6 * q + 2] + s_cg[6 * q + 5]};
        double hv[3];
        hmul(p.H, vi, hv);
        for (int x = 0; x < 3; ++x) acc[x] += hv[x] - 0.5 * p.glap[x] - d[x] * ir3;
      } else {
        const double Z = c.Z[q - c.ne];
        for (int x = 0; x < 3; ++x) acc[x] += Z * d[x] * ir3;
      }
    }
    double hv[3];
    hmul(Hk, vk, hv);
    for (int x = 0; x < 3; ++x) acc[x] -= hv[x];
    acc[0] = sum64(acc[0]); acc[1] = sum64(acc[1]); acc[2] = sum64(acc[2]);
    if (lane == 0)
      for (int x = 0; x < 3; ++x) gjv[((size_t)w * c.ne + k) * 3 + x] = acc[x];
  }
  // direct ion derivative of E_J, one wave per atom
  for (int A = wid; A < c.n_atom; A += NWV) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = lane; i < c.ne; i += 64) {
      const double d[3] = {Rw[3 * i] - c.ion[3 * A], Rw[3 * i + 1] - c.ion[3 * A + 1],
                           Rw[3 * i + 2] - c.ion[3 * A + 2]};
      const PadeD p = pade_d3(c.jen_a[A], c.jen_b, d);
      const double vi[3] = {s_cg[6 * i] + s_cg[6 * i + 3], s_cg[6 * i + 1] + s_cg[6 * i + 4],
                            s_cg[6 * i + 2] + s_cg[6 * i + 5]};
      double hv[3];
      hmul(p.H, vi, hv);
      for (int x = 0; x < 3; ++x) acc[x] += hv[x] + 0.5 * p.glap[x];
    }
    acc[0] = sum64(acc[0]); acc[1] = sum64(acc[1]); acc[2] = sum64(acc[2]);
    if (lane == 0)
      for (int x = 0; x < 3; ++x) djv[((size_t)w * c.n_atom + A) * 3 + x] = acc[x];
  }
}

// X^T = G^T B^T G^T per walker and spin (rows b of the result are the columns
// of X = A^{-1} B A^{-1}, laid out like GT), with B_ij = lap phi_j(r_i) +
// 2 c_i . grad phi_j(r_i).  Two MFMA GEMMs over NP x NP tiles:
//   T'[b][i] = sum_j GT[b][j] B[i][j],   XT[b][j] = sum_i T'[b][i] GT[i][j].
// grid (Wpad, 2), block NT_AUX; scratch tp [Wpad][2][NP][NP] (working precision).
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_zv_x(DevCtx c, const double *cg, T *tp, T *xt) {
  const int w = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? c.n_up : c.n_dn, e0 = sp == 0 ? 0 : c.n_up;
  const int NP = c.NP, nob = NP / 16;
  const int wid = wave_id(), lane = threadIdx.x & 63, kq = lane >> 4, cl = lane & 15;
  const T *GT = (const T *)c.GT + gt_off(c, w, sp);
  T *Tp = tp + gt_off(c, w, sp);
  T *XT = xt + gt_off(c, w, sp);
  const double *cgw = cg + (size_t)w * c.ne * 6;
  for (int tt = wid; tt < nob * nob; tt += NT_AUX / 64) {
    const int b0 = (tt / nob) * 16, i0 = (tt % nob) * 16;
    const auto acc = mfma_tile<T>(
        NP, [&](int r, int k) { return GT[(size_t)(b0 + r) * NP + k]; },
        [&](int k, int col) {
          const int i = i0 + col;
          if (i >= n) return (T)0;
          const T *row = (const T *)c.vglc + vglc_off(c, w, e0 + i);
          const double *ci = cgw + (size_t)(e0 + i) * 6;
          return (T)((double)row[4 * NP + k] +
                     2.0 * (ci[0] * (double)row[NP + k] + ci[1] * (double)row[2 * NP + k] +
                            ci[2] * (double)row[3 * NP + k]));
        });
#pragma unroll
    for (int r = 0; r < 4; ++r) Tp[(size_t)(b0 + Acc4<T>::row(kq, r)) * NP + i0 + cl] = acc[r];
  }
  __syncthreads();
  for (int tt = wid; tt < nob * nob; tt += NT_AUX / 64) {
    const int b0 = (tt / nob) * 16, j0 = (tt % nob) * 16;
    const auto acc = mfma_tile<T>(
        NP, [&](int r, int k) { return Tp[(size_t)(b0 + r) * NP + k]; },
        [&](int k, int col) { return GT[(size_t)k * NP + j0 + col]; });
#pragma unroll
    for (int r = 0; r < 4; ++r) XT[(size_t)(b0 + Acc4<T>::row(kq, r)) * NP + j0 + cl] = acc[r];
  }
}

// Cartesian polynomial P of component COMP of angular momentum L with its
// gradient, Hessian (xx, xy, xz, yy, yz, zz; constants for L <= 2) and
// Laplacian.
template <int L, int COMP, typename R>
__device__ __forceinline__ void cart_poly_h(R x, R y, R z, R &P, R (&Pg)[3], R (&Ph)[6], R &Lp) {
  R Px, Py, Pz;
  cart_poly_t<L, COMP, R>(x, y, z, P, Px, Py, Pz, Lp);
  Pg[0] = Px; Pg[1] = Py; Pg[2] = Pz;
#pragma unroll
  for (int k = 0; k < 6; ++k) Ph[k] = 0;
  if constexpr (L == 2) {
    if constexpr (COMP == 0) Ph[0] = 2;
    else if constexpr (COMP == 1) Ph[1] = 1;
    else if constexpr (COMP == 2) Ph[2] = 1;
    else if constexpr (COMP == 3) Ph[3] = 2;
    else if constexpr (COMP == 4) Ph[4] = 1;
    else Ph[5] = 2;
  }
}

// One stage of the determinant adjoint: for the tile's points n (lane % 32)
// and the stage's shells, q_n^x = sum over the shell's functions of
//   y1 (d_x lap Phi + 2 c_n . H_x Phi) - y2 d_x Phi,
// reduced over the 32 points into the shell's slot total (slot, satom;
// binned by atom with bin_slots after a barrier) and accumulated per point in
// the thread's own registers (sacc: each thread serves one point), so no sum
// depends on how the waves were scheduled.  Radial part R(s^2) with derivatives R1..R3:
//   d_a Phi = P_a R + 2 d_a P R1,
//   d_ab Phi = P_ab R + 2 (P_a d_b + P_b d_a) R1 + 2 delta_ab P R1 + 4 d_a d_b P R2,
//   d_c lap Phi = 2 lapP d_c R1 + 4 R1 (H_P d)_c + 4 P_c R1 + 8 d_c R2 (grad P . d)
//                 + P_c (6 R1 + 4 s2 R2) + P d_c (20 R2 + 8 s2 R3).
template <typename T, int L, int NPR>
__device__ void zv_stage_t(const BasisLDS &B, const int *gatom, int g_begin, int g_end,
                           int fn_begin, const double (*pts)[3], const double (*cj)[3], int npts,
                           const T *Ys, double *slot, int *satom, double (&sacc)[3],
                           int npr_rt = NPR) {
  constexpr int NC = L == 0 ? 1 : (L == 1 ? 3 : 6);
  const int nsh = 4 * (g_end - g_begin);
  const int tid = threadIdx.x;
  const int n = tid & 31;
  for (int sl = tid >> 5; sl < nsh; sl += NT_FORCE / 32) {
    const int g = g_begin + (sl >> 2), s = sl & 3;
    const int4 gi = B.ginfo[g];
    double f[3] = {0.0, 0.0, 0.0};
    if (n < npts) {
      const double *cxyz = B.xyz + (size_t)(g * 4 + s) * 3;
      const T d[3] = {(T)(pts[n][0] - cxyz[0]), (T)(pts[n][1] - cxyz[1]), (T)(pts[n][2] - cxyz[2])};
      const T s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      T R0 = 0, R1 = 0, R2 = 0, R3 = 0;
      if constexpr (NPR > 0) {
        T e[NPR], a[NPR];
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
          a[p] = (T)B.alpha[gi.w + p * 4 + s];
          e[p] = (T)B.coef[gi.w + p * 4 + s] * texp(-a[p] * s2);
        }
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
          R0 += e[p];
          R1 -= a[p] * e[p];
          R2 += a[p] * a[p] * e[p];
          R3 -= a[p] * a[p] * a[p] * e[p];
        }
      } else {
        for (int p = 0; p < npr_rt; ++p) {
          const T ap = (T)B.alpha[gi.w + p * 4 + s];
          const T ep = (T)B.coef[gi.w + p * 4 + s] * texp(-ap * s2);
          R0 += ep;
          R1 -= ap * ep;
          R2 += ap * ap * ep;
          R3 -= ap * ap * ap * ep;
        }
      }
      const T cjn[3] = {(T)cj[n][0], (T)cj[n][1], (T)cj[n][2]};
      const T *yrow = Ys + (size_t)(gi.z - fn_begin + s) * (2 * FPTS) + n;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        T P, Pg[3], Ph[6], Lp;
        switch (cc) {  // resolved at compile time after unrolling
          case 0: cart_poly_h<L, 0, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
          case 1: cart_poly_h<L, 1, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
          case 2: cart_poly_h<L, 2, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
          case 3: cart_poly_h<L, 3, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
          case 4: cart_poly_h<L, 4, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
          default: cart_poly_h<L, 5, T>(d[0], d[1], d[2], P, Pg, Ph, Lp); break;
        }
        const T pd = Pg[0] * d[0] + Pg[1] * d[1] + Pg[2] * d[2];
        T Hd[3];
        Hd[0] = Ph[0] * d[0] + Ph[1] * d[1] + Ph[2] * d[2];
        Hd[1] = Ph[1] * d[0] + Ph[3] * d[1] + Ph[4] * d[2];
        Hd[2] = Ph[2] * d[0] + Ph[4] * d[1] + Ph[5] * d[2];
        T gr[3], hs[6], gl[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          gr[x] = Pg[x] * R0 + (T)2 * d[x] * P * R1;
          gl[x] = (T)2 * Lp * d[x] * R1 + (T)4 * R1 * Hd[x] + (T)4 * Pg[x] * R1 +
                  (T)8 * d[x] * R2 * pd + Pg[x] * ((T)6 * R1 + (T)4 * s2 * R2) +
                  P * d[x] * ((T)20 * R2 + (T)8 * s2 * R3);
        }
        const int hx[6] = {0, 0, 0, 1, 1, 2}, hy[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const int a = hx[k], b = hy[k];
          hs[k] = Ph[k] * R0 + (T)2 * (Pg[a] * d[b] + Pg[b] * d[a]) * R1 +
                  (a == b ? (T)2 * P * R1 : (T)0) + (T)4 * d[a] * d[b] * P * R2;
        }
        const double y1 = (double)yrow[(size_t)cc * 4 * (2 * FPTS)];
        const double y2 = (double)yrow[(size_t)cc * 4 * (2 * FPTS) + FPTS];
        T hc[3];  // H c
        hc[0] = hs[0] * cjn[0] + hs[1] * cjn[1] + hs[2] * cjn[2];
        hc[1] = hs[1] * cjn[0] + hs[3] * cjn[1] + hs[4] * cjn[2];
        hc[2] = hs[2] * cjn[0] + hs[4] * cjn[1] + hs[5] * cjn[2];
#pragma unroll
        for (int x = 0; x < 3; ++x)
          f[x] += y1 * (double)(gl[x] + (T)2 * hc[x]) - y2 * (double)gr[x];
      }
      sacc[0] += f[0];
      sacc[1] += f[1];
      sacc[2] += f[2];
    }
    f[0] = sum32(f[0]);
    f[1] = sum32(f[1]);
    f[2] = sum32(f[2]);
    if (n == 0) {
      slot[sl * 3 + 0] = f[0];
      slot[sl * 3 + 1] = f[1];
      slot[sl * 3 + 2] = f[2];
      satom[sl] = gatom[g * 4 + s];
    }
  }
}

template <typename T>
__device__ inline void zv_stage(const BasisLDS &B, const int *gatom, int g_begin, int g_end,
                                int fn_begin, const double (*pts)[3], const double (*cj)[3],
                                int npts, const T *Ys, double *slot, int *satom,
                                double (&sacc)[3]) {
  const int4 gi = B.ginfo[g_begin];
#define DMCX_ZV_CASE(LL, NN)                                                                 \
  case LL * 16 + NN:                                                                         \
    zv_stage_t<T, LL, NN>(B, gatom, g_begin, g_end, fn_begin, pts, cj, npts, Ys, slot, satom, sacc); \
    break;
  switch (gi.x * 16 + (gi.y <= 4 ? gi.y : 0)) {
    DMCX_ZV_CASE(0, 1) DMCX_ZV_CASE(0, 2) DMCX_ZV_CASE(0, 3) DMCX_ZV_CASE(0, 4)
    DMCX_ZV_CASE(1, 1) DMCX_ZV_CASE(1, 2) DMCX_ZV_CASE(1, 3) DMCX_ZV_CASE(1, 4)
    DMCX_ZV_CASE(2, 1) DMCX_ZV_CASE(2, 2) DMCX_ZV_CASE(2, 3) DMCX_ZV_CASE(2, 4)
    case 0: zv_stage_t<T, 0, 0>(B, gatom, g_begin, g_end, fn_begin, pts, cj, npts, Ys, slot, satom, sacc, gi.y); break;
    case 16: zv_stage_t<T, 1, 0>(B, gatom, g_begin, g_end, fn_begin, pts, cj, npts, Ys, slot, satom, sacc, gi.y); break;
    case 32: zv_stage_t<T, 2, 0>(B, gatom, g_begin, g_end, fn_begin, pts, cj, npts, Ys, slot, satom, sacc, gi.y); break;
    default: break;
  }
#undef DMCX_ZV_CASE
}

// Determinant adjoint of Eq. 4 for a tile of FPTS electrons of one walker;
// grid = Wpad * ntile.  Per stage: Ys[f][(y1 | y2), n] = sum_k Cp[f][k]
// [g_n | x_n][k] (MFMA), then the basis derivatives weighted by Ys.  Writes
// the tile's per-atom sums zpart[w][tile][atom][3] = sum_i sum_{l on atom}
// q_i(l) and the per-electron sums zs[w][e][3] = sum_l q_e(l).
template <typename T, int NOB>
__global__ __launch_bounds__(NT_FORCE) void k_zv_det(DevCtx c, const T *xt, const double *cg,
                                                    double *zpart, double *zs) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  constexpr int NC2 = 2 * FPTS;
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Gp[NP * NC2];   // B operand: Gp[k][n] = g_n[k], Gp[k][FPTS + n] = x_n[k]
  __shared__ T Ys[FM * NC2];
  __shared__ double pbin[MAX_ATOM * 3];
  __shared__ double slot[FM * 3];  // shell totals of the current stage
  __shared__ int satom[FM];
  __shared__ double sred[NT_FORCE / 32][FPTS * 3];  // per-point sums of each half-wave
  __shared__ double pts[FPTS][3];
  __shared__ double cj[FPTS][3];
  const int ntile = (c.ne + FPTS - 1) / FPTS;
  const int w = blockIdx.x / ntile, tile = blockIdx.x % ntile;
  const int e0 = tile * FPTS, npts = min(FPTS, c.ne - e0);
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  const int kq = lane >> 4, cl = lane & 15;
  const T *Cp;
  if constexpr (sizeof(T) == 8) Cp = (const T *)c.B.Cp; else Cp = (const T *)c.B.Cp32;
  for (int i = tid; i < NP * NC2; i += NT_FORCE) {
    const int k = i / NC2, col = i % NC2, n = col % FPTS;
    T v = 0;
    if (n < npts) {
      const int e = e0 + n, sp = e < c.n_up ? 0 : 1, ii = e - sp * c.n_up;
      const T *src = col < FPTS ? (const T *)c.GT : xt;
      v = src[gt_off(c, w, sp) + (size_t)ii * NP + k];
    }
    Gp[i] = v;
  }
  for (int i = tid; i < c.n_atom * 3; i += NT_FORCE) pbin[i] = 0.0;
  if (tid < FPTS * 3) {
    const int n = tid / 3, x = tid % 3;
    const int e = e0 + min(n, npts - 1);
    pts[n][x] = c.R[((size_t)w * c.ne + e) * 3 + x];
    cj[n][x] = cg[((size_t)w * c.ne + e) * 6 + x];
  }
  double sacc[3] = {0.0, 0.0, 0.0};  // point tid % 32, shells of half-wave tid / 32
  __syncthreads();
  for (int st = 0; st < c.B.n_stage; ++st) {
    const int2 sg = BL.stages[st];
    const int fb = BL.ginfo[sg.x].z;
    const int fe = sg.y < c.B.n_group ? BL.ginfo[sg.y].z : c.B.Kp;
    const int nft = (fe - fb + 15) / 16;
    for (int tt = wid; tt < nft * (NC2 / 16); tt += NT_FORCE / 64) {
      const int f0 = (tt / (NC2 / 16)) * 16, n0 = (tt % (NC2 / 16)) * 16;
      const auto y = mfma_tile<T>(
          NP,
          [&](int i, int k) {
            const T v = Cp[(size_t)(fb + f0 + i) * NP + k];
            return (fb + f0 + i < fe) ? v : (T)0;
          },
          [&](int k, int j) { return Gp[k * NC2 + n0 + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = f0 + Acc4<T>::row(kq, r);
        if (f < FM) Ys[f * NC2 + n0 + cl] = y[r];
      }
    }
    __syncthreads();
    zv_stage<T>(BL, c.B.gatom, sg.x, sg.y, fb, pts, cj, npts, Ys, slot, satom, sacc);
    __syncthreads();
    bin_slots(4 * (sg.y - sg.x), slot, satom, pbin, c.n_atom);
  }
  double *out = zpart + ((size_t)w * ntile + tile) * c.n_atom * 3;
  for (int i = tid; i < c.n_atom * 3; i += NT_FORCE) out[i] = pbin[i];
  // per-point sums: the half-waves' partial sums added in half-wave order
  for (int x = 0; x < 3; ++x) sred[tid >> 5][(tid & 31) * 3 + x] = sacc[x];
  __syncthreads();
  for (int i = tid; i < npts * 3; i += NT_FORCE) {
    double v = 0.0;
#pragma unroll
    for (int h = 0; h < NT_FORCE / 32; ++h) v += sred[h][i];
    zs[((size_t)w * c.ne + e0) * 3 + i] = v;
  }
}

}  // namespace dmcx
