// Ion-coordinate derivatives (Hellmann-Feynman + Pulay parts) by a
// hand-written reverse-mode adjoint (Eq. 3 with lambda = an ion coordinate).
//
// For spin sigma, d ln|D| / dR_A = tr(A^{-1} dA/dR_A) with
// dA_ij/dR_A = -sum_{l on A} C_lj grad Phi_l(r_i).  Contracting the orbital
// index first,
//   d ln|D| / dR_A = -sum_i sum_{l on A} grad Phi_l(r_i) y_i[l],
//   y_i = C g_i,  g_i = column i of A^{-1} (row i of GT),
// so the adjoint of the MO contraction is one GEMM per tile of electron
// points (MFMA: basis functions x points x orbitals) and the adjoint of the
// basis is a gradient evaluation weighted by y, summed per atom.  Neither the
// basis gradients nor y ever go to HBM.
#pragma once
#include "kernels.h"

namespace dmcx {

constexpr int FPTS = 32;        // electron points per force tile
constexpr int MAX_ATOM = 256;   // per-tile atom accumulators in LDS
constexpr int NT_FORCE = 256;

// Shell totals of one stage, binned by atom: slot[sl][3] holds the total of
// the stage's shell slot sl and satom[sl] its atom (-1: padding).  Thread i
// (i < 3 n_atom) adds the totals of atom i / 3 in slot order, so the sums do
// not depend on how the waves were scheduled (no atomics).
__device__ __forceinline__ void bin_slots(int nsh, const double *slot, const int *satom,
                                          double *bin, int n_atom) {
  for (int i = threadIdx.x; i < n_atom * 3; i += NT_FORCE) {
    const int a = i / 3, x = i % 3;
    double s = bin[i];
    for (int sl = 0; sl < nsh; ++sl)
      if (satom[sl] == a) s += slot[sl * 3 + x];
    bin[i] = s;
  }
}

// Gradient-only evaluation of one stage's shells at the tile's points,
// weighted by Ys[f][n]; lane task (point n = lane % 32, shell).  The 32
// points of a shell are reduced across lanes into the shell's slot total
// (slot, satom; binned by atom with bin_slots after a barrier).
template <typename T, int L, int NPR>
__device__ void force_stage_t(const BasisLDS &B, const int *gatom, int g_begin, int g_end,
                              int fn_begin, const double (*pts)[3], int npts, const T *Ys,
                              double *slot, int *satom, int npr_rt = NPR) {
  constexpr int NC = L == 0 ? 1 : (L == 1 ? 3 : 6);
  const int nsh = 4 * (g_end - g_begin);
  const int tid = threadIdx.x;
  const int n = tid & 31;
  for (int sl = tid >> 5; sl < nsh; sl += NT_FORCE / 32) {
    const int g = g_begin + (sl >> 2), s = sl & 3;
    const int4 gi = B.ginfo[g];
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    if (n < npts) {
      const double *cxyz = B.xyz + (size_t)(g * 4 + s) * 3;
      const T x = (T)(pts[n][0] - cxyz[0]), y = (T)(pts[n][1] - cxyz[1]), z = (T)(pts[n][2] - cxyz[2]);
      const T s2 = x * x + y * y + z * z;
      T R0 = 0, R1 = 0;
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
        }
      } else {
        for (int p = 0; p < npr_rt; ++p) {
          const T ap = (T)B.alpha[gi.w + p * 4 + s];
          const T ep = (T)B.coef[gi.w + p * 4 + s] * texp(-ap * s2);
          R0 += ep;
          R1 -= ap * ep;
        }
      }
      const T *yrow = Ys + (size_t)(gi.z - fn_begin + s) * FPTS + n;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        T P, Px, Py, Pz, Lp;
        switch (cc) {  // resolved at compile time after unrolling
          case 0: cart_poly_t<L, 0, T>(x, y, z, P, Px, Py, Pz, Lp); break;
          case 1: cart_poly_t<L, 1, T>(x, y, z, P, Px, Py, Pz, Lp); break;
          case 2: cart_poly_t<L, 2, T>(x, y, z, P, Px, Py, Pz, Lp); break;
          case 3: cart_poly_t<L, 3, T>(x, y, z, P, Px, Py, Pz, Lp); break;
          case 4: cart_poly_t<L, 4, T>(x, y, z, P, Px, Py, Pz, Lp); break;
          default: cart_poly_t<L, 5, T>(x, y, z, P, Px, Py, Pz, Lp); break;
        }
        const T tr = (T)2 * R1 * P;
        const double yv = (double)yrow[(size_t)cc * 4 * FPTS];
        f0 += (double)(Px * R0 + x * tr) * yv;
        f1 += (double)(Py * R0 + y * tr) * yv;
        f2 += (double)(Pz * R0 + z * tr) * yv;
      }
    }
    f0 = sum32(f0);
    f1 = sum32(f1);
    f2 = sum32(f2);
    if (n == 0) {
      slot[sl * 3 + 0] = f0;
      slot[sl * 3 + 1] = f1;
      slot[sl * 3 + 2] = f2;
      satom[sl] = gatom[g * 4 + s];
    }
  }
}

template <typename T>
__device__ inline void force_stage(const BasisLDS &B, const int *gatom, int g_begin, int g_end,
                                   int fn_begin, const double (*pts)[3], int npts,
                                   const T *Ys, double *slot, int *satom) {
  const int4 gi = B.ginfo[g_begin];
#define DMCX_FORCE_CASE(LL, NN)                                                              \
  case LL * 16 + NN:                                                                         \
    force_stage_t<T, LL, NN>(B, gatom, g_begin, g_end, fn_begin, pts, npts, Ys, slot, satom); break;
  switch (gi.x * 16 + (gi.y <= 4 ? gi.y : 0)) {
    DMCX_FORCE_CASE(0, 1) DMCX_FORCE_CASE(0, 2) DMCX_FORCE_CASE(0, 3) DMCX_FORCE_CASE(0, 4)
    DMCX_FORCE_CASE(1, 1) DMCX_FORCE_CASE(1, 2) DMCX_FORCE_CASE(1, 3) DMCX_FORCE_CASE(1, 4)
    DMCX_FORCE_CASE(2, 1) DMCX_FORCE_CASE(2, 2) DMCX_FORCE_CASE(2, 3) DMCX_FORCE_CASE(2, 4)
    case 0: force_stage_t<T, 0, 0>(B, gatom, g_begin, g_end, fn_begin, pts, npts, Ys, slot, satom, gi.y); break;
    case 16: force_stage_t<T, 1, 0>(B, gatom, g_begin, g_end, fn_begin, pts, npts, Ys, slot, satom, gi.y); break;
    case 32: force_stage_t<T, 2, 0>(B, gatom, g_begin, g_end, fn_begin, pts, npts, Ys, slot, satom, gi.y); break;
    default: break;
  }
#undef DMCX_FORCE_CASE
}

// Determinant part of d ln|Psi| / dR for a tile of FPTS electrons of one
// walker; grid = Wpad * ntile, ntile = ceil(ne / FPTS).  Writes the tile's
// per-atom sums sum_i sum_{l on A} grad Phi_l(r_i) y_i[l] to
// partial[w][tile][atom][3] (the derivative is minus their sum).
template <typename T, int NOB>
__global__ __launch_bounds__(NT_FORCE) void k_ion_grad_det(DevCtx c, double *partial) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Gp[NP * FPTS];   // B operand: Gp[k][n] = g_n[k]
  __shared__ T Ys[FM * FPTS];   // y of the stage's functions
  __shared__ double fbin[MAX_ATOM * 3];
  __shared__ double slot[FM * 3];  // shell totals of the current stage
  __shared__ int satom[FM];
  __shared__ double pts[FPTS][3];
  const int ntile = (c.ne + FPTS - 1) / FPTS;
  const int w = blockIdx.x / ntile, tile = blockIdx.x % ntile;
  const int e0 = tile * FPTS, npts = min(FPTS, c.ne - e0);
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  const int kq = lane >> 4, cl = lane & 15;
  const T *Cp;
  if constexpr (sizeof(T) == 8) Cp = (const T *)c.B.Cp; else Cp = (const T *)c.B.Cp32;
  for (int i = tid; i < NP * FPTS; i += NT_FORCE) {
    const int k = i / FPTS, n = i % FPTS;
    T v = 0;
    if (n < npts) {
      const int e = e0 + n, sp = e < c.n_up ? 0 : 1, ii = e - sp * c.n_up;
      v = ((const T *)c.GT)[gt_off(c, w, sp) + (size_t)ii * NP + k];
    }
    Gp[i] = v;
  }
  for (int i = tid; i < c.n_atom * 3; i += NT_FORCE) fbin[i] = 0.0;
  if (tid < FPTS * 3) {
    const int n = tid / 3, x = tid % 3;
    pts[n][x] = c.R[((size_t)w * c.ne + e0 + min(n, npts - 1)) * 3 + x];
  }
  __syncthreads();
  for (int st = 0; st < c.B.n_stage; ++st) {
    const int2 sg = BL.stages[st];
    const int fb = BL.ginfo[sg.x].z;
    const int fe = sg.y < c.B.n_group ? BL.ginfo[sg.y].z : c.B.Kp;
    const int nft = (fe - fb + 15) / 16;  // 16-row function tiles (stage size is a multiple of 4)
    // Ys[f][n] = sum_k Cp[fb + f][k] Gp[k][n]
    for (int tt = wid; tt < nft * (FPTS / 16); tt += NT_FORCE / 64) {
      const int f0 = (tt / (FPTS / 16)) * 16, n0 = (tt % (FPTS / 16)) * 16;
      const auto y = mfma_tile<T>(
          NP,
          [&](int i, int k) {
            // rows past the stage are read (the LCAO array has zero rows past
            // its end) and masked, so the loads carry no branches
            const T v = Cp[(size_t)(fb + f0 + i) * NP + k];
            return (fb + f0 + i < fe) ? v : (T)0;
          },
          [&](int k, int j) { return Gp[k * FPTS + n0 + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = f0 + Acc4<T>::row(kq, r);
        if (f < FM) Ys[f * FPTS + n0 + cl] = y[r];
      }
    }
    __syncthreads();
    force_stage<T>(BL, c.B.gatom, sg.x, sg.y, fb, pts, npts, Ys, slot, satom);
    __syncthreads();
    bin_slots(4 * (sg.y - sg.x), slot, satom, fbin, c.n_atom);
  }
  double *out = partial + ((size_t)w * ntile + tile) * c.n_atom * 3;
  for (int i = tid; i < c.n_atom * 3; i += NT_FORCE) out[i] = fbin[i];
}

}  // namespace dmcx
