// Jastrow parameter derivatives and the linear-method matrices: what one step
// of the variational optimisation of the Jastrow factor of Eq. 2 needs from
// the walkers (QMC section: the trial function is optimised in VMC before
// the DMC projection of Eq. 1).
//
// Parameters, in order (DMCX_N_JASTROW_PARAMS = 8):
//   0  b of the electron-electron Pade terms u = a r / (1 + b r),
//   1  b of the electron-nucleus Pade terms,
//   2..7  the coefficients c_k of a three-body electron-electron-nucleus term
//      sum_k c_k sum_A sum_{i<j} f_k,  f_k = (s_iA^l s_jA^m + s_iA^m s_jA^l) s_ij^n,
//      s(r) = r / (1 + r), (l, m, n) = (1,1,0), (1,0,1), (1,1,1), (2,1,0),
//      (2,0,1), (1,0,2), taken at c = 0 (the trial function is unchanged).
// Per walker, O_p = d ln Psi / dp and, with v_i = grad_i ln|Psi|,
//   dE_L / dp = -1/2 sum_i [lap_i O_p + 2 v_i . grad_i O_p].
//
// k_jparam: one workgroup per walker.  The drift v_i goes to LDS first (one
// wave per electron).  Every unordered electron pair {i, j} is visited once
// and contributes to both electrons: for a pair term f(x, y, z) with
// x = |r_i - R_A|, y = |r_j - R_A|, z = |r_i - r_j|,
//   lap_i f + lap_j f = f_xx + f_yy + 2 f_zz + 2 f_xz cos_i - 2 f_yz cos_j
//                       + 2 f_x / x + 2 f_y / y + 4 f_z / z,
//   2 (v_i . grad_i f + v_j . grad_j f) = 2 [f_x v_i.e_iA + f_y v_j.e_jA
//                                          + f_z (v_i - v_j).e_ij],
// cos_i = e_iA . e_ij, cos_j = e_jA . e_ij (unit vectors e_iA along r_i - R_A,
// e_ij along r_i - r_j).  The atoms are taken one at a time: the per-electron
// quantities for atom A (r_i - R_A, 1/x, s, s', s'', v_i . e_iA) are staged
// in LDS, then the threads run over the pairs.  Each thread keeps its 16 sums
// in registers; the block adds them in a fixed order (bit-reproducible).
#pragma once
#include "zv.h"

namespace dmcx {

constexpr int NJP = 8;       // Jastrow parameters
constexpr int JE = 8;        // LDS doubles per electron and atom
constexpr int LM_NT = 256;   // threads of the linear-method kernel
constexpr int LM_CH = 128;   // walkers staged per chunk
constexpr int LM_Z = 2 + 2 * NJP;  // staged values per walker: omega, E, O[8], dE[8]

// Unordered pair p of n electrons: electron i with its h = (n - 1) / 2 cyclic
// successors (p < n h), then for even n the pairs (i, i + n / 2), i < n / 2.
// Every pair {i, j}, i != j, appears exactly once.
__device__ __forceinline__ void pair_of(int p, int n, int h, int &i, int &j) {
  if (p < n * h) {
    i = p / h;
    j = i + 1 + (p - i * h);
    if (j >= n) j -= n;
  } else {
    i = p - n * h;
    j = i + n / 2;
  }
}

template <int K>
__device__ __forceinline__ double pw(double x) {
  if constexpr (K == 0) return 1.0;
  else return x * pw<K - 1>(x);
}
template <int K>
__device__ __forceinline__ double dpw(double x) {  // d/dx x^K
  if constexpr (K == 0) return 0.0;
  else return K * pw<K - 1>(x);
}
template <int K>
__device__ __forceinline__ double d2pw(double x) {  // d^2/dx^2 x^K
  if constexpr (K < 2) return 0.0;
  else return K * (K - 1) * pw<K - 2>(x);
}

// Scaled distance s = r / (1 + r) with s' and s'' at one distance.
struct Scaled {
  double s, s1, s2;
};
__device__ __forceinline__ Scaled scaled(double r) {
  const double q = 1.0 / (1.0 + r);
  return Scaled{r * q, q * q, -2.0 * q * q * q};
}

// One three-body term f = P(s_x, s_y) Q(s_z), P(a, b) = a^L b^M + a^M b^L,
// Q(c) = c^N, for one pair and atom: adds f to o and the pair's
// lap + 2 v . grad to l (see the header comment).
template <int L, int M, int N>
__device__ __forceinline__ void j3_term(const Scaled &X, const Scaled &Y, const Scaled &Zs,
                                        double ix, double iy, double iz, double ci, double cj,
                                        double vxi, double vyj, double vz, double &o, double &l) {
  const double a = X.s, b = Y.s;
  const double P = pw<L>(a) * pw<M>(b) + pw<M>(a) * pw<L>(b);
  const double Pa = dpw<L>(a) * pw<M>(b) + dpw<M>(a) * pw<L>(b);
  const double Pb = pw<L>(a) * dpw<M>(b) + pw<M>(a) * dpw<L>(b);
  const double Paa = d2pw<L>(a) * pw<M>(b) + d2pw<M>(a) * pw<L>(b);
  const double Pbb = pw<L>(a) * d2pw<M>(b) + pw<M>(a) * d2pw<L>(b);
  const double Q = pw<N>(Zs.s), Q1 = dpw<N>(Zs.s), Q2 = d2pw<N>(Zs.s);
  const double fx = Pa * X.s1 * Q, fy = Pb * Y.s1 * Q, fz = P * Q1 * Zs.s1;
  const double fxx = (Paa * X.s1 * X.s1 + Pa * X.s2) * Q;
  const double fyy = (Pbb * Y.s1 * Y.s1 + Pb * Y.s2) * Q;
  const double fzz = P * (Q2 * Zs.s1 * Zs.s1 + Q1 * Zs.s2);
  const double fxz = Pa * X.s1 * Q1 * Zs.s1, fyz = Pb * Y.s1 * Q1 * Zs.s1;
  o += P * Q;
  l += fxx + fyy + 2.0 * fzz + 2.0 * (fxz * ci - fyz * cj) + 2.0 * (fx * ix + fy * iy) +
       4.0 * fz * iz + 2.0 * (fx * vxi + fy * vyj + fz * vz);
}

// d/db of the Pade term a r / (1 + b r): value and first two r-derivatives.
__device__ __forceinline__ void pade_db(double a, double b, double r, double &h, double &h1,
                                        double &h2) {
  const double q = 1.0 / (1.0 + b * r), q2 = q * q;
  h = -a * r * r * q2;
  h1 = -2.0 * a * r * q2 * q;
  h2 = -2.0 * a * (1.0 - 2.0 * b * r) * q2 * q2;
}

// grid W (one workgroup per walker), block NT_AUX, dynamic LDS 11 ne doubles.
// O [W][8] = d ln Psi / dp, D [W][8] = dE_L / dp.
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_jparam(DevCtx c, double *Oout, double *Dout) {
  extern __shared__ double sm[];
  __shared__ double red[NT_AUX / 64][2 * NJP];
  const int ne = c.ne;
  double *s_v = sm;           // [ne][3] drift
  double *s_e = sm + 3 * ne;  // [ne][JE] for the current atom
  const int w = blockIdx.x;
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  constexpr int NWV = NT_AUX / 64;
  const double *Rw = c.R + (size_t)w * ne * 3;
  for (int i = wid; i < ne; i += NWV) {
    double o[6];
    electron_cg<T>(c, Rw, w, i, lane, o);
    if (lane == 0)
      for (int x = 0; x < 3; ++x) s_v[3 * i + x] = o[x] + o[3 + x];
  }
  __syncthreads();
  double O[NJP], Ls[NJP];
#pragma unroll
  for (int k = 0; k < NJP; ++k) O[k] = Ls[k] = 0.0;
  const int h = (ne - 1) / 2, npair = ne * h + ((ne & 1) ? 0 : ne / 2);
  // electron-electron Pade b: both electrons of the pair
  for (int p = tid; p < npair; p += NT_AUX) {
    int i, j;
    pair_of(p, ne, h, i, j);
    double d[3], z2 = 0.0, vd = 0.0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      d[x] = Rw[3 * i + x] - Rw[3 * j + x];
      z2 += d[x] * d[x];
    }
    const double z = sqrt(z2), iz = 1.0 / z;
#pragma unroll
    for (int x = 0; x < 3; ++x) vd += (s_v[3 * i + x] - s_v[3 * j + x]) * d[x];
    const double a = ((i < c.n_up) == (j < c.n_up)) ? c.jee_para : c.jee_anti;
    double hb, h1, h2;
    pade_db(a, c.jee_b, z, hb, h1, h2);
    O[0] += hb;
    Ls[0] += 2.0 * (h2 + 2.0 * h1 * iz) + 2.0 * h1 * vd * iz;
  }
  for (int A = 0; A < c.n_atom; ++A) {
    const double RA[3] = {c.ion[3 * A], c.ion[3 * A + 1], c.ion[3 * A + 2]};
    const double aA = c.jen_a[A];
    for (int e = tid; e < ne; e += NT_AUX) {
      double X[3], x2 = 0.0, vX = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        X[q] = Rw[3 * e + q] - RA[q];
        x2 += X[q] * X[q];
        vX += s_v[3 * e + q] * X[q];
      }
      const double x = sqrt(x2), ix = 1.0 / x;
      const Scaled S = scaled(x);
      double hb, h1, h2;
      pade_db(aA, c.jen_b, x, hb, h1, h2);
      O[1] += hb;
      Ls[1] += h2 + 2.0 * h1 * ix + 2.0 * h1 * vX * ix;
      double *o = s_e + (size_t)e * JE;
      o[0] = X[0]; o[1] = X[1]; o[2] = X[2]; o[3] = ix;
      o[4] = S.s; o[5] = S.s1; o[6] = S.s2; o[7] = vX * ix;
    }
    __syncthreads();
    for (int p = tid; p < npair; p += NT_AUX) {
      int i, j;
      pair_of(p, ne, h, i, j);
      const double *ei = s_e + (size_t)i * JE, *ej = s_e + (size_t)j * JE;
      double d[3], z2 = 0.0, xd = 0.0, yd = 0.0, vd = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        d[q] = ei[q] - ej[q];
        z2 += d[q] * d[q];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xd += ei[q] * d[q];
        yd += ej[q] * d[q];
        vd += (s_v[3 * i + q] - s_v[3 * j + q]) * d[q];
      }
      const double z = sqrt(z2), iz = 1.0 / z;
      const Scaled X{ei[4], ei[5], ei[6]}, Y{ej[4], ej[5], ej[6]}, Zs = scaled(z);
      const double ix = ei[3], iy = ej[3];
      const double ci = xd * ix * iz, cj = yd * iy * iz, vz = vd * iz;
      const double vxi = ei[7], vyj = ej[7];
      j3_term<1, 1, 0>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[2], Ls[2]);
      j3_term<1, 0, 1>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[3], Ls[3]);
      j3_term<1, 1, 1>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[4], Ls[4]);
      j3_term<2, 1, 0>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[5], Ls[5]);
      j3_term<2, 0, 1>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[6], Ls[6]);
      j3_term<1, 0, 2>(X, Y, Zs, ix, iy, iz, ci, cj, vxi, vyj, vz, O[7], Ls[7]);
    }
    __syncthreads();  // s_e is rewritten for the next atom
  }
#pragma unroll
  for (int k = 0; k < NJP; ++k) {
    const double so = sum64(O[k]), sl = sum64(Ls[k]);
    if (lane == 0) {
      red[wid][k] = so;
      red[wid][NJP + k] = sl;
    }
  }
  __syncthreads();
  if (tid < 2 * NJP) {
    double r = red[0][tid];
#pragma unroll
    for (int q = 1; q < NWV; ++q) r += red[q][tid];
    if (tid < NJP)
      Oout[(size_t)w * NJP + tid] = r;
    else
      Dout[(size_t)w * NJP + tid - NJP] = -0.5 * r;
  }
}

// Linear-method matrices of one context's walkers, one workgroup of LM_NT
// threads.  Weights omega = exp(log w - m), m the largest counted log w; a
// walker counts when its log w and E_L are finite and its flags are clear.
// With <x> = sum omega x / sum omega (sums in walker order) and
// dO_k = O_k - <O_k>:
//   S[0][0] = 1, S[0][k] = S[k][0] = 0, S[k][l] = <dO_k dO_l>,
//   H[0][0] = <E>, H[k][0] = <dO_k E>, H[0][l] = <E dO_l> + <dE_l>,
//   H[k][l] = <dO_k (dO_l E + dE_l)>;
// out = S [9][9] then H [9][9].  With no walker counted every entry is NaN.
// Two passes over the walkers (the means, then the centred sums), each
// staging LM_CH walkers at a time in LDS; thread t owns one sum and adds the
// staged walkers in order.
__global__ __launch_bounds__(LM_NT) void k_linear_method(int W, const double *logw,
                                                         const double *eloc,
                                                         const unsigned *flags, const double *O,
                                                         const double *D, double *out) {
  __shared__ double st[LM_CH][LM_Z + 1];
  __shared__ double red[LM_NT / 64];
  __shared__ double mean[LM_Z];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NE = 1 + NJP * (NJP + 1) / 2 + NJP + NJP * NJP;  // sums of the second pass
  // the largest counted log-weight
  double m = -INFINITY;
  for (int w = tid; w < W; w += LM_NT) {
    const double lw = logw[w], e = eloc[w];
    if (flags[w] == 0u && isfinite(lw) && isfinite(e)) m = fmax(m, lw);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wv] = m;
  __syncthreads();
  m = red[0];
#pragma unroll
  for (int q = 1; q < LM_NT / 64; ++q) m = fmax(m, red[q]);
  // stage walkers [w0, w0 + LM_CH): omega, E, O, dE (zeros for walkers that do not count)
  auto stage = [&](int w0) {
    for (int t = tid; t < LM_CH; t += LM_NT) {
      const int w = w0 + t;
      double *z = st[t];
      const bool ok = w < W && flags[w] == 0u && isfinite(logw[w]) && isfinite(eloc[w]);
      z[0] = ok ? exp(logw[w] - m) : 0.0;
      z[1] = ok ? eloc[w] : 0.0;
      for (int k = 0; k < NJP; ++k) {
        z[2 + k] = ok ? O[(size_t)w * NJP + k] : 0.0;
        z[2 + NJP + k] = ok ? D[(size_t)w * NJP + k] : 0.0;
      }
    }
  };
  // first pass: sum omega and sum omega z_t (t = E, O_k, dE_k)
  double acc = 0.0;
  for (int w0 = 0; w0 < W; w0 += LM_CH) {
    __syncthreads();
    stage(w0);
    __syncthreads();
    if (tid < LM_Z) {
      const int n = min(LM_CH, W - w0);
      for (int t = 0; t < n; ++t) acc += tid == 0 ? st[t][0] : st[t][0] * st[t][tid];
    }
  }
  if (tid < LM_Z) mean[tid] = acc;
  __syncthreads();
  const double s0 = mean[0];
  __syncthreads();
  if (tid > 0 && tid < LM_Z) mean[tid] = acc / s0;
  __syncthreads();
  // second pass: entry e of thread tid
  //   0: (unused), 1..36: S[k][l] k <= l, 37..44: H[k][0], 45..108: H[k][l]
  int ek = 0, el = 0, kind = -1;
  if (tid >= 1 && tid < 1 + NJP * (NJP + 1) / 2) {
    int r = tid - 1;
    ek = 0;
    while (r >= NJP - ek) r -= NJP - ek, ++ek;
    el = ek + r;
    kind = 0;
  } else if (tid >= 1 + NJP * (NJP + 1) / 2 && tid < 1 + NJP * (NJP + 1) / 2 + NJP) {
    ek = tid - 1 - NJP * (NJP + 1) / 2;
    kind = 1;
  } else if (tid >= 1 + NJP * (NJP + 1) / 2 + NJP && tid < NE) {
    const int r = tid - 1 - NJP * (NJP + 1) / 2 - NJP;
    ek = r / NJP;
    el = r % NJP;
    kind = 2;
  }
  const double mk = mean[2 + ek], ml = mean[2 + el];
  acc = 0.0;
  for (int w0 = 0; w0 < W; w0 += LM_CH) {
    __syncthreads();
    stage(w0);
    __syncthreads();
    if (kind >= 0) {
      const int n = min(LM_CH, W - w0);
      for (int t = 0; t < n; ++t) {
        const double *z = st[t];
        const double dk = z[2 + ek] - mk;
        double v;
        if (kind == 0)
          v = dk * (z[2 + el] - ml);
        else if (kind == 1)
          v = dk * z[1];
        else
          v = dk * ((z[2 + el] - ml) * z[1] + z[2 + NJP + el]);
        acc += z[0] * v;
      }
    }
  }
  constexpr int P1 = NJP + 1;
  double *S = out, *H = out + P1 * P1;
  const bool any = s0 > 0.0;
  const double nan = __builtin_nan("");
  if (kind == 0) {
    const double v = any ? acc / s0 : nan;
    S[(1 + ek) * P1 + 1 + el] = v;
    S[(1 + el) * P1 + 1 + ek] = v;
  } else if (kind == 1) {
    const double v = any ? acc / s0 : nan;
    H[(1 + ek) * P1] = v;
    H[1 + ek] = any ? v + mean[2 + NJP + ek] : nan;  // <E dO_l> + <dE_l>
  } else if (kind == 2) {
    H[(1 + ek) * P1 + 1 + el] = any ? acc / s0 : nan;
  } else if (tid == 0) {
    S[0] = any ? 1.0 : nan;
    H[0] = any ? mean[1] : nan;
    for (int k = 1; k < P1; ++k) S[k] = S[k * P1] = any ? 0.0 : nan;
  }
}

}  // namespace dmcx
