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
// k_jparam: one workgroup per walker.  The drift v_i and the positions go
// to LDS first (one wave per electron).  Every unordered electron pair {i, j}
// is visited once and contributes to both electrons.  For a pair term
// f = P(a, b) Q(c) with a = s(x), b = s(y), c = s(z), x = |r_i - R_A|,
// y = |r_j - R_A|, z = |r_i - r_j| (P symmetric), the chain rule gives
//   lap_i f + lap_j f + 2 v_i . grad_i f + 2 v_j . grad_j f
//     = Q [P_aa al_x + P_a be_x + P_bb al_y + P_b be_y]
//       + 2 Q' c' [P_a u - P_b w] + P ga,
// al_x = a'^2, be_x = a'' + 2 a' (1/x + v_i . e_iA), u = a' e_iA . e_ij,
// w = b' e_jA . e_ij, ga = 2 (Q'' c'^2 + Q' c'') + 2 Q' c' (2/z + (v_i - v_j) . e_ij)
// (unit vectors e_iA along r_i - R_A, e_ij along r_i - r_j).  al, be, a and
// a'/x depend on one electron and one atom: they are staged in LDS for a
// chunk of atoms; z, c, c', c'', ga and r_i . (r_i - r_j) depend on the pair
// only and are formed once per pair and chunk, so the work per pair and atom
// is the two dot products that give u and w and the six terms, written out
// with their P polynomials.  Each thread keeps its 16 sums in registers; the
// block adds them in a fixed order (bit-reproducible).
#pragma once
#include "zv.h"

namespace dmcx {

constexpr int NJP = 8;       // Jastrow parameters

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

// Scaled distance s = r / (1 + r) with s' and s'' at one distance.
struct Scaled {
  double s, s1, s2;
};
__device__ __forceinline__ Scaled scaled(double r) {
  const double q = 1.0 / (1.0 + r);
  return Scaled{r * q, q * q, -2.0 * q * q * q};
}

// d/db of the Pade term a r / (1 + b r): value and first two r-derivatives.
__device__ __forceinline__ void pade_db(double a, double b, double r, double &h, double &h1,
                                        double &h2) {
  const double q = 1.0 / (1.0 + b * r), q2 = q * q;
  h = -a * r * r * q2;
  h1 = -2.0 * a * r * q2 * q;
  h2 = -2.0 * a * (1.0 - 2.0 * b * r) * q2 * q2;
}

// Atoms per LDS chunk for ne electrons: the staged table (4 doubles per
// electron and atom) plus positions and drifts within about 40 KB.
inline int jparam_chunk(int ne) {
  const int n = (40960 / 8 - 6 * ne) / (4 * ne);
  return n < 1 ? 1 : (n > 8 ? 8 : n);
}
inline size_t jparam_lds(int ne) {
  return (size_t)ne * (6 + 4 * jparam_chunk(ne)) * sizeof(double);
}

// grid W (one workgroup per walker), block NT_AUX, dynamic LDS jparam_lds(ne).
// O [W][8] = d ln Psi / dp, D [W][8] = dE_L / dp.
template <typename T>
__global__ __launch_bounds__(NT_AUX) void k_jparam(DevCtx c, int nch, double *Oout,
                                                   double *Dout) {
  extern __shared__ double sm[];
  __shared__ double red[NT_AUX / 64][2 * NJP];
  const int ne = c.ne;
  double *s_v = sm;           // [ne][3] drift
  double *s_r = sm + 3 * ne;  // [ne][3] positions
  double *s_e = sm + 6 * ne;  // [nch][ne][4]: a, a'^2, be, a'/x for the chunk's atoms
  const int w = blockIdx.x;
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  constexpr int NWV = NT_AUX / 64;
  const double *Rw = c.R + (size_t)w * ne * 3;
  for (int i = wid; i < ne; i += NWV) {
    double o[6];
    electron_cg<T>(c, Rw, w, i, lane, o);
    if (lane == 0)
      for (int x = 0; x < 3; ++x) {
        s_v[3 * i + x] = o[x] + o[3 + x];
        s_r[3 * i + x] = Rw[3 * i + x];
      }
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
      d[x] = s_r[3 * i + x] - s_r[3 * j + x];
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
  for (int A0 = 0; A0 < c.n_atom; A0 += nch) {
    const int na = min(nch, c.n_atom - A0);
    // stage the chunk; the electron-nucleus Pade b terms on the way
    for (int t = tid; t < na * ne; t += NT_AUX) {
      const int al = t / ne, e = t - al * ne, A = A0 + al;
      double X[3], x2 = 0.0, vX = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        X[q] = s_r[3 * e + q] - c.ion[3 * A + q];
        x2 += X[q] * X[q];
        vX += s_v[3 * e + q] * X[q];
      }
      const double x = sqrt(x2), ix = 1.0 / x;
      const Scaled S = scaled(x);
      double hb, h1, h2;
      pade_db(c.jen_a[A], c.jen_b, x, hb, h1, h2);
      O[1] += hb;
      Ls[1] += h2 + 2.0 * h1 * ix + 2.0 * h1 * vX * ix;
      double *o = s_e + (size_t)t * 4;
      o[0] = S.s;
      o[1] = S.s1 * S.s1;
      o[2] = S.s2 + 2.0 * S.s1 * (ix + vX * ix);
      o[3] = S.s1 * ix;
    }
    __syncthreads();
    for (int p = tid; p < npair; p += NT_AUX) {
      int i, j;
      pair_of(p, ne, h, i, j);
      const double ri[3] = {s_r[3 * i], s_r[3 * i + 1], s_r[3 * i + 2]};
      const double rj[3] = {s_r[3 * j], s_r[3 * j + 1], s_r[3 * j + 2]};
      double d[3], z2 = 0.0, vd = 0.0, rid = 0.0, rjd = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        d[q] = ri[q] - rj[q];
        z2 += d[q] * d[q];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        vd += (s_v[3 * i + q] - s_v[3 * j + q]) * d[q];
        rid += ri[q] * d[q];
        rjd += rj[q] * d[q];
      }
      const double z = sqrt(z2), iz = 1.0 / z;
      const Scaled Z = scaled(z);
      const double cz = Z.s, cz2 = cz * cz;
      const double g = 2.0 * iz + vd * iz;
      const double dl1 = 2.0 * Z.s1, dl2 = 4.0 * cz * Z.s1;   // 2 Q' c' for Q = c, c^2
      const double ga1 = 2.0 * Z.s2 + dl1 * g;                 // ga for Q = c
      const double ga2 = 4.0 * (Z.s1 * Z.s1 + cz * Z.s2) + dl2 * g;  // ga for Q = c^2
      for (int al = 0; al < na; ++al) {
        const double *RA = c.ion + 3 * (A0 + al);
        const double RAd = RA[0] * d[0] + RA[1] * d[1] + RA[2] * d[2];
        const double *ei = s_e + ((size_t)al * ne + i) * 4, *ej = s_e + ((size_t)al * ne + j) * 4;
        const double a = ei[0], Ax = ei[1], Bx = ei[2];
        const double b = ej[0], Ay = ej[1], By = ej[2];
        const double u = ei[3] * (rid - RAd) * iz, v = ej[3] * (rjd - RAd) * iz;
        const double ab = a * b, apb = a + b, a2b2 = a * a + b * b;
        const double Bs = Bx + By, bBaB = b * Bx + a * By, uv = u - v;
        // (1,1,0): P = 2ab
        O[2] += 2.0 * ab;
        Ls[2] += 2.0 * bBaB;
        // (1,0,1): P = a + b, Q = c
        O[3] += apb * cz;
        Ls[3] += cz * Bs + dl1 * uv + apb * ga1;
        // (1,1,1): P = 2ab, Q = c
        O[4] += 2.0 * ab * cz;
        Ls[4] += 2.0 * (cz * bBaB + dl1 * (b * u - a * v) + ab * ga1);
        // (2,1,0): P = a^2 b + a b^2
        O[5] += ab * apb;
        Ls[5] += 2.0 * (b * Ax + a * Ay) + (2.0 * ab + b * b) * Bx + (a * a + 2.0 * ab) * By;
        // (2,0,1): P = a^2 + b^2, Q = c
        O[6] += a2b2 * cz;
        Ls[6] += 2.0 * (cz * (Ax + Ay + a * Bx + b * By) + dl1 * (a * u - b * v)) + a2b2 * ga1;
        // (1,0,2): P = a + b, Q = c^2
        O[7] += apb * cz2;
        Ls[7] += cz2 * Bs + dl2 * uv + apb * ga2;
      }
    }
    __syncthreads();  // s_e is rewritten for the next chunk
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

// Linear-method matrices of one context's walkers.  Weights
// omega = exp(log w - m), m the largest counted log w; a walker counts when
// its log w and E_L are finite and its flags are clear.  With
// <x> = sum omega x / sum omega and dO_k = O_k - <O_k>:
//   S[0][0] = 1, S[0][k] = S[k][0] = 0, S[k][l] = <dO_k dO_l>,
//   H[0][0] = <E>, H[k][0] = <dO_k E>, H[0][l] = <E dO_l> + <dE_l>,
//   H[k][l] = <dO_k (dO_l E + dE_l)>;
// out = S [9][9] then H [9][9]; with no walker counted every entry is NaN.
// Two passes over blocks of LM_NB walkers, each block writing one record of
// sums taken in walker order, and a merge of the records in block order
// after each pass (bit-reproducible):
//   pass 1: record b = {m_b, sum omega_b, sum omega_b z} over z = E, O_k, dE_k,
//           omega_b = exp(log w - m_b); the merge rescales by exp(m_b - m)
//           and gives m, sum omega and the means;
//   pass 2: record b = the centred sums with omega = exp(log w - m).
constexpr int LM_NB = 128;                 // walkers (threads) per block
constexpr int LM_Z = 2 + 2 * NJP;          // staged per walker: omega, E, O[8], dE[8]
constexpr int LM_NS = NJP * (NJP + 1) / 2; // S[k][l], k <= l
constexpr int LM_NE = LM_NS + NJP + NJP * NJP;  // second-pass sums: S, H[k][0], H[k][l]
constexpr int LM_REC = LM_NE;              // doubles per block record (>= 1 + LM_Z)
static_assert(LM_REC >= 1 + LM_Z && LM_NE <= LM_NB, "record layout");

inline int lm_blocks(int W) { return (W + LM_NB - 1) / LM_NB; }

// Stage this block's walkers (one per thread): omega relative to the shift,
// E, O, dE, zeros for walkers that do not count.  Returns whether it counts.
__device__ __forceinline__ bool lm_stage(int W, const double *logw, const double *eloc,
                                         const unsigned *flags, const double *O, const double *D,
                                         double shift, bool use_shift, double (*st)[LM_Z + 1]) {
  const int w = blockIdx.x * LM_NB + threadIdx.x;
  const bool ok = w < W && flags[w] == 0u && isfinite(logw[w]) && isfinite(eloc[w]);
  double *z = st[threadIdx.x];
  z[0] = ok && use_shift ? exp(logw[w] - shift) : 0.0;
  z[1] = ok ? eloc[w] : 0.0;
  for (int k = 0; k < NJP; ++k) {
    z[2 + k] = ok ? O[(size_t)w * NJP + k] : 0.0;
    z[2 + NJP + k] = ok ? D[(size_t)w * NJP + k] : 0.0;
  }
  return ok;
}

__global__ __launch_bounds__(LM_NB) void k_lm_pass1(int W, const double *logw, const double *eloc,
                                                    const unsigned *flags, const double *O,
                                                    const double *D, double *part) {
  __shared__ double st[LM_NB][LM_Z + 1];
  __shared__ double red[LM_NB / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = blockIdx.x * LM_NB + tid;
  const bool ok = w < W && flags[w] == 0u && isfinite(logw[w]) && isfinite(eloc[w]);
  double m = ok ? logw[w] : -INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[tid >> 6] = m;
  __syncthreads();
  m = red[0];
#pragma unroll
  for (int q = 1; q < LM_NB / 64; ++q) m = fmax(m, red[q]);
  lm_stage(W, logw, eloc, flags, O, D, m, m > -INFINITY, st);
  __syncthreads();
  double *r = part + (size_t)blockIdx.x * LM_REC;
  if (tid < LM_Z) {
    const int n = min(LM_NB, W - (int)blockIdx.x * LM_NB);
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += tid == 0 ? st[t][0] : st[t][0] * st[t][tid];
    r[1 + tid] = acc;
  }
  if (tid == 0) r[0] = m;
}

// mm = {sum omega, <E>, <O_k>, <dE_k>, m} (LM_Z + 1 values), one block of LM_NB threads.
__global__ __launch_bounds__(LM_NB) void k_lm_merge(int nblk, const double *part, double *mm) {
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int b = 0; b < nblk; ++b) m = fmax(m, part[(size_t)b * LM_REC]);
  double acc = 0.0;
  if (tid < LM_Z && m > -INFINITY)
    for (int b = 0; b < nblk; ++b) {
      const double *r = part + (size_t)b * LM_REC;
      if (r[0] > -INFINITY) acc += exp(r[0] - m) * r[1 + tid];
    }
  __shared__ double s0;
  if (tid == 0) s0 = acc;
  __syncthreads();
  if (tid < LM_Z) mm[tid] = tid == 0 ? acc : acc / s0;
  if (tid == 0) mm[LM_Z] = m;
}

// Second-pass sum e of thread tid: kind 0 S[k][l] (k <= l), 1 H[k][0], 2 H[k][l].
__device__ __forceinline__ int lm_entry(int e, int &k, int &l) {
  if (e < LM_NS) {
    int r = e;
    k = 0;
    while (r >= NJP - k) r -= NJP - k, ++k;
    l = k + r;
    return 0;
  }
  if (e < LM_NS + NJP) {
    k = e - LM_NS;
    l = 0;
    return 1;
  }
  const int r = e - LM_NS - NJP;
  k = r / NJP;
  l = r % NJP;
  return 2;
}

__global__ __launch_bounds__(LM_NB) void k_lm_pass2(int W, const double *logw, const double *eloc,
                                                    const unsigned *flags, const double *O,
                                                    const double *D, const double *mm,
                                                    double *part) {
  __shared__ double st[LM_NB][LM_Z + 1];
  const int tid = threadIdx.x;
  const double m = mm[LM_Z];
  lm_stage(W, logw, eloc, flags, O, D, m, m > -INFINITY, st);
  __syncthreads();
  if (tid >= LM_NE) return;
  int k, l;
  const int kind = lm_entry(tid, k, l);
  const double mk = mm[2 + k], ml = mm[2 + l];
  const int n = min(LM_NB, W - (int)blockIdx.x * LM_NB);
  double acc = 0.0;
  for (int t = 0; t < n; ++t) {
    const double *z = st[t];
    const double dk = z[2 + k] - mk;
    double v;
    if (kind == 0)
      v = dk * (z[2 + l] - ml);
    else if (kind == 1)
      v = dk * z[1];
    else
      v = dk * ((z[2 + l] - ml) * z[1] + z[2 + NJP + l]);
    acc += z[0] * v;
  }
  part[(size_t)blockIdx.x * LM_REC + tid] = acc;
}

__global__ __launch_bounds__(LM_NB) void k_lm_final(int nblk, const double *part,
                                                    const double *mm, double *out) {
  const int tid = threadIdx.x;
  constexpr int P1 = NJP + 1;
  double *S = out, *H = out + P1 * P1;
  const double s0 = mm[0];
  const bool any = s0 > 0.0;
  const double nan = __builtin_nan("");
  if (tid < LM_NE) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * LM_REC + tid];
    const double v = any ? acc / s0 : nan;
    int k, l;
    const int kind = lm_entry(tid, k, l);
    if (kind == 0) {
      S[(1 + k) * P1 + 1 + l] = v;
      S[(1 + l) * P1 + 1 + k] = v;
    } else if (kind == 1) {
      H[(1 + k) * P1] = v;
      H[1 + k] = any ? v + mm[2 + NJP + k] : nan;  // <E dO_l> + <dE_l>
    } else {
      H[(1 + k) * P1 + 1 + l] = v;
    }
  } else if (tid == LM_NE) {
    S[0] = any ? 1.0 : nan;
    H[0] = any ? mm[1] : nan;
    for (int k = 1; k < P1; ++k) S[k] = S[k * P1] = any ? 0.0 : nan;
  }
}

}  // namespace dmcx
