// dmcx kernels for gfx950.
//
// Work decomposition: a workgroup of 256 threads (4 waves) owns a tile of
// TW = 8 walkers.  Walkers are independent Markov chains, so a whole sweep
// (every electron of every walker in the tile) runs inside one launch with
// workgroup barriers only.  The 32 lanes tid/32 == slot serve walker `slot`
// for per-walker vector work (dot products over orbitals, Jastrow sums);
// the four waves cooperate on the orbital contraction, which is an MFMA GEMM
//   out[(walker, vgl), orbital] = sum_l Phi[(walker, vgl), l] C[l, orbital]
// with the basis values Phi produced in LDS stage by stage (never in HBM).
//
// Basis layout: shells are sorted on the host by (l, nprim) and packed in
// groups of four; within a group the K index runs component-major
// (comp * 4 + shell), and the LCAO matrix rows are permuted to match.  One
// lane task evaluates the radial part of one shell once and all of its
// Cartesian components.
//
// Inverse storage: GT[w][spin][b][j] = (A^{-1})_{j b}, i.e. row b is the
// column of A^{-1} that belongs to electron b, so the ratio for electron b
// is a contiguous dot product.
#pragma once
#include "device_common.h"

namespace dmcx {

constexpr int TW = 8;        // walkers (or points) per workgroup tile
constexpr int NCOL = 48;     // 5 VGL rows x 8 walkers = 40 MFMA columns, padded to 3 x 16
constexpr int FMAX = 96;     // basis functions per LDS stage
constexpr int NTHREADS = 256;
constexpr int KMAX = 64;     // largest delay rank

struct DevBasis {
  int n_group;
  const int4 *ginfo;     // per group: (l, nprim, first permuted function, first prim slot)
  const double *gxyz;    // [n_group*4][3] shell centres
  const double *galpha;  // prim slot + p*4 + shell
  const double *gcoef;
  const int *gatom;      // [n_group*4] atom of each shell, -1 for padding
  int n_stage;
  const int2 *stages;    // [n_stage] (first group, end group)
  int Kp;                // permuted function count
  const double *Cp;      // [Kp][NP] permuted LCAO coefficients (zero padded)
  const float *Cp32;
};

struct DevCtx {
  DevBasis B;
  int NP;                // padded orbital count (multiple of 16)
  int ne, n_up, n_dn, n_atom;
  const double *ion;     // [n_atom][3]
  const double *Z;       // [n_atom]
  const double *jen_a;   // [n_atom]
  double jen_b, jee_anti, jee_para, jee_b, v_nn;
  int W, Wpad, K;
  double tau;
  uint64_t seed;
  // walker state
  double *R;       // [Wpad][ne][3]
  double *vglc;    // [Wpad][ne][5][NP] orbital VGL rows at the current positions
  double *GT;      // [Wpad][2][NP][NP]
  double *Gb;      // [Wpad][K][NP] current inverse columns of the electron block
  double *Dl;      // [Wpad][K][NP] value-row changes of the block's moves
  double *Zs;      // [Wpad][K][NP] flush scratch
  double *logdet;  // [Wpad][2]
  double *sgn;     // [Wpad][2]
  double *eloc;    // [Wpad]
  double *logw;    // [Wpad]
  double *logpsi;  // [Wpad]
  unsigned *flags; // [Wpad] bit 0 non-finite, bit 1 singular
};

__device__ __forceinline__ size_t vglc_off(const DevCtx &c, int w, int e) {
  return ((size_t)w * c.ne + e) * 5 * c.NP;
}
__device__ __forceinline__ size_t gt_off(const DevCtx &c, int w, int sp) {
  return ((size_t)w * 2 + sp) * c.NP * c.NP;
}
__device__ __forceinline__ size_t blk_off(const DevCtx &c, int w) {
  return (size_t)w * c.K * c.NP;
}

// ------------------------------------------------------------ basis ----
// Cartesian monomial P, its gradient and Laplacian for component `comp` of
// angular momentum l at displacement (x, y, z); order p: x y z,
// d: xx xy xz yy yz zz.
__device__ __forceinline__ void cart_poly(int l, int comp, double x, double y, double z, double &P,
                                          double &Px, double &Py, double &Pz, double &L) {
  P = 1.0; Px = 0.0; Py = 0.0; Pz = 0.0; L = 0.0;
  if (l == 1) {
    if (comp == 0) { P = x; Px = 1.0; }
    else if (comp == 1) { P = y; Py = 1.0; }
    else { P = z; Pz = 1.0; }
  } else if (l == 2) {
    switch (comp) {
      case 0: P = x * x; Px = 2.0 * x; L = 2.0; break;
      case 1: P = x * y; Px = y; Py = x; break;
      case 2: P = x * z; Px = z; Pz = x; break;
      case 3: P = y * y; Py = 2.0 * y; L = 2.0; break;
      case 4: P = y * z; Py = z; Pz = y; break;
      default: P = z * z; Pz = 2.0 * z; L = 2.0; break;
    }
  }
}

// Evaluate the stage's shells at the tile's points into Bs[f][w*5 + q].
template <typename T>
__device__ void basis_stage(const DevBasis &B, int g_begin, int g_end, int fn_begin,
                            const double (*pts)[3], T *Bs) {
  const int nsh = 4 * (g_end - g_begin);
  for (int task = threadIdx.x; task < TW * nsh; task += NTHREADS) {
    const int w = task & (TW - 1);
    const int sl = task >> 3;
    const int g = g_begin + (sl >> 2), s = sl & 3;
    const int4 gi = B.ginfo[g];
    const double *cxyz = B.gxyz + (size_t)(g * 4 + s) * 3;
    const double x = pts[w][0] - cxyz[0], y = pts[w][1] - cxyz[1], z = pts[w][2] - cxyz[2];
    const double s2 = x * x + y * y + z * z;
    double R0 = 0.0, R1 = 0.0, R2 = 0.0;
    for (int p = 0; p < gi.y; ++p) {
      const double a = B.galpha[gi.w + p * 4 + s];
      const double e = B.gcoef[gi.w + p * 4 + s] * exp(-a * s2);
      R0 += e;
      R1 -= a * e;
      R2 += a * a * e;
    }
    // grad R = 2 r R1 ; lap R = 6 R1 + 4 s2 R2
    const double lapR = 6.0 * R1 + 4.0 * s2 * R2;
    const int ncomp = gi.x == 0 ? 1 : (gi.x == 1 ? 3 : 6);
    for (int comp = 0; comp < ncomp; ++comp) {
      double P, Px, Py, Pz, L;
      cart_poly(gi.x, comp, x, y, z, P, Px, Py, Pz, L);
      T *dst = Bs + (size_t)(gi.z - fn_begin + comp * 4 + s) * NCOL + w * 5;
      dst[0] = (T)(P * R0);
      dst[1] = (T)(Px * R0 + 2.0 * x * R1 * P);
      dst[2] = (T)(Py * R0 + 2.0 * y * R1 * P);
      dst[3] = (T)(Pz * R0 + 2.0 * z * R1 * P);
      dst[4] = (T)(L * R0 + 4.0 * R1 * (Px * x + Py * y + Pz * z) + P * lapR);
    }
  }
}

// Orbital VGL of the tile's TW points: out[w][q][orbital] (LDS, FP64).
// All 256 threads must call.  Bs must hold FMAX*NCOL elements; its padding
// columns 40..47 are cleared here.
template <typename T, int NOB>
__device__ void mo_tile(const DevCtx &c, const double (*pts)[3], T *Bs, double *out) {
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  constexpr int NQ = (NOB + 3) / 4;
  constexpr int NP = NOB * 16;
  typedef typename Acc4<T>::type acc_t;
  acc_t acc[NQ][3];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int cb = 0; cb < 3; ++cb) acc[q][cb] = acc_t{0, 0, 0, 0};
  const T *Cp;
  if constexpr (sizeof(T) == 8) Cp = (const T *)c.B.Cp; else Cp = (const T *)c.B.Cp32;
  for (int i = tid; i < FMAX * (NCOL - 40); i += NTHREADS)
    Bs[(i / (NCOL - 40)) * NCOL + 40 + i % (NCOL - 40)] = (T)0;
  const int kq = lane >> 4, col = lane & 15;
  for (int st = 0; st < c.B.n_stage; ++st) {
    const int2 sg = c.B.stages[st];
    const int fn_begin = c.B.ginfo[sg.x].z;
    const int fn_end = sg.y < c.B.n_group ? c.B.ginfo[sg.y].z : c.B.Kp;
    __syncthreads();
    basis_stage<T>(c.B, sg.x, sg.y, fn_begin, pts, Bs);
    __syncthreads();
    const int nk = (fn_end - fn_begin) >> 2;
    for (int kk = 0; kk < nk; ++kk) {
      const T *brow = Bs + (4 * kk + kq) * NCOL + col;
      const T b0 = brow[0], b1 = brow[16], b2 = brow[32];
      const T *arow = Cp + (size_t)(fn_begin + 4 * kk + kq) * NP + col;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int ob = wid + 4 * q;
        if (ob < NOB) {
          const T a = arow[ob * 16];
          acc[q][0] = mfma16x16x4(a, b0, acc[q][0]);
          acc[q][1] = mfma16x16x4(a, b1, acc[q][1]);
          acc[q][2] = mfma16x16x4(a, b2, acc[q][2]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int ob = wid + 4 * q;
    if (ob < NOB) {
#pragma unroll
      for (int cb = 0; cb < 3; ++cb) {
        const int n = cb * 16 + col;
        if (n < 40) {
#pragma unroll
          for (int r = 0; r < 4; ++r) out[n * NP + ob * 16 + Acc4<T>::row(kq, r)] = (double)acc[q][cb][r];
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------- Jastrow ----
// Lane-partial sums for electron i at position r against the other
// electrons of walker positions Rw and all ions: value u and gradient g.
__device__ __forceinline__ void jastrow_one_partial(const DevCtx &c, const double *Rw, int i,
                                                    const double r[3], int t, int nt, double &u,
                                                    double g[3]) {
  const int si = i < c.n_up ? 0 : 1;
  for (int j = t; j < c.ne + c.n_atom; j += nt) {
    const double *p;
    double a, b;
    if (j < c.ne) {
      if (j == i) continue;
      p = Rw + 3 * j;
      a = ((j < c.n_up ? 0 : 1) == si) ? c.jee_para : c.jee_anti;
      b = c.jee_b;
    } else {
      const int A = j - c.ne;
      p = c.ion + 3 * A;
      a = c.jen_a[A];
      b = c.jen_b;
    }
    const double dx = r[0] - p[0], dy = r[1] - p[1], dz = r[2] - p[2];
    const double rr = sqrt(dx * dx + dy * dy + dz * dz);
    const Pade pd = pade(a, b, rr);
    const double f = pd.d1 / rr;
    u += pd.u;
    g[0] += f * dx;
    g[1] += f * dy;
    g[2] += f * dz;
  }
}

// ------------------------------------------------------------ kernels ----
// Orbital VGL at (walker, electron) points -> vglc (all electrons).
template <int NOB>
__global__ __launch_bounds__(NTHREADS) void k_orbitals_all(DevCtx c) {
  __shared__ double Bs[FMAX * NCOL];
  __shared__ double out[TW * 5 * NOB * 16];
  __shared__ double pts[TW][3];
  const int npts = c.Wpad * c.ne;
  const int p0 = blockIdx.x * TW;
  if (threadIdx.x < TW * 3) {
    const int p = min(p0 + (int)threadIdx.x / 3, npts - 1);
    pts[threadIdx.x / 3][threadIdx.x % 3] = c.R[(size_t)p * 3 + threadIdx.x % 3];
  }
  __syncthreads();
  mo_tile<double, NOB>(c, pts, Bs, out);
  constexpr int NP = NOB * 16;
  for (int i = threadIdx.x; i < TW * 5 * NP; i += NTHREADS) {
    const int w = i / (5 * NP);
    const int p = p0 + w;
    if (p < npts) c.vglc[(size_t)p * 5 * NP + (i - w * 5 * NP)] = out[i];
  }
}

// Orbital VGL at one point per walker: pos [W][3] -> dst [W][5][NP].
template <int NOB>
__global__ __launch_bounds__(NTHREADS) void k_orbitals_at(DevCtx c, const double *pos, int npts,
                                                          double *dst) {
  __shared__ double Bs[FMAX * NCOL];
  __shared__ double out[TW * 5 * NOB * 16];
  __shared__ double pts[TW][3];
  const int p0 = blockIdx.x * TW;
  if (threadIdx.x < TW * 3) {
    const int p = min(p0 + (int)threadIdx.x / 3, npts - 1);
    pts[threadIdx.x / 3][threadIdx.x % 3] = pos[(size_t)p * 3 + threadIdx.x % 3];
  }
  __syncthreads();
  mo_tile<double, NOB>(c, pts, Bs, out);
  constexpr int NP = NOB * 16;
  for (int i = threadIdx.x; i < TW * 5 * NP; i += NTHREADS) {
    const int w = i / (5 * NP);
    if (p0 + w < npts) dst[(size_t)(p0 + w) * 5 * NP + (i - w * 5 * NP)] = out[i];
  }
}

// FP64 inverse of each walker's Slater matrix by in-place Gauss-Jordan
// elimination with partial pivoting, built from the cached value rows.
// grid (Wpad, 2); dynamic LDS n*n doubles.  Writes GT (transposed, zero
// padded), log|det| and sign; flags singular matrices.
__global__ __launch_bounds__(NTHREADS) void k_inverse(DevCtx c) {
  extern __shared__ double A[];
  __shared__ int piv[128];
  __shared__ double fcol[128];
  __shared__ double pv_val[NTHREADS / 64];
  __shared__ int pv_idx[NTHREADS / 64];
  __shared__ double s_logdet;
  __shared__ int s_sign, s_sing;
  const int w = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? c.n_up : c.n_dn;
  const int NP = c.NP;
  const int tid = threadIdx.x;
  double *GT = c.GT + gt_off(c, w, sp);
  if (n == 0) {
    for (int i = tid; i < NP * NP; i += NTHREADS) GT[i] = 0.0;
    if (tid == 0) { c.logdet[w * 2 + sp] = 0.0; c.sgn[w * 2 + sp] = 1.0; }
    return;
  }
  const int e0 = sp == 0 ? 0 : c.n_up;
  for (int i = tid; i < n * n; i += NTHREADS) {
    const int r = i / n, j = i % n;
    A[i] = c.vglc[vglc_off(c, w, e0 + r) + j];
  }
  if (tid == 0) { s_logdet = 0.0; s_sign = 1; s_sing = 0; }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot search over rows k..n-1 of column k
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += NTHREADS) {
      const double v = fabs(A[i * n + k]);
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((tid & 63) == 0) { pv_val[tid >> 6] = best; pv_idx[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = pv_val[0];
      int p = pv_idx[0];
      for (int q = 1; q < NTHREADS / 64; ++q)
        if (pv_val[q] > b || (pv_val[q] == b && pv_idx[q] < p)) { b = pv_val[q]; p = pv_idx[q]; }
      piv[k] = p;
      if (p != k) s_sign = -s_sign;
      const double d = A[p * n + k];
      if (d == 0.0) s_sing = 1;
      else {
        if (d < 0.0) s_sign = -s_sign;
        s_logdet += log(fabs(d));
      }
    }
    __syncthreads();
    if (s_sing) break;
    const int p = piv[k];
    if (p != k)
      for (int j = tid; j < n; j += NTHREADS) {
        const double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    __syncthreads();
    const double dinv = 1.0 / A[k * n + k];
    for (int r = tid; r < n; r += NTHREADS) fcol[r] = A[r * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += NTHREADS) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * dinv;
    __syncthreads();
    for (int i = tid; i < n * n; i += NTHREADS) {
      const int r = i / n, j = i % n;
      if (r == k) continue;
      A[i] = (j == k ? 0.0 : A[i]) - fcol[r] * A[k * n + j];
    }
    __syncthreads();
  }
  if (s_sing) {
    if (tid == 0) {
      c.logdet[w * 2 + sp] = -INFINITY;
      c.sgn[w * 2 + sp] = 0.0;
      c.flags[w] |= 2u;
    }
    return;
  }
  // undo the row exchanges: swap columns in reverse order
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int r = tid; r < n; r += NTHREADS) {
        const double t = A[r * n + k];
        A[r * n + k] = A[r * n + p];
        A[r * n + p] = t;
      }
    __syncthreads();
  }
  // GT[b][j] = Ainv[j][b]
  for (int i = tid; i < NP * NP; i += NTHREADS) {
    const int b = i / NP, j = i % NP;
    GT[i] = (b < n && j < n) ? A[j * n + b] : 0.0;
  }
  if (tid == 0) {
    c.logdet[w * 2 + sp] = s_logdet;
    c.sgn[w * 2 + sp] = (double)s_sign;
  }
}

// Local energy of each walker from the cached orbital rows and inverses:
//   E_L = -1/2 sum_i [lap_i J + |grad_i J|^2 + 2 grad_i J . g_i + l_i] + V,
//   g_i = sum_j grad phi_j(r_i) A^{-1}_{j i},  l_i = sum_j lap phi_j(r_i) A^{-1}_{j i}.
// One workgroup per walker.  mode: -1 = measure only, 0 = VMC step, 1 = DMC
// step (log w += -tau ((E_old + E_new)/2 - E_T)).
__global__ __launch_bounds__(NTHREADS) void k_local_energy(DevCtx c, int mode, double e_trial,
                                                           double *e_log_row) {
  __shared__ double part[NTHREADS / 64][3];
  const int w = blockIdx.x;
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int NP = c.NP;
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  double kin = 0.0, pot = 0.0, jv = 0.0;
  for (int i = wid; i < c.ne; i += NTHREADS / 64) {
    const int sp = i < c.n_up ? 0 : 1, ii = i - sp * c.n_up;
    const double *row = c.vglc + vglc_off(c, w, i);
    const double *gcol = c.GT + gt_off(c, w, sp) + (size_t)ii * NP;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0;
    for (int j = lane; j < NP; j += 64) {
      const double gj = gcol[j];
      g0 += row[NP + j] * gj;
      g1 += row[2 * NP + j] * gj;
      g2 += row[3 * NP + j] * gj;
      l += row[4 * NP + j] * gj;
    }
    // Jastrow gradient / Laplacian, value (pairs counted once) and potential
    const double *ri = Rw + 3 * i;
    double jg0 = 0.0, jg1 = 0.0, jg2 = 0.0, jl = 0.0, ju = 0.0, v = 0.0;
    for (int j = lane; j < c.ne + c.n_atom; j += 64) {
      const double *p;
      double a, b, q;
      bool ee = j < c.ne;
      if (ee) {
        if (j == i) continue;
        p = Rw + 3 * j;
        a = ((j < c.n_up ? 0 : 1) == sp) ? c.jee_para : c.jee_anti;
        b = c.jee_b;
        q = 0.5;  // each e-e pair is visited twice
      } else {
        const int A = j - c.ne;
        p = c.ion + 3 * A;
        a = c.jen_a[A];
        b = c.jen_b;
        q = 1.0;
      }
      const double dx = ri[0] - p[0], dy = ri[1] - p[1], dz = ri[2] - p[2];
      const double rr = sqrt(dx * dx + dy * dy + dz * dz);
      const Pade pd = pade(a, b, rr);
      const double f = pd.d1 / rr;
      jg0 += f * dx;
      jg1 += f * dy;
      jg2 += f * dz;
      jl += pd.d2 + 2.0 * f;
      ju += q * pd.u;
      v += ee ? 0.5 / rr : -c.Z[j - c.ne] / rr;
    }
    g0 = sum64(g0); g1 = sum64(g1); g2 = sum64(g2); l = sum64(l);
    jg0 = sum64(jg0); jg1 = sum64(jg1); jg2 = sum64(jg2); jl = sum64(jl);
    ju = sum64(ju); v = sum64(v);
    kin += jl + jg0 * jg0 + jg1 * jg1 + jg2 * jg2 + 2.0 * (jg0 * g0 + jg1 * g1 + jg2 * g2) + l;
    pot += v;
    jv += ju;
  }
  if (lane == 0) { part[wid][0] = kin; part[wid][1] = pot; part[wid][2] = jv; }
  __syncthreads();
  if (tid == 0) {
    double K = 0.0, V = 0.0, J = 0.0;
    for (int q = 0; q < NTHREADS / 64; ++q) { K += part[q][0]; V += part[q][1]; J += part[q][2]; }
    const double e = -0.5 * K + V + c.v_nn;
    const double eold = c.eloc[w];
    if (mode == 1) c.logw[w] += -c.tau * (0.5 * (eold + e) - e_trial);
    c.eloc[w] = e;
    c.logpsi[w] = J + c.logdet[w * 2] + c.logdet[w * 2 + 1];
    if (!isfinite(e) || !isfinite(c.logpsi[w])) c.flags[w] |= 1u;
    if (e_log_row && w < c.W) e_log_row[w] = e;
  }
}

// One full sweep: every electron of every walker in the tile proposes a
// drift-diffusion move r' = r + tau v + sqrt(tau) chi, is accepted with the
// Metropolis-Hastings probability (fixed node: DMC rejects sign changes),
// and accepted moves enter a delayed update of the inverse: within a block
// of k consecutive electrons of one spin, the block's inverse columns are
// updated by Sherman-Morrison, and at the block end the full inverse takes
// all k changes at once (rank-k Woodbury form, see flush_block).
template <int NOB>
__global__ __launch_bounds__(NTHREADS) void k_sweep(DevCtx c, int mode, uint32_t step,
                                                    uint8_t *acc_log /* [W][ne] or null */) {
  constexpr int NP = NOB * 16;
  __shared__ double Bs[FMAX * NCOL];
  __shared__ double vnew[TW * 5 * NP];
  __shared__ double colm[TW][NP];
  __shared__ double aold[TW][NP];
  __shared__ double pts[TW][3];
  __shared__ double s_v[TW][3];
  __shared__ double s_uacc[TW], s_uold[TW], s_rho[TW];
  __shared__ int s_acc[TW];
  const int tid = threadIdx.x;
  const int ws = tid >> 5, t = tid & 31;
  const int w = blockIdx.x * TW + ws;
  double *Rw = c.R + (size_t)w * c.ne * 3;
  double *Gb = c.Gb + blk_off(c, w);
  double *Dl = c.Dl + blk_off(c, w);
  const double tau = c.tau, sqt = sqrt(c.tau);
  for (int i = 0; i < c.ne; ++i) {
    const int sp = i < c.n_up ? 0 : 1;
    const int ii = i - sp * c.n_up;
    const int nsig = sp == 0 ? c.n_up : c.n_dn;
    const int m = ii % c.K, b0 = ii - m;
    const int kb = min(c.K, nsig - b0);
    double *GT = c.GT + gt_off(c, w, sp);
    if (m == 0) {
      // block start: copy the block's inverse columns
      for (int b = 0; b < kb; ++b)
        for (int j = t; j < NP; j += 32) Gb[b * NP + j] = GT[(size_t)(b0 + b) * NP + j];
    }
    // ---- P1: drift at the current position, proposal
    const double *row = c.vglc + vglc_off(c, w, i);
    double gd0 = 0.0, gd1 = 0.0, gd2 = 0.0;
    for (int j = t; j < NP; j += 32) {
      const double gj = Gb[m * NP + j];
      colm[ws][j] = gj;
      aold[ws][j] = row[j];
      gd0 += row[NP + j] * gj;
      gd1 += row[2 * NP + j] * gj;
      gd2 += row[3 * NP + j] * gj;
    }
    double ro[3] = {Rw[3 * i], Rw[3 * i + 1], Rw[3 * i + 2]};
    double uo = 0.0, gj[3] = {0.0, 0.0, 0.0};
    jastrow_one_partial(c, Rw, i, ro, t, 32, uo, gj);
    gd0 = sum32(gd0); gd1 = sum32(gd1); gd2 = sum32(gd2);
    uo = sum32(uo); gj[0] = sum32(gj[0]); gj[1] = sum32(gj[1]); gj[2] = sum32(gj[2]);
    if (t == 0) {
      const double v[3] = {gj[0] + gd0, gj[1] + gd1, gj[2] + gd2};
      double chi[3], ua;
      move_draws(c.seed, step, (uint32_t)w, (uint32_t)i, chi, ua);
      for (int x = 0; x < 3; ++x) {
        pts[ws][x] = ro[x] + tau * v[x] + sqt * chi[x];
        s_v[ws][x] = v[x];
      }
      s_uacc[ws] = ua;
      s_uold[ws] = uo;
    }
    __syncthreads();
    // ---- P2: orbitals at the proposed positions (MFMA)
    mo_tile<double, NOB>(c, pts, Bs, vnew);
    // ---- P3: ratio, new drift, Metropolis-Hastings decision
    const double *vw = vnew + ws * 5 * NP;
    double rho = 0.0, gn0 = 0.0, gn1 = 0.0, gn2 = 0.0;
    for (int j = t; j < NP; j += 32) {
      const double gjj = colm[ws][j];
      rho += vw[j] * gjj;
      gn0 += vw[NP + j] * gjj;
      gn1 += vw[2 * NP + j] * gjj;
      gn2 += vw[3 * NP + j] * gjj;
    }
    const double rn[3] = {pts[ws][0], pts[ws][1], pts[ws][2]};
    double un = 0.0, gjn[3] = {0.0, 0.0, 0.0};
    jastrow_one_partial(c, Rw, i, rn, t, 32, un, gjn);
    rho = sum32(rho); gn0 = sum32(gn0); gn1 = sum32(gn1); gn2 = sum32(gn2);
    un = sum32(un); gjn[0] = sum32(gjn[0]); gjn[1] = sum32(gjn[1]); gjn[2] = sum32(gjn[2]);
    int accepted = 0;
    if (!(mode == 1 && !(rho > 0.0))) {
      const double vn[3] = {gjn[0] + gn0 / rho, gjn[1] + gn1 / rho, gjn[2] + gn2 / rho};
      double fwd = 0.0, bwd = 0.0;
      for (int x = 0; x < 3; ++x) {
        const double a = rn[x] - ro[x] - tau * s_v[ws][x];
        const double b = ro[x] - rn[x] - tau * vn[x];
        fwd += a * a;
        bwd += b * b;
      }
      const double lnq = 2.0 * (log(fabs(rho)) + (un - s_uold[ws])) + (fwd - bwd) / (2.0 * tau);
      const double p = lnq >= 0.0 ? 1.0 : exp(lnq);
      accepted = s_uacc[ws] < p;
    }
    if (!isfinite(rho)) c.flags[w] |= 1u;
    // ---- P4: delayed update of the block (lanes of this walker only)
    if (accepted) {
      const double irho = 1.0 / rho;
      constexpr int NJ = (NP + 31) / 32;
      double dlt[NJ];
#pragma unroll
      for (int q = 0; q < NJ; ++q) {
        const int j = t + 32 * q;
        dlt[q] = j < NP ? vw[j] - aold[ws][j] : 0.0;
        if (j < NP) Dl[m * NP + j] = dlt[q];
      }
      for (int b = m + 1; b < kb; ++b) {
        double z = 0.0;
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
          const int j = t + 32 * q;
          if (j < NP) z += dlt[q] * Gb[b * NP + j];
        }
        z = sum32(z) * irho;
        for (int j = t; j < NP; j += 32) Gb[b * NP + j] -= z * colm[ws][j];
      }
      for (int j = t; j < NP; j += 32) Gb[m * NP + j] = colm[ws][j] * irho;
      double *dst = c.vglc + vglc_off(c, w, i);
      for (int j = t; j < 5 * NP; j += 32) dst[j] = vw[j];
      if (t < 3) Rw[3 * i + t] = rn[t];
      if (t == 0) {
        c.logdet[w * 2 + sp] += log(fabs(rho));
        if (rho < 0.0) c.sgn[w * 2 + sp] = -c.sgn[w * 2 + sp];
      }
    } else {
      for (int j = t; j < NP; j += 32) Dl[m * NP + j] = 0.0;
    }
    if (acc_log && t == 0 && w < c.W) acc_log[(size_t)w * c.ne + i] = (uint8_t)accepted;
    // ---- P5: block end -> rank-k flush of the full inverse
    if (m == kb - 1) {
      __syncthreads();
      // Z[l][b] = Dl[l] . GT[b]  (row l of Delta times the old inverse)
      double *Zs = c.Zs + blk_off(c, w);
      for (int l = 0; l < kb; ++l)
        for (int b = t; b < nsig; b += 32) {
          double z = 0.0;
          for (int j = 0; j < nsig; ++j) z += Dl[l * NP + j] * GT[(size_t)b * NP + j];
          Zs[l * NP + b] = z;
        }
      // z'_l = Z_l - sum_{p<l} (Dl[l] . u_p) z'_p, u_p = Gb[p]
      for (int l = 1; l < kb; ++l)
        for (int p = 0; p < l; ++p) {
          double cc = 0.0;
          for (int j = t; j < nsig; j += 32) cc += Dl[l * NP + j] * Gb[p * NP + j];
          cc = sum32(cc);
          for (int b = t; b < nsig; b += 32) Zs[l * NP + b] -= cc * Zs[p * NP + b];
        }
      // GT[b][:] -= sum_l z'_l[b] u_l
      for (int b = t; b < nsig; b += 32)
        for (int j = 0; j < nsig; ++j) {
          double s = 0.0;
          for (int l = 0; l < kb; ++l) s += Zs[l * NP + b] * Gb[l * NP + j];
          GT[(size_t)b * NP + j] -= s;
        }
    }
    __syncthreads();
  }
}

}  // namespace dmcx
