// Semilocal pseudopotential energy (the ccECP form of the paper's QMC runs):
// local terms beta r^(n-2) exp(-alpha r^2) added to V, and the non-local
// channels v_l(r) projected on angular momentum l about their atom.  The
// projection acts on Psi through the angular integral over the sphere of
// radius r_iA about atom A,
//   V_NL Psi / Psi = sum_l v_l(r_iA) (2l+1)/(4 pi) int dOmega P_l(cos) Psi(r')/Psi,
// taken by the 12-point icosahedral rule (weights 1/12) turned by a random
// rotation per electron and evaluation: Shoemake's quaternion from the
// Philox draws 3 and 4 of (electron, walker, step) under the run's key.
//
// Psi(r')/Psi(R) for electron e moved to r' is the determinant ratio
// sum_j phi_j(r') (A^{-1})_je times the Jastrow ratio.  With
// y_e = C (A^{-1})_{:,e} (one vector over the basis per electron, k_pp_y: an
// MFMA product of the inverse and the LCAO matrix) the determinant ratio at a
// point is the dot product of the basis values there with y_e, so a point
// costs one basis evaluation (values only) and no orbital GEMM.
//
// k_pp: one workgroup per walker.  Electron positions, rotations and the
// electrons' own Jastrow sums go to LDS; the (electron, atom) pairs within
// the atoms' cutoffs are listed electron by electron (a block scan, so the
// order is fixed); then one lane per quadrature point.  Sums are added in a
// fixed order per walker (bit-reproducible).
#pragma once
#include "kernels.h"

namespace dmcx {

constexpr int PP_MAXA = 8;  // listed (electron, atom) pairs: at most ne x min(nl atoms, 8)

// Direction q (0..11) of the icosahedral rule: the cyclic arrangements of
// (0, +-1, +-phi), normalised; bit 0 of q flips the phi entry, bit 1 the 1.
__device__ __forceinline__ void ico_dir(int q, double d[3]) {
  const double phi = 1.6180339887498948482;
  const double a = (q & 1) ? -phi : phi, b = (q & 2) ? -1.0 : 1.0;
  const double nrm = 1.0 / sqrt(1.0 + phi * phi);
  const int k = q >> 2;
  d[0] = (k == 0 ? 0.0 : (k == 1 ? b : a)) * nrm;
  d[1] = (k == 0 ? b : (k == 1 ? a : 0.0)) * nrm;
  d[2] = (k == 0 ? a : (k == 1 ? 0.0 : b)) * nrm;
}

// Rotation matrix of the unit quaternion (x, y, z, w) = (sqrt(1-u0) sin 2pi u1,
// sqrt(1-u0) cos 2pi u1, sqrt(u0) sin 2pi u2, sqrt(u0) cos 2pi u2)
// (Shoemake's uniform random rotation), row-major.
__device__ inline void pp_rotation(uint64_t seed, uint32_t step, uint32_t walker, uint32_t elec,
                                   double rot[9]) {
  const double two_pi = 6.283185307179586476925286766559;
  double u0, u1, u2, unused;
  uniform_pair(seed, step, walker, elec, 3u, u0, u1);
  uniform_pair(seed, step, walker, elec, 4u, u2, unused);
  const double s1 = sqrt(1.0 - u0), s2 = sqrt(u0);
  const double x = s1 * sin(two_pi * u1), y = s1 * cos(two_pi * u1);
  const double z = s2 * sin(two_pi * u2), w = s2 * cos(two_pi * u2);
  rot[0] = 1.0 - 2.0 * (y * y + z * z); rot[1] = 2.0 * (x * y - z * w); rot[2] = 2.0 * (x * z + y * w);
  rot[3] = 2.0 * (x * y + z * w); rot[4] = 1.0 - 2.0 * (x * x + z * z); rot[5] = 2.0 * (y * z - x * w);
  rot[6] = 2.0 * (x * z - y * w); rot[7] = 2.0 * (y * z + x * w); rot[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ __forceinline__ double legendre_pl(int l, double x) {
  return l == 0 ? 1.0 : (l == 1 ? x : (l == 2 ? 0.5 * (3.0 * x * x - 1.0) : 0.5 * (5.0 * x * x * x - 3.0 * x)));
}

// beta r^(n-2) exp(-alpha r^2), n in 0..4
__device__ __forceinline__ double pp_term(int n, double beta, double alpha, double r) {
  const double ir = 1.0 / r;
  const double pw = n == 0 ? ir * ir : (n == 1 ? ir : (n == 2 ? 1.0 : (n == 3 ? r : r * r)));
  return beta * pw * exp(-alpha * r * r);
}

// y_e = C (A^{-1})_{:,e} for every electron of walker w and spin sp, into
// Y [W][ne][ldy] (FP64, permuted basis order).  G is the inverse in the GT
// layout (row e = column e of A^{-1}, zero padded to NP = 16 NOB), of element
// type TG.  grid (W, 2), block 256, dynamic LDS NP (NP + 1) doubles: the
// block stages the spin's inverse in LDS (row stride NP + 1, so the 16 rows
// an MFMA operand reads fall in distinct banks); wave v takes the function
// tiles v, v + 4, ..., holds that tile's LCAO operand (NP / 4 registers) and
// runs the 16 x 16 MFMA tiles of every 16 electrons against it.
template <typename TG, int NOB>
__global__ __launch_bounds__(256) void k_pp_y(DevCtx c, const TG *G, double *Y, int ldy) {
  constexpr int NP = 16 * NOB, KS = NP / 4, LD = NP + 1;
  extern __shared__ double s_g[];
  const int w = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? c.n_up : c.n_dn;
  if (n == 0) return;
  const int e0 = sp == 0 ? 0 : c.n_up;
  const int Kp = c.B.Kp, lane = threadIdx.x & 63;
  const TG *Gw = G + gt_off(c, w, sp);
  for (int i = threadIdx.x; i < NP * NP; i += 256) s_g[(i / NP) * LD + i % NP] = (double)Gw[i];
  __syncthreads();
  const int ntile = (Kp + 15) / 16, nm = (n + 15) / 16;
  for (int t = wave_id(); t < ntile; t += 4) {
    const int fnl = t * 16 + (lane & 15);
    const bool fok = fnl < Kp;
    // B operand of k-step s: Cp[fn][4 s + lane / 16]
    const double *Crow = c.B.Cp + (size_t)(fok ? fnl : 0) * NP + (lane >> 4);
    double b[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) b[st] = fok ? Crow[4 * st] : 0.0;
    for (int mt = 0; mt < nm; ++mt) {
      // A operand of k-step s: G[16 mt + lane % 16][4 s + lane / 16]
      const double *arow = s_g + (size_t)(16 * mt + (lane & 15)) * LD + (lane >> 4);
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < KS; ++st) acc = mfma16x16x4(arow[4 * st], b[st], acc);
      // lane l, element r: electron 16 mt + l / 16 + 4 r, function fnl
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * mt + (lane >> 4) + 4 * r;
        if (m < n && fok) Y[((size_t)w * c.ne + e0 + m) * ldy + fnl] = acc[r];
      }
    }
  }
}

template <typename TG>
inline void launch_pp_y(int nob, const DevCtx &c, const TG *G, double *Y, int ldy, hipStream_t s) {
  const size_t lds = (size_t)16 * nob * (16 * nob + 1) * sizeof(double);
  const dim3 grid(c.W, 2);
#define DMCX_CALL(N)                                                                  \
  if (hipFuncSetAttribute((const void *)k_pp_y<TG, N>,                                \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess) \
  k_pp_y<TG, N><<<grid, dim3(256), lds, s>>>(c, G, Y, ldy)
  switch (nob) {
    case 1: DMCX_CALL(1); break;
    case 2: DMCX_CALL(2); break;
    case 3: DMCX_CALL(3); break;
    case 4: DMCX_CALL(4); break;
    case 5: DMCX_CALL(5); break;
    case 6: DMCX_CALL(6); break;
    case 7: DMCX_CALL(7); break;
    default: DMCX_CALL(8); break;
  }
#undef DMCX_CALL
}

// Basis values at p dotted with y (permuted order): sum_fn Phi_fn(p) y[fn].
// Called by every active lane of a wave, one point per lane.
__device__ inline double basis_dot(const DevBasis &B, const double p[3], const double *y) {
  double acc = 0.0;
  for (int g = 0; g < B.n_group; ++g) {
    const int4 gi = B.ginfo[g];  // (l, nprim, first permuted function, first primitive slot)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double *ctr = B.gxyz + (size_t)(g * 4 + q) * 3;
      const double dx = p[0] - ctr[0], dy = p[1] - ctr[1], dz = p[2] - ctr[2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      double rad = 0.0;
      for (int k = 0; k < gi.y; ++k) {
        const int sl = gi.w + k * 4 + q;
        // a primitive below exp(-46) (1e-20) at every point of the wave is
        // skipped by the whole wave
        const double ar = B.galpha[sl] * r2;
        if (__any(ar < 46.0)) rad += B.gcoef[sl] * exp(-ar);
      }
      const double *yq = y + gi.z + q;  // component c of shell q at gi.z + 4 c + q
      if (gi.x == 0) {
        acc += rad * yq[0];
      } else if (gi.x == 1) {
        acc += rad * (dx * yq[0] + dy * yq[4] + dz * yq[8]);
      } else {
        acc += rad * (dx * dx * yq[0] + dx * dy * yq[4] + dx * dz * yq[8] + dy * dy * yq[12] +
                      dy * dz * yq[16] + dz * dz * yq[20]);
      }
    }
  }
  return acc;
}

// J terms of electron e placed at p, summed over the other electrons (LDS
// positions s_r) and the atoms.
__device__ inline double jastrow_at(const DevCtx &c, const double *s_r, int e, const double p[3]) {
  const int se = e < c.n_up ? 0 : 1;
  double u = 0.0;
  for (int j = 0; j < c.ne; ++j) {
    if (j == e) continue;
    const double dx = p[0] - s_r[3 * j], dy = p[1] - s_r[3 * j + 1], dz = p[2] - s_r[3 * j + 2];
    const double a = ((j < c.n_up ? 0 : 1) == se) ? c.jee_para : c.jee_anti;
    u += pade(a, c.jee_b, sqrt(dx * dx + dy * dy + dz * dz)).u;
  }
  for (int A = 0; A < c.n_atom; ++A) {
    const double dx = p[0] - c.ion[3 * A], dy = p[1] - c.ion[3 * A + 1], dz = p[2] - c.ion[3 * A + 2];
    u += pade(c.jen_a[A], c.jen_b, sqrt(dx * dx + dy * dy + dz * dz)).u;
  }
  return u;
}

inline size_t pp_lds_bytes(int ne, int n_nl) {
  const int cap = ne * (n_nl < PP_MAXA ? n_nl : PP_MAXA);
  return (size_t)ne * 13 * sizeof(double) + (size_t)(cap > 0 ? cap : 1) * sizeof(int);
}

// Per-walker set-up shared by the energy and force kernels: positions to
// s_r, the rotations of electrons with pairs to s_rot, their own Jastrow
// sums to s_J, and the (electron, atom) pairs within the cutoffs to s_pair,
// electron by electron (a block scan, so the order is fixed).  Returns the
// pair count (block-uniform); *over is set when it exceeds the list.  e_loc
// receives this thread's share of the local-term energy.
__device__ inline int pp_setup(const DevCtx &c, int w, double *sm, int *s_cnt, bool &over,
                               double &e_loc) {
  const int ne = c.ne, tid = threadIdx.x;
  double *s_r = sm, *s_rot = sm + 3 * ne, *s_J = sm + 12 * ne;
  int *s_pair = (int *)(sm + 13 * ne);
  const int cap = ne * (c.pp_nl < PP_MAXA ? c.pp_nl : PP_MAXA);
  const double *Rw = c.R + (size_t)w * ne * 3;
  const uint32_t step = (uint32_t)c.run->step;
  e_loc = 0.0;
  int cnt = 0;
  if (tid < ne) {
    const double r[3] = {Rw[3 * tid], Rw[3 * tid + 1], Rw[3 * tid + 2]};
    for (int x = 0; x < 3; ++x) s_r[3 * tid + x] = r[x];
    // local terms, and the atoms whose non-local channels reach this electron
    for (int t = 0; t < c.pp_n; ++t) {
      const int4 tt = c.pp_t[t];
      if (tt.y != -1) continue;
      const double *RA = c.ion + 3 * tt.x;
      const double dx = r[0] - RA[0], dy = r[1] - RA[1], dz = r[2] - RA[2];
      const double2 ba = c.pp_ba[t];
      e_loc += pp_term(tt.z, ba.x, ba.y, sqrt(dx * dx + dy * dy + dz * dz));
    }
    for (int k = 0; k < c.pp_nl; ++k) {
      const double *RA = c.ion + 3 * c.pp_nl_atom[k];
      const double dx = r[0] - RA[0], dy = r[1] - RA[1], dz = r[2] - RA[2];
      if (sqrt(dx * dx + dy * dy + dz * dz) < c.pp_rcut[c.pp_nl_atom[k]]) ++cnt;
    }
    if (cnt) pp_rotation(c.seed, step, (uint32_t)w, (uint32_t)tid, s_rot + 9 * tid);
  }
  s_cnt[tid] = cnt;
  __syncthreads();
  // inclusive scan of the per-electron pair counts (electron order)
  for (int o = 1; o < NT_AUX; o <<= 1) {
    const int v = tid >= o ? s_cnt[tid - o] : 0;
    __syncthreads();
    s_cnt[tid] += v;
    __syncthreads();
  }
  const int npair = s_cnt[NT_AUX - 1];
  over = npair > cap;
  if (tid < ne) {
    s_J[tid] = cnt ? jastrow_at(c, s_r, tid, s_r + 3 * tid) : 0.0;
    if (!over && cnt) {
      int slot = s_cnt[tid] - cnt;
      const double r[3] = {s_r[3 * tid], s_r[3 * tid + 1], s_r[3 * tid + 2]};
      for (int k = 0; k < c.pp_nl; ++k) {
        const int A = c.pp_nl_atom[k];
        const double *RA = c.ion + 3 * A;
        const double dx = r[0] - RA[0], dy = r[1] - RA[1], dz = r[2] - RA[2];
        if (sqrt(dx * dx + dy * dy + dz * dz) < c.pp_rcut[A]) s_pair[slot++] = tid | (A << 16);
      }
    }
  }
  __syncthreads();
  return npair;
}

// Geometry of quadrature point q of pair pr: the electron e, atom A, the
// electron's offset d from the atom, its distance r, the rotated direction od,
// cos theta and the point itself.
struct PPPoint {
  int e, A;
  double d[3], r, od[3], cth, p[3];
};
__device__ __forceinline__ PPPoint pp_point(const DevCtx &c, const double *s_r,
                                            const double *s_rot, int pr, int q) {
  PPPoint P;
  P.e = pr & 0xffff;
  P.A = pr >> 16;
  const double *RA = c.ion + 3 * P.A;
  for (int x = 0; x < 3; ++x) P.d[x] = s_r[3 * P.e + x] - RA[x];
  P.r = sqrt(P.d[0] * P.d[0] + P.d[1] * P.d[1] + P.d[2] * P.d[2]);
  double o[3];
  ico_dir(q, o);
  const double *rot = s_rot + 9 * P.e;
#pragma unroll
  for (int x = 0; x < 3; ++x) P.od[x] = rot[3 * x] * o[0] + rot[3 * x + 1] * o[1] + rot[3 * x + 2] * o[2];
  P.cth = (P.od[0] * P.d[0] + P.od[1] * P.d[1] + P.od[2] * P.d[2]) / P.r;
  for (int x = 0; x < 3; ++x) P.p[x] = RA[x] + P.r * P.od[x];
  return P;
}

// Pseudopotential energy (local terms + non-local quadrature) of every walker
// into c.vps [W].  grid W, block NT_AUX (NT_AUX >= ne), dynamic LDS
// pp_lds_bytes(ne, c.pp_nl).  A walker whose listed pairs exceed the LDS list
// gets NaN (flagged by the energy kernel), never a partial sum.
__global__ __launch_bounds__(NT_AUX) void k_pp(DevCtx c, const double *Y, int ldy) {
  extern __shared__ double sm[];
  __shared__ int s_cnt[NT_AUX];
  __shared__ double red[NT_AUX / 64];
  const int ne = c.ne, w = blockIdx.x, tid = threadIdx.x;
  const double *s_r = sm, *s_rot = sm + 3 * ne, *s_J = sm + 12 * ne;
  const int *s_pair = (const int *)(sm + 13 * ne);
  bool over;
  double acc;
  const int npair = pp_setup(c, w, sm, s_cnt, over, acc);
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
      acc += f * ratio * (1.0 / 12.0);
    }
  }
  // fixed-order block sum
  double v = sum64(acc);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < NT_AUX / 64; ++k) t += red[k];
    c.vps[w] = over ? __builtin_nan("") : t;
  }
}

// Basis values and gradients at p dotted with y: val = sum Phi y,
// grad = sum grad Phi y.  Called by every active lane of a wave.
__device__ inline void basis_dot_grad(const DevBasis &B, const double p[3], const double *y,
                                      double &val, double grad[3]) {
  val = 0.0;
  grad[0] = grad[1] = grad[2] = 0.0;
  for (int g = 0; g < B.n_group; ++g) {
    const int4 gi = B.ginfo[g];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double *ctr = B.gxyz + (size_t)(g * 4 + q) * 3;
      const double dx = p[0] - ctr[0], dy = p[1] - ctr[1], dz = p[2] - ctr[2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      double rad = 0.0, rp = 0.0;  // sum c e^{-a r^2}, sum -2 a c e^{-a r^2}
      for (int k = 0; k < gi.y; ++k) {
        const int sl = gi.w + k * 4 + q;
        const double ar = B.galpha[sl] * r2;
        if (__any(ar < 46.0)) {
          const double e = B.gcoef[sl] * exp(-ar);
          rad += e;
          rp -= 2.0 * B.galpha[sl] * e;
        }
      }
      const double *yq = y + gi.z + q;
      // Phi = P rad, grad Phi = grad P rad + P rp (dx, dy, dz)
      double P = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
      if (gi.x == 0) {
        P = yq[0];
      } else if (gi.x == 1) {
        P = dx * yq[0] + dy * yq[4] + dz * yq[8];
        Px = yq[0];
        Py = yq[4];
        Pz = yq[8];
      } else {
        const double xx = yq[0], xy = yq[4], xz = yq[8], yy = yq[12], yz = yq[16], zz = yq[20];
        P = dx * dx * xx + dx * dy * xy + dx * dz * xz + dy * dy * yy + dy * dz * yz + dz * dz * zz;
        Px = 2.0 * dx * xx + dy * xy + dz * xz;
        Py = dx * xy + 2.0 * dy * yy + dz * yz;
        Pz = dx * xz + dy * yz + 2.0 * dz * zz;
      }
      val += P * rad;
      grad[0] += Px * rad + P * rp * dx;
      grad[1] += Py * rad + P * rp * dy;
      grad[2] += Pz * rad + P * rp * dz;
    }
  }
}

// J terms of electron e at p and their gradient with respect to p.
__device__ inline double jastrow_at_grad(const DevCtx &c, const double *s_r, int e,
                                         const double p[3], double g[3]) {
  const int se = e < c.n_up ? 0 : 1;
  double u = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  for (int j = 0; j < c.ne + c.n_atom; ++j) {
    if (j == e) continue;
    const bool el = j < c.ne;
    const double *x = el ? s_r + 3 * j : c.ion + 3 * (j - c.ne);
    const double dx = p[0] - x[0], dy = p[1] - x[1], dz = p[2] - x[2];
    const double rr = sqrt(dx * dx + dy * dy + dz * dz);
    const double a = el ? (((j < c.n_up ? 0 : 1) == se) ? c.jee_para : c.jee_anti) : c.jen_a[j - c.ne];
    const Pade pd = pade(a, el ? c.jee_b : c.jen_b, rr);
    u += pd.u;
    const double f = pd.d1 / rr;
    g[0] += f * dx;
    g[1] += f * dy;
    g[2] += f * dz;
  }
  return u;
}

constexpr int PP_CHUNK = 20;  // pairs per round of the force kernel (240 points)

// Hellmann-Feynman term of the pseudopotential in the ion derivative of V:
// d(V_loc + V_NL)/dR_A at fixed electrons, rotations and Psi, added to
// dv [W][n_atom][3].  Per quadrature point, with n = d / r, c = od . n,
// rho = Psi(p)/Psi(R) and g = grad_p rho:
//   -(f' n + f_c (od - c n) / r) rho + f (g - n (od . g)),
//   f = sum_l (2l+1)/12 v_l P_l(c), f' its r-derivative, f_c its c-derivative.
// The 12 points of a pair are taken by 12 lanes of one round (20 pairs per
// round) and summed through LDS in point order, the pairs of an atom in pair
// order: no atomics, bit-reproducible.  grid W, block NT_AUX, dynamic LDS
// pp_grad_lds_bytes(ne, c.pp_nl).
__global__ __launch_bounds__(NT_AUX) void k_pp_grad(DevCtx c, const double *Y, int ldy,
                                                    double *dv) {
  extern __shared__ double sm[];
  __shared__ int s_cnt[NT_AUX];
  __shared__ double s_pt[PP_CHUNK * 12][3];
  const int ne = c.ne, w = blockIdx.x, tid = threadIdx.x;
  const double *s_r = sm, *s_rot = sm + 3 * ne, *s_J = sm + 12 * ne;
  const int *s_pair = (const int *)(sm + 13 * ne);
  const int cap = ne * (c.pp_nl < PP_MAXA ? c.pp_nl : PP_MAXA);
  double *s_pv = sm + 13 * ne + (cap + 1) / 2;  // [cap][3] per-pair sums
  bool over;
  double e_unused;
  const int npair = pp_setup(c, w, sm, s_cnt, over, e_unused);
  for (int p0 = 0; p0 < npair && !over; p0 += PP_CHUNK) {
    const int pl = p0 + tid / 12;
    double v[3] = {0.0, 0.0, 0.0};
    if (tid < PP_CHUNK * 12 && pl < npair) {
      const PPPoint P = pp_point(c, s_r, s_rot, s_pair[pl], tid % 12);
      double rdet, gdet[3], gj[3];
      basis_dot_grad(c.B, P.p, Y + ((size_t)w * ne + P.e) * ldy, rdet, gdet);
      const double ej = exp(jastrow_at_grad(c, s_r, P.e, P.p, gj) - s_J[P.e]);
      const double rho = rdet * ej;
      double g[3];
      for (int x = 0; x < 3; ++x) g[x] = ej * (gdet[x] + rdet * gj[x]);
      double vl[4] = {0, 0, 0, 0}, vlp[4] = {0, 0, 0, 0};
      for (int t = 0; t < c.pp_n; ++t) {
        const int4 tt = c.pp_t[t];
        if (tt.x == P.A && tt.y >= 0) {
          const double f = pp_term(tt.z, c.pp_ba[t].x, c.pp_ba[t].y, P.r);
          vl[tt.y] += f;
          vlp[tt.y] += f * ((tt.z - 2) / P.r - 2.0 * c.pp_ba[t].y * P.r);
        }
      }
      const double cq = P.cth;
      double f = 0.0, fp = 0.0, fc = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const double Pl = legendre_pl(l, cq);
        const double dP = l == 0 ? 0.0 : (l == 1 ? 1.0 : (l == 2 ? 3.0 * cq : 0.5 * (15.0 * cq * cq - 3.0)));
        f += (2 * l + 1) / 12.0 * vl[l] * Pl;
        fp += (2 * l + 1) / 12.0 * vlp[l] * Pl;
        fc += (2 * l + 1) / 12.0 * vl[l] * dP;
      }
      const double n[3] = {P.d[0] / P.r, P.d[1] / P.r, P.d[2] / P.r};
      const double og = P.od[0] * g[0] + P.od[1] * g[1] + P.od[2] * g[2];
      for (int x = 0; x < 3; ++x)
        v[x] = -fp * n[x] * rho - fc * (P.od[x] - cq * n[x]) / P.r * rho + f * (g[x] - n[x] * og);
    }
    if (tid < PP_CHUNK * 12)
      for (int x = 0; x < 3; ++x) s_pt[tid][x] = v[x];
    __syncthreads();
    if (tid < PP_CHUNK && p0 + tid < npair)
      for (int x = 0; x < 3; ++x) {
        double t = 0.0;
        for (int q = 0; q < 12; ++q) t += s_pt[tid * 12 + q][x];
        s_pv[(p0 + tid) * 3 + x] = t;
      }
    __syncthreads();
  }
  // per atom: the local terms over electrons, then the pairs in pair order
  for (int A = tid; A < c.n_atom; A += NT_AUX) {
    double g[3] = {0.0, 0.0, 0.0};
    const double *RA = c.ion + 3 * A;
    for (int t = 0; t < c.pp_n; ++t) {
      const int4 tt = c.pp_t[t];
      if (tt.x != A || tt.y != -1) continue;
      for (int e = 0; e < ne; ++e) {
        const double d[3] = {s_r[3 * e] - RA[0], s_r[3 * e + 1] - RA[1], s_r[3 * e + 2] - RA[2]};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double f = pp_term(tt.z, c.pp_ba[t].x, c.pp_ba[t].y, r);
        const double fp = f * ((tt.z - 2) / r - 2.0 * c.pp_ba[t].y * r);
        for (int x = 0; x < 3; ++x) g[x] -= fp * d[x] / r;
      }
    }
    if (!over)
      for (int p = 0; p < npair; ++p)
        if ((s_pair[p] >> 16) == A)
          for (int x = 0; x < 3; ++x) g[x] += s_pv[p * 3 + x];
    double *o = dv + ((size_t)w * c.n_atom + A) * 3;
    for (int x = 0; x < 3; ++x) o[x] = over ? __builtin_nan("") : o[x] + g[x];
  }
}

inline size_t pp_grad_lds_bytes(int ne, int n_nl) {
  const int cap = ne * (n_nl < PP_MAXA ? n_nl : PP_MAXA);
  return (size_t)ne * 13 * sizeof(double) + (size_t)((cap + 1) / 2) * sizeof(double) +
         (size_t)(cap > 0 ? cap : 1) * 3 * sizeof(double);
}

}  // namespace dmcx
