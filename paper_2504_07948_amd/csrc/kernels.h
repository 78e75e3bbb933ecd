// dmcx kernels for gfx950.
//
// Work decomposition: a workgroup of 64*TW threads (TW = 8 walkers: 512
// threads, 8 waves) owns a tile of TW walkers.  Walkers are independent
// Markov chains, so a whole sweep (every electron of every walker in the
// tile) runs inside one launch with workgroup barriers only.  Wave `ws`
// serves walker `ws` of the tile for per-walker vector work (dot products
// over orbitals, Jastrow sums; 64-lane wave reductions); all waves
// cooperate on the orbital contraction, which is an MFMA GEMM
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

// Optional per-phase cycle accounting of the sweep (off unless the library
// is built with -DDMCX_PHASE_TIMING; used for profiling builds only).
#ifdef DMCX_PHASE_TIMING
static __device__ unsigned long long g_phase_cycles[16];
#define SUB_T(v) const unsigned long long v = __builtin_readcyclecounter()
#define SUB_ADD(slot, a, b) \
  do { if (threadIdx.x == 0) atomicAdd(&g_phase_cycles[slot], (b) - (a)); } while (0)
#define SUB_ADD_ANY(slot, a, b) atomicAdd(&g_phase_cycles[slot], (b) - (a))
#define PHASE_BEGIN() unsigned long long _ph_t = __builtin_readcyclecounter(), _ph_acc[8] = {0}
#define PHASE_MARK(id)                                        \
  do {                                                        \
    const unsigned long long _n = __builtin_readcyclecounter(); \
    _ph_acc[id] += _n - _ph_t;                                \
    _ph_t = _n;                                               \
  } while (0)
#define PHASE_END()                                                            \
  do {                                                                         \
    if (threadIdx.x == 0)                                                      \
      for (int _q = 0; _q < 8; ++_q) atomicAdd(&g_phase_cycles[_q], _ph_acc[_q]); \
  } while (0)
#else
#define SUB_T(v) do {} while (0)
#define SUB_ADD(slot, a, b) do {} while (0)
#define SUB_ADD_ANY(slot, a, b) do {} while (0)
#define PHASE_BEGIN() do {} while (0)
#define PHASE_MARK(id) do {} while (0)
#define PHASE_END() do {} while (0)
#endif

// Walkers (or points) per workgroup tile: 8 (one workgroup of 8 waves per
// CU at 2048 walkers) or 4 (two workgroups of 4 waves per CU, whose
// latency-bound per-walker phases overlap each other's orbital tiles).
#ifndef DMCX_TW
#define DMCX_TW 8
#endif
constexpr int TW = DMCX_TW;
static_assert(TW == 4 || TW == 8, "tile width");
constexpr int NVALID = 5 * TW;              // MFMA columns in use: 5 VGL rows per walker
constexpr int NCB = (NVALID + 15) / 16;     // 16-column MFMA blocks (3 or 2)
constexpr int NCOL = 16 * NCB;              // padded column count (48 or 32)
constexpr int NPV = NCOL;                   // values-only tile: one point per column
constexpr int NT_TILE = 64 * TW;            // tile kernels: one wave per walker
constexpr int NW_TILE = TW;
constexpr int NKH = NW_TILE / 4;            // K-parity groups of the orbital tile (2 or 1)
// Tile kernels keep two waves per SIMD (at most 256 registers per lane), so
// that two four-wave workgroups can share a CU.
#define DMCX_TILE_KERNEL __global__ __launch_bounds__(NT_TILE) __attribute__((amdgpu_waves_per_eu(2)))
// The FP32 single-determinant sweep: four waves per SIMD (128 registers,
// some spilled) and half-depth basis stages (half the LDS), so two 8-walker
// workgroups share a CU and one's latency-bound per-walker phases overlap
// the other's orbital tile.
#define DMCX_TILE_KERNEL_W4 \
  __global__ __launch_bounds__(NT_TILE) __attribute__((amdgpu_waves_per_eu(4)))
constexpr int NT_AUX = 256;  // per-walker kernels (inverse, local energy)
constexpr int KMAX = 64;         // largest delay rank
constexpr int MSD_NV_MAX = 144;  // virtual orbitals of a multideterminant expansion

// K-steps (4 basis functions each) per LDS stage of the orbital tile; the
// LCAO operands of a stage are held in registers, so wider orbital tiles use
// shorter stages.  This is the capacity every kernel sizes its buffers for;
// a context packs its stages for its sweep kernel (stage_ksteps, or half of
// it for the FP32 single-determinant sweep), never deeper.
__host__ __device__ constexpr int stage_ksteps(int nob) {
  return NKH == 2 ? (nob <= 4 ? 24 : 12) : (nob <= 4 ? 12 : 6);
}

// Basis work of one shell is split into this many lane tasks (s and p: the
// whole shell; d: components {xx, xy, xz} and {yy, yz, zz}).  Every task
// evaluates its shell's radial part, so fewer tasks per shell means fewer
// repeated exponentials; a stage still fits one task per thread.
__host__ __device__ constexpr int shell_split(int l) { return l == 2 ? 2 : 1; }

// Largest number of 4-shell groups of angular momentum l in one stage, so
// that a stage has at most one basis task per thread and fits the stage's
// register-held LCAO operands.
__host__ __device__ constexpr int stage_ksteps_w4(int nob) { return stage_ksteps(nob) / 2; }
// groups of one (l, nprim) type per stage of ks K-steps (every task of a
// stage gets a thread of its own)
__host__ __device__ constexpr int stage_max_groups(int l, int ks) {
  return (NT_TILE / (TW * 4 * shell_split(l))) < (ks / (l == 0 ? 1 : (l == 1 ? 3 : 6)))
             ? (NT_TILE / (TW * 4 * shell_split(l)))
             : (ks / (l == 0 ? 1 : (l == 1 ? 3 : 6)));
}

struct DevBasis {
  int n_group;
  const int4 *ginfo;     // per group: (l, nprim, first permuted function, first prim slot)
  const double *gxyz;    // [n_group*4][3] shell centres
  const double *galpha;  // prim slot + p*4 + shell
  const double *gcoef;
  const int *gatom;      // [n_group*4] atom of each shell, -1 for padding
  int n_stage;
  const int2 *stages;    // [n_stage] (first group, end group)
  int n_slot;            // primitive slots (4 per primitive of each group)
  int Kp;                // permuted function count
  const double *Cp;      // [Kp][NP] permuted LCAO coefficients (zero padded)
  const float *Cp32;
};

// Shell tables staged in LDS once per launch, so that evaluating the basis
// issues no global loads (which would drain the LCAO operand prefetch).
struct BasisLDS {
  const int4 *ginfo;
  const double *xyz, *alpha, *coef;
  const int2 *stages;
};

__host__ __device__ inline size_t basis_lds_bytes(int n_group, int n_slot, int n_stage) {
  return (size_t)n_group * sizeof(int4) + ((size_t)n_group * 12 + 2 * (size_t)n_slot) * 8 +
         (size_t)n_stage * sizeof(int2);
}

__device__ inline BasisLDS stage_basis_lds(const DevBasis &B, char *smem) {
  int4 *gi = (int4 *)smem;
  double *xyz = (double *)(smem + (size_t)B.n_group * sizeof(int4));
  double *al = xyz + (size_t)B.n_group * 12;
  double *co = al + B.n_slot;
  int2 *sg = (int2 *)(co + B.n_slot);
  for (int i = threadIdx.x; i < B.n_group; i += blockDim.x) gi[i] = B.ginfo[i];
  for (int i = threadIdx.x; i < B.n_stage; i += blockDim.x) sg[i] = B.stages[i];
  for (int i = threadIdx.x; i < B.n_group * 12; i += blockDim.x) xyz[i] = B.gxyz[i];
  for (int i = threadIdx.x; i < B.n_slot; i += blockDim.x) {
    al[i] = B.galpha[i];
    co[i] = B.gcoef[i];
  }
  BasisLDS L;
  L.ginfo = gi;
  L.xyz = xyz;
  L.alpha = al;
  L.coef = co;
  L.stages = sg;
  return L;
}

// Per-context run parameters kept in device memory, so that one captured
// step (a hipGraph) stays valid across replays: kernels read the step index
// (Philox counter field, recompute phase), the mode and E_T from here, and a
// one-thread kernel advances the counters at the end of each step.
struct RunState {
  unsigned long long step;      // global step index
  long long s_in_run;           // step index within the current run (log rows)
  double e_trial;               // E_T of the DMC weight update
  int mode;                     // 0 = VMC, 1 = DMC
  int pad_;
};

// Multideterminant expansion (Eq. 2 with M > 1) by the table method.  With
// A_ij = phi_j(r_i) over the occupied orbitals and M_iv = phi_v(r_i) over
// the virtual orbitals the expansion refers to, T = A^{-1} M (orbital x
// virtual) gives every excited-determinant ratio as a minor of T:
// D_{h->v} / D_0 = T_hv and D_{h1 h2 -> v1 v2} / D_0 = T_h1v1 T_h2v2 - T_h1v2 T_h2v1
// (holes replaced in place).  A move of electron i changes T by rank one.
struct DevMsd {
  int on;                 // 0: single determinant
  int n_det;
  int nv;                 // virtual orbitals referenced (table columns)
  int ldt;                // row stride of the table
  const int *vcol;        // [nv] column of virtual v in the orbital rows
  const double *coef;     // [n_det] CI coefficients
  const int4 *dexc;       // [n_det][2] per spin {n_exc, h0 | h1 << 16, v0 | v1 << 16, 0}
  int n_lst[2];           // determinants with an excitation of spin s
  const int4 *lst[2];     // {det, n_exc, h0 | h1 << 16, v0 | v1 << 16}
  const double *lcoef[2]; // their coefficients
  int n_ref[2];           // determinants without an excitation of spin s
  const int *rlst[2];
  const double *rcoef[2];
  int max_lst;
  // Gamma = d ln S / dT of the force adjoint, gathered per entry: entry
  // (h, v) of spin s sums its contributions gcon[s][gptr[s][h nv + v] ..) in
  // determinant order, each {list index q, h', v', sign} meaning
  // sign c_q R^other_q T[h'][v'] / S (h' < 0: no table factor)
  const int *gptr[2];
  const int4 *gcon[2];
  void *Tt;               // [Wpad][2][NP][ldt] the table (working precision)
  double *Rdet;           // [Wpad][2][n_det] D_d^s / D_0^s
  double *S;              // [Wpad] sum_d c_d R_d^up R_d^dn
  double *Rnew;           // [Wpad][max_lst] proposal scratch
};

struct DevCtx {
  DevBasis B;
  int NP;                // padded orbital count (multiple of 16)
  int ne, n_up, n_dn, n_atom;
  const double *ion;     // [n_atom][3]
  const double *Z;       // [n_atom]
  const double *jen_a;   // [n_atom]
  double jen_b, jee_anti, jee_para, jee_b, v_nn;
  int W, Wpad, K, K16;  // delay rank and its multiple-of-16 padding
  int P;                // FP64 inverse recompute period (steps)
  RunState *run;        // device run parameters
  double tau;
  uint64_t seed;
  // walker state
  double *R;       // [Wpad][ne][3]
  // Arrays below hold elements of the working precision T (double for the
  // FP64 path, float for the mixed path); kernels cast them to T*.
  void *vglc;      // [Wpad][ne][5][NP] orbital VGL rows at the current positions
  void *GT;        // [Wpad][2][NP][NP]
  void *Gb;        // [Wpad][K][NP] current inverse columns of the electron block
  void *Dl;        // [Wpad][K][NP] value-row changes of the block's moves
  void *Zs;        // [Wpad][K16][NP] flush scratch: Z = Delta G0 (16-row padded)
  void *Vs;        // [Wpad][K16][NP] flush scratch: Z' = M Z
  void *Ms;        // [Wpad][K][K] M = (I + L)^{-1}, L[l][p] = Delta_l . u_p (p < l)
  double *logdet;  // [Wpad][2]
  double *sgn;     // [Wpad][2]
  double *eloc;    // [Wpad]
  double *logw;    // [Wpad]
  double *logpsi;  // [Wpad]
  double *vpot;    // [Wpad] Coulomb potential V(R) of the current configuration
  unsigned *flags; // [Wpad] bit 0 non-finite, bit 1 singular
  unsigned *nacc;  // [Wpad] moves accepted since the last estimator call
  unsigned *nprop; // [Wpad] moves proposed since the last estimator call
  DevMsd M;        // multideterminant expansion (M.on == 0: none)
  // semilocal pseudopotential (pp_n == 0: none)
  int pp_n;                  // terms
  const int4 *pp_t;          // [pp_n] (atom, l (-1 local), n, 0)
  const double2 *pp_ba;      // [pp_n] (beta, alpha)
  const double *pp_rcut;     // [n_atom]
  int pp_nl;                 // atoms with non-local channels
  const int *pp_nl_atom;     // [pp_nl] their indices, ascending
  double *vps;               // [Wpad] pseudopotential energy of the current configuration
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
__device__ __forceinline__ double texp(double x) { return exp(x); }
__device__ __forceinline__ float texp(float x) { return expf(x); }

// Cartesian monomial data for component COMP of angular momentum L.
template <int L, int COMP, typename R = double>
__device__ __forceinline__ void cart_poly_t(R x, R y, R z, R &P, R &Px, R &Py, R &Pz, R &Lp) {
  Px = 0.0; Py = 0.0; Pz = 0.0; Lp = 0.0;
  if constexpr (L == 0) { P = 1.0; }
  else if constexpr (L == 1) {
    if constexpr (COMP == 0) { P = x; Px = 1.0; }
    else if constexpr (COMP == 1) { P = y; Py = 1.0; }
    else { P = z; Pz = 1.0; }
  } else {
    if constexpr (COMP == 0) { P = x * x; Px = 2.0 * x; Lp = 2.0; }
    else if constexpr (COMP == 1) { P = x * y; Px = y; Py = x; }
    else if constexpr (COMP == 2) { P = x * z; Px = z; Pz = x; }
    else if constexpr (COMP == 3) { P = y * y; Py = 2.0 * y; Lp = 2.0; }
    else if constexpr (COMP == 4) { P = y * z; Py = z; Pz = y; }
    else { P = z * z; Pz = 2.0 * z; Lp = 2.0; }
  }
}

// VGL of one Cartesian function from the radial sums R0 = sum c e^{-a s2},
// R1 = dR/d(s2), R2 = d2R/d(s2)^2:  grad = grad P R0 + 2 r R1 P,
// lap = lap P R0 + 4 R1 (grad P . r) + P (6 R1 + 4 s2 R2).
template <typename T, int L, int COMP>
__device__ __forceinline__ void store_vgl(T *dst, T x, T y, T z, T s2, T R0, T R1, T R2) {
  T P, Px, Py, Pz, Lp;
  cart_poly_t<L, COMP, T>(x, y, z, P, Px, Py, Pz, Lp);
  const T tr = (T)2 * R1 * P;
  dst[0] = P * R0;
  dst[1] = Px * R0 + x * tr;
  dst[2] = Py * R0 + y * tr;
  dst[3] = Pz * R0 + z * tr;
  dst[4] = Lp * R0 + (T)4 * R1 * (Px * x + Py * y + Pz * z) + P * ((T)6 * R1 + (T)4 * s2 * R2);
}

// Basis values of one stage (groups g_begin..g_end, all with angular
// momentum L and NPR primitives) at the tile's points into Bs[f][w*5 + q].
// Tasks: s and p -> (point, shell); d -> (point, shell, {xx, xy, xz} or
// {yy, yz, zz}).  A task evaluates its
// shell's radial part (NPR independent exponentials) and its components.
template <typename T, int L, int NPR>
__device__ void basis_stage_t(const BasisLDS &B, int g_begin, int g_end, int fn_begin,
                              const double (*pts)[3], T *Bs, int vt, int nvt, int npr_rt = NPR) {
  constexpr int SPLIT = shell_split(L);
  const int nsh = 4 * (g_end - g_begin);
  const int ntask = TW * nsh * SPLIT;
  for (int task = vt; task < ntask; task += nvt) {
    const int w = task & (TW - 1);
    const int rest = task / TW;
    const int sl = rest % nsh, part = rest / nsh;
    const int g = g_begin + (sl >> 2), s = sl & 3;
    const int4 gi = B.ginfo[g];
    const double *cxyz = B.xyz + (size_t)(g * 4 + s) * 3;
    const T x = (T)(pts[w][0] - cxyz[0]), y = (T)(pts[w][1] - cxyz[1]), z = (T)(pts[w][2] - cxyz[2]);
    const T s2 = x * x + y * y + z * z;
    T R0 = 0, R1 = 0, R2 = 0;
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
      }
    } else {  // generic contraction depth
      for (int p = 0; p < npr_rt; ++p) {
        const T ap = (T)B.alpha[gi.w + p * 4 + s];
        const T ep = (T)B.coef[gi.w + p * 4 + s] * texp(-ap * s2);
        R0 += ep;
        R1 -= ap * ep;
        R2 += ap * ap * ep;
      }
    }
    T *base = Bs + (size_t)(gi.z - fn_begin + s) * NCOL + w * 5;  // comp 0 of this shell
    if constexpr (L == 0) {
      store_vgl<T, 0, 0>(base, x, y, z, s2, R0, R1, R2);
    } else if constexpr (L == 1) {
      store_vgl<T, 1, 0>(base, x, y, z, s2, R0, R1, R2);
      store_vgl<T, 1, 1>(base + 4 * NCOL, x, y, z, s2, R0, R1, R2);
      store_vgl<T, 1, 2>(base + 8 * NCOL, x, y, z, s2, R0, R1, R2);
    } else {
      if (part == 0) {
        store_vgl<T, 2, 0>(base, x, y, z, s2, R0, R1, R2);
        store_vgl<T, 2, 1>(base + 4 * NCOL, x, y, z, s2, R0, R1, R2);
        store_vgl<T, 2, 2>(base + 8 * NCOL, x, y, z, s2, R0, R1, R2);
      } else {
        store_vgl<T, 2, 3>(base + 12 * NCOL, x, y, z, s2, R0, R1, R2);
        store_vgl<T, 2, 4>(base + 16 * NCOL, x, y, z, s2, R0, R1, R2);
        store_vgl<T, 2, 5>(base + 20 * NCOL, x, y, z, s2, R0, R1, R2);
      }
    }
  }
}

// Dispatch a uniform stage to its (l, nprim) specialisation.
template <typename T>
__device__ void basis_stage(const BasisLDS &B, int g_begin, int g_end, int fn_begin,
                            const double (*pts)[3], T *Bs, int vt, int nvt) {
  const int4 gi = B.ginfo[g_begin];
#define DMCX_BASIS_CASE(LL, NN) \
  case LL * 16 + NN: basis_stage_t<T, LL, NN>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt); break;
  switch (gi.x * 16 + (gi.y <= 4 ? gi.y : 0)) {
    DMCX_BASIS_CASE(0, 1) DMCX_BASIS_CASE(0, 2) DMCX_BASIS_CASE(0, 3) DMCX_BASIS_CASE(0, 4)
    DMCX_BASIS_CASE(1, 1) DMCX_BASIS_CASE(1, 2) DMCX_BASIS_CASE(1, 3) DMCX_BASIS_CASE(1, 4)
    DMCX_BASIS_CASE(2, 1) DMCX_BASIS_CASE(2, 2) DMCX_BASIS_CASE(2, 3) DMCX_BASIS_CASE(2, 4)
    case 0: basis_stage_t<T, 0, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    case 16: basis_stage_t<T, 1, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    case 32: basis_stage_t<T, 2, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    default: break;
  }
#undef DMCX_BASIS_CASE
}

// Basis values only (no derivatives) of one stage at NPV points into
// Bs[f][point] (the orbital-value tile: one MFMA column per point).  A task is
// one (point, shell): its radial part once, then every Cartesian component.
template <typename T, int L, int NPR>
__device__ void basis_stage_val_t(const BasisLDS &B, int g_begin, int g_end, int fn_begin,
                                  const double (*pts)[3], T *Bs, int vt, int nvt,
                                  int npr_rt = NPR) {
  const int nsh = 4 * (g_end - g_begin);
  const int ntask = NPV * nsh;
  for (int task = vt; task < ntask; task += nvt) {
    const int pt = task % NPV, sl = task / NPV;
    const int g = g_begin + (sl >> 2), s = sl & 3;
    const int4 gi = B.ginfo[g];
    const double *cxyz = B.xyz + (size_t)(g * 4 + s) * 3;
    const T x = (T)(pts[pt][0] - cxyz[0]), y = (T)(pts[pt][1] - cxyz[1]), z = (T)(pts[pt][2] - cxyz[2]);
    const T s2 = x * x + y * y + z * z;
    T R0 = 0;
    if constexpr (NPR > 0) {
      T e[NPR];
#pragma unroll
      for (int p = 0; p < NPR; ++p) e[p] = (T)B.coef[gi.w + p * 4 + s] * texp(-(T)B.alpha[gi.w + p * 4 + s] * s2);
#pragma unroll
      for (int p = 0; p < NPR; ++p) R0 += e[p];
    } else {
      for (int p = 0; p < npr_rt; ++p)
        R0 += (T)B.coef[gi.w + p * 4 + s] * texp(-(T)B.alpha[gi.w + p * 4 + s] * s2);
    }
    T *base = Bs + (size_t)(gi.z - fn_begin + s) * NCOL + pt;  // comp 0 of this shell
    constexpr int NC = L == 0 ? 1 : (L == 1 ? 3 : 6);
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
      base[(size_t)cc * 4 * NCOL] = P * R0;
    }
  }
}

template <typename T>
__device__ void basis_stage_val(const BasisLDS &B, int g_begin, int g_end, int fn_begin,
                                const double (*pts)[3], T *Bs, int vt, int nvt) {
  const int4 gi = B.ginfo[g_begin];
#define DMCX_BASIS_CASE(LL, NN) \
  case LL * 16 + NN: basis_stage_val_t<T, LL, NN>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt); break;
  switch (gi.x * 16 + (gi.y <= 4 ? gi.y : 0)) {
    DMCX_BASIS_CASE(0, 1) DMCX_BASIS_CASE(0, 2) DMCX_BASIS_CASE(0, 3) DMCX_BASIS_CASE(0, 4)
    DMCX_BASIS_CASE(1, 1) DMCX_BASIS_CASE(1, 2) DMCX_BASIS_CASE(1, 3) DMCX_BASIS_CASE(1, 4)
    DMCX_BASIS_CASE(2, 1) DMCX_BASIS_CASE(2, 2) DMCX_BASIS_CASE(2, 3) DMCX_BASIS_CASE(2, 4)
    case 0: basis_stage_val_t<T, 0, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    case 16: basis_stage_val_t<T, 1, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    case 32: basis_stage_val_t<T, 2, 0>(B, g_begin, g_end, fn_begin, pts, Bs, vt, nvt, gi.y); break;
    default: break;
  }
#undef DMCX_BASIS_CASE
}

// Workgroup barrier that orders LDS traffic only: waits for this wave's LDS
// operations, then synchronises.  Outstanding global loads stay in flight
// (a plain __syncthreads would drain them), which lets the LCAO operands of
// a stage load while the basis is being evaluated.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt untouched
  __builtin_amdgcn_s_barrier();
}

// LCAO operands of one stage for this wave's orbital blocks and K-parity
// group kh (A operand; lane l holds C[f0 + 4 kk + l/16][ob*16 + l%16] for
// K-steps kk = NKH i + kh).
template <typename T, int NOB, int KH>
__device__ __forceinline__ void load_stage_a(const T *Cp, int fn_begin, int ob0, int kh,
                                             int kq, int col, T (&a)[(NOB + 3) / 4][KH]) {
  constexpr int NQ = (NOB + 3) / 4;
  constexpr int NP = NOB * 16;
  // Unconditional loads: the LCAO array carries zero rows past its end, so
  // K-steps past the stage and orbital blocks past NOB read valid memory
  // (mfma_stage never uses those registers), and the loads form one
  // straight run whose completion the MFMAs can wait for one at a time.
  const T *abase = Cp + (size_t)(fn_begin + 4 * kh + kq) * NP + col + ob0 * 16;
#pragma unroll
  for (int i = 0; i < KH; ++i)
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q][i] = abase[(size_t)(4 * NKH * i) * NP + 64 * q];
}

// This wave's K-steps of one stage: acc[q][cb] += A(block) * B(column block).
// B operands come from LDS one K-step ahead of the MFMAs that use them.  The
// K-step and block tests use wave-uniform values read into scalars (scalar
// branches, no exec-mask work); the look-ahead read is unconditional (every
// row it touches lies inside the stage buffer, and rows past the stage are
// never multiplied), so the unrolled K-steps need no operand copies.
template <typename T, int NOB, int KH>
__device__ __forceinline__ void mfma_stage(typename Acc4<T>::type (&acc)[(NOB + 3) / 4][NCB],
                                           const T (&a)[(NOB + 3) / 4][KH], const T *Bsb, int nk,
                                           int ob0, int kh, int kq, int col) {
  constexpr int NQ = (NOB + 3) / 4;
  const int khs = __builtin_amdgcn_readfirstlane(kh);
  const int nks = __builtin_amdgcn_readfirstlane(nk);
  const int obs = __builtin_amdgcn_readfirstlane(ob0);
  if (khs >= nks) return;
  const T *bbase = Bsb + (4 * khs + kq) * NCOL + col;
  T bv[KH][NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) bv[0][cb] = bbase[16 * cb];
#pragma unroll
  for (int i = 0; i < KH; ++i) {
    if (i + 1 < KH) {
      const T *brow = bbase + 4 * NKH * (i + 1) * NCOL;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) bv[i + 1][cb] = brow[16 * cb];
    }
    if (NKH * i + khs < nks) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (NOB % 4 == 0 || obs + 4 * q < NOB) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = mfma16x16x4(a[q][i], bv[i][cb], acc[q][cb]);
        }
      }
    }
  }
}

// Orbital VGL of the tile's TW points: out[w][q][orbital] (LDS, precision T).
// All NT_TILE threads must call.  Stages of basis functions flow through two
// LDS buffers: in each phase every wave runs its MFMAs on stage s (wave w
// owns orbital blocks w%4 (+4, ...) and the K-steps of parity w/4 when there
// are eight waves, all K-steps when there are four) and then
// all 512 threads evaluate the basis of stage s+1 into the other buffer;
// the LCAO operands of stage s+1 are requested just before the MFMAs of
// stage s, so they arrive during those MFMAs, the basis evaluation and the
// barrier.  One barrier per stage; the two K-parity partial sums are added
// once at the end.
// VAL: the tile's NPV columns are NPV points with their values only
// (basis_stage_val) instead of TW points with five VGL rows each.
template <typename T, int NOB, int KS = stage_ksteps(NOB), bool VAL = false>
__device__ void mo_tile(const DevCtx &c, const BasisLDS &BL, const double (*pts)[3], T *Bs0,
                        T *Bs1, T *out) {
  constexpr int NQ = (NOB + 3) / 4;
  constexpr int NP = NOB * 16;
  constexpr int KH = KS / NKH;
  constexpr int FM = 4 * KS;
  typedef typename Acc4<T>::type acc_t;
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  const int ob0 = wid & 3, kh = wid >> 2;
  const int kq = lane >> 4, col = lane & 15;
  const int S = c.B.n_stage;
  const T *Cp;
  if constexpr (sizeof(T) == 8) Cp = (const T *)c.B.Cp; else Cp = (const T *)c.B.Cp32;
  acc_t acc[NQ][NCB];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = acc_t{0, 0, 0, 0};
  T a0[NQ][KH], a1[NQ][KH];
  int g0, g1, fb, nk;
  auto stage_range = [&](int s) {
    const int2 sg = BL.stages[s];
    g0 = sg.x;
    g1 = sg.y;
    fb = BL.ginfo[sg.x].z;
    const int fe = sg.y < c.B.n_group ? BL.ginfo[sg.y].z : c.B.Kp;
    nk = (fe - fb) >> 2;
  };
  stage_range(0);
  load_stage_a<T, NOB, KH>(Cp, fb, ob0, kh, kq, col, a0);
  constexpr int NUSE = VAL ? NPV : NVALID;  // columns in use
  constexpr int NPADC = NCOL - NUSE;       // padding columns, zero for every stage
  if constexpr (NPADC > 0) {
    for (int i = tid; i < FM * NPADC; i += NT_TILE) {
      Bs0[(i / NPADC) * NCOL + NUSE + i % NPADC] = (T)0;
      Bs1[(i / NPADC) * NCOL + NUSE + i % NPADC] = (T)0;
    }
  }
  if constexpr (VAL) basis_stage_val<T>(BL, g0, g1, fb, pts, Bs0, tid, NT_TILE);
  else basis_stage<T>(BL, g0, g1, fb, pts, Bs0, tid, NT_TILE);
  lds_barrier();
  // The LCAO operands of stage s+1 are requested before the MFMAs of stage s
  // (their registers are free by then), so they have the MFMAs, the basis
  // evaluation and the barrier to arrive.
  for (int st = 0; st < S; st += 2) {
    {  // stage st+1 -> a1; MFMAs of stage st (a0, Bs0); basis st+1 -> Bs1
      const int nk_cur = nk;
      if (st + 1 < S) {
        stage_range(st + 1);
        load_stage_a<T, NOB, KH>(Cp, fb, ob0, kh, kq, col, a1);
      }
      SUB_T(tm0);
      mfma_stage<T, NOB, KH>(acc, a0, Bs0, nk_cur, ob0, kh, kq, col);
      SUB_T(tm1);
      if (st + 1 < S) {
        if constexpr (VAL) basis_stage_val<T>(BL, g0, g1, fb, pts, Bs1, tid, NT_TILE);
        else basis_stage<T>(BL, g0, g1, fb, pts, Bs1, tid, NT_TILE);
      }
      SUB_T(tm2);
      SUB_ADD(11, tm0, tm1);
      SUB_ADD(9, tm1, tm2);
      lds_barrier();
    }
    if (st + 1 >= S) break;
    {  // stage st+2 -> a0; MFMAs of stage st+1 (a1, Bs1); basis st+2 -> Bs0
      const int nk_cur = nk;
      if (st + 2 < S) {
        stage_range(st + 2);
        load_stage_a<T, NOB, KH>(Cp, fb, ob0, kh, kq, col, a0);
      }
      SUB_T(tm0);
      mfma_stage<T, NOB, KH>(acc, a1, Bs1, nk_cur, ob0, kh, kq, col);
      SUB_T(tm1);
      if (st + 2 < S) {
        if constexpr (VAL) basis_stage_val<T>(BL, g0, g1, fb, pts, Bs0, tid, NT_TILE);
        else basis_stage<T>(BL, g0, g1, fb, pts, Bs0, tid, NT_TILE);
      }
      SUB_T(tm2);
      SUB_ADD(11, tm0, tm1);
      SUB_ADD(9, tm1, tm2);
      lds_barrier();
    }
  }
  // sum the K-parity partial results into out
#pragma unroll
  for (int half = NKH - 1; half >= 0; --half) {
    if (kh == half) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int ob = ob0 + 4 * q;
        if (NOB % 4 == 0 || ob < NOB) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            const int n = cb * 16 + col;
            if (n < NUSE) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                T *o = out + n * NP + ob * 16 + Acc4<T>::row(kq, r);
                *o = (half == NKH - 1 ? (T)0 : *o) + (T)acc[q][cb][r];
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------- Jastrow ----
// Lane-partial sums for electron i at position r against the other
// electrons of walker positions Rw and all ions: value u and gradient g.
// BATCHED: three partners per lane and round, their loads issued before the
// arithmetic (the single-determinant sweeps); otherwise one partner per
// iteration (the multideterminant sweep, where the batched form measured
// slower).
template <bool BATCHED = false>
__device__ __forceinline__ void jastrow_one_partial(const DevCtx &c, const double *Rw, int i,
                                                    const double r[3], int t, int nt, double &u,
                                                    double g[3]) {
  if constexpr (BATCHED) {
    const int si = i < c.n_up ? 0 : 1;
    const int N = c.ne + c.n_atom;
    // three partners per lane and round: their loads go out together (a clamped
    // index and a branch-free address select), then the terms are added for
    // the partners that exist and differ from i
    for (int j0 = t; j0 < N; j0 += 3 * nt) {
      double px[3], py[3], pz[3], pa[3], pb[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int jc = min(j0 + q * nt, N - 1);
        const bool el = jc < c.ne;
        const int A = el ? 0 : jc - c.ne;
        const double *p = el ? Rw + 3 * jc : c.ion + 3 * A;
        px[q] = p[0];
        py[q] = p[1];
        pz[q] = p[2];
        const double aen = c.jen_a[A];
        pa[q] = el ? (((jc < c.n_up ? 0 : 1) == si) ? c.jee_para : c.jee_anti) : aen;
        pb[q] = el ? c.jee_b : c.jen_b;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j = j0 + q * nt;
        if (j < N && j != i) {
          const double dx = r[0] - px[q], dy = r[1] - py[q], dz = r[2] - pz[q];
          const double rr = sqrt(dx * dx + dy * dy + dz * dz);
          const Pade pd = pade(pa[q], pb[q], rr);
          const double f = pd.d1 / rr;
          u += pd.u;
          g[0] += f * dx;
          g[1] += f * dy;
          g[2] += f * dz;
        }
      }
    }
  } else {
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
}

// ------------------------------------------------------------ kernels ----
// Orbital VGL at (walker, electron) points -> vglc (all electrons).
template <typename T, int NOB>
__global__ __launch_bounds__(NT_TILE) void k_orbitals_all(DevCtx c) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Bs0[FM * NCOL], Bs1[FM * NCOL];
  __shared__ T out[TW * 5 * NP];
  __shared__ double pts[TW][3];
  const int npts = c.Wpad * c.ne;
  const int p0 = blockIdx.x * TW;
  if (threadIdx.x < TW * 3) {
    const int p = min(p0 + (int)threadIdx.x / 3, npts - 1);
    pts[threadIdx.x / 3][threadIdx.x % 3] = c.R[(size_t)p * 3 + threadIdx.x % 3];
  }
  __syncthreads();
  mo_tile<T, NOB>(c, BL, pts, Bs0, Bs1, out);
  for (int i = threadIdx.x; i < TW * 5 * NP; i += NT_TILE) {
    const int w = i / (5 * NP);
    const int p = p0 + w;
    if (p < npts) ((T *)c.vglc)[(size_t)p * 5 * NP + (i - w * 5 * NP)] = out[i];
  }
}

// Orbital VGL at one point per walker: pos [W][3] -> dst [W][5][NP].
template <typename T, int NOB>
__global__ __launch_bounds__(NT_TILE) void k_orbitals_at(DevCtx c, const double *pos, int npts,
                                                         T *dst) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Bs0[FM * NCOL], Bs1[FM * NCOL];
  __shared__ T out[TW * 5 * NP];
  __shared__ double pts[TW][3];
  const int p0 = blockIdx.x * TW;
  if (threadIdx.x < TW * 3) {
    const int p = min(p0 + (int)threadIdx.x / 3, npts - 1);
    pts[threadIdx.x / 3][threadIdx.x % 3] = pos[(size_t)p * 3 + threadIdx.x % 3];
  }
  __syncthreads();
  mo_tile<T, NOB>(c, BL, pts, Bs0, Bs1, out);
  for (int i = threadIdx.x; i < TW * 5 * NP; i += NT_TILE) {
    const int w = i / (5 * NP);
    if (p0 + w < npts) dst[(size_t)(p0 + w) * 5 * NP + (i - w * 5 * NP)] = out[i];
  }
}

// FP64 orbital values (no derivatives) of every electron of every walker,
// NPV (walker, electron) points per tile (one per MFMA column): A64[w][e][NP], the Slater
// matrices from which the mixed form takes its FP64 inverse and energy each
// step.  The working-precision value rows of vglc are refreshed from them, so
// the next sweep's delayed updates start from rows that match the inverse.
// The mixed form's stages are packed at half depth (its FP32 sweep's), so
// this kernel sizes its stage buffers for that, keeps the output tile in the
// same LDS (it is written after the last stage), and runs at four waves per
// SIMD: two workgroups share a CU, and one's basis evaluation overlaps the
// other's MFMAs.
template <typename T, int NOB>
__global__ __launch_bounds__(NT_TILE) __attribute__((amdgpu_waves_per_eu(4)))
void k_values64(DevCtx c, double *A64) {
  constexpr int NP = NOB * 16;
  constexpr int KS = stage_ksteps_w4(NOB);
  constexpr int FM = 4 * KS;
  constexpr int NBS = 2 * FM * NCOL > NPV * NP ? 2 * FM * NCOL : NPV * NP;
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ double Bsm[NBS];  // two stage buffers, then the output tile
  double *Bs0 = Bsm, *Bs1 = Bsm + FM * NCOL, *out = Bsm;
  __shared__ double pts[NPV][3];
  const int npts = c.Wpad * c.ne;
  const int p0 = blockIdx.x * NPV;
  for (int i = threadIdx.x; i < NPV * 3; i += NT_TILE) {
    const int p = min(p0 + i / 3, npts - 1);
    pts[i / 3][i % 3] = c.R[(size_t)p * 3 + i % 3];
  }
  __syncthreads();
  mo_tile<double, NOB, KS, true>(c, BL, pts, Bs0, Bs1, out);
  for (int i = threadIdx.x; i < NPV * NP; i += NT_TILE) {
    const int pl = i / NP, j = i - pl * NP, p = p0 + pl;
    if (p < npts) {
      A64[(size_t)p * NP + j] = out[i];
      ((T *)c.vglc)[(size_t)p * 5 * NP + j] = (T)out[i];
    }
  }
}

// FP64 inverse of each walker's Slater matrix by in-place Gauss-Jordan
// elimination with partial pivoting, one workgroup per matrix (the form for
// matrices wider than a wave; inverse.h has the one-wave form).  Value rows
// of precision S at rows + (w ne + e) rs.  grid (Wpad, 2); dynamic LDS n*n
// doubles.  Writes GT (transposed, zero padded), log|det| and sign, and an
// FP64 copy of the inverse to G64 if not null; flags singular matrices.
// periodic != 0: runs only at steps s = 0 (mod P) of the device step counter
// (the form captured into a step graph); periodic == 0: always.
template <typename T, typename S>
__global__ __launch_bounds__(NT_AUX) void k_inverse(DevCtx c, const S *rows, int rs, double *G64,
                                                    int periodic) {
  extern __shared__ double A[];
  __shared__ int piv[128];
  __shared__ double fcol[128];
  __shared__ double pv_val[NT_AUX / 64];
  __shared__ int pv_idx[NT_AUX / 64];
  __shared__ double s_logdet;
  __shared__ int s_sign, s_sing;
  if (periodic && (c.run->step % (unsigned long long)c.P) != 0ull) return;
  const int w = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? c.n_up : c.n_dn;
  const int NP = c.NP;
  const int tid = threadIdx.x;
  T *GT = (T *)c.GT + gt_off(c, w, sp);
  if (n == 0) {
    for (int i = tid; i < NP * NP; i += NT_AUX) {
      GT[i] = (T)0;
      if (G64) G64[gt_off(c, w, sp) + i] = 0.0;
    }
    if (tid == 0) { c.logdet[w * 2 + sp] = 0.0; c.sgn[w * 2 + sp] = 1.0; }
    return;
  }
  const int e0 = sp == 0 ? 0 : c.n_up;
  for (int i = tid; i < n * n; i += NT_AUX) {
    const int r = i / n, j = i % n;
    A[i] = (double)rows[((size_t)w * c.ne + e0 + r) * rs + j];
  }
  if (tid == 0) { s_logdet = 0.0; s_sign = 1; s_sing = 0; }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot search over rows k..n-1 of column k
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += NT_AUX) {
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
      for (int q = 1; q < NT_AUX / 64; ++q)
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
      for (int j = tid; j < n; j += NT_AUX) {
        const double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    __syncthreads();
    const double dinv = 1.0 / A[k * n + k];
    for (int r = tid; r < n; r += NT_AUX) fcol[r] = A[r * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += NT_AUX) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * dinv;
    __syncthreads();
    for (int i = tid; i < n * n; i += NT_AUX) {
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
      for (int r = tid; r < n; r += NT_AUX) {
        const double t = A[r * n + k];
        A[r * n + k] = A[r * n + p];
        A[r * n + p] = t;
      }
    __syncthreads();
  }
  // GT[b][j] = Ainv[j][b]
  double *G6 = G64 ? G64 + gt_off(c, w, sp) : nullptr;
  for (int i = tid; i < NP * NP; i += NT_AUX) {
    const int b = i / NP, j = i % NP;
    const double v = (b < n && j < n) ? A[j * n + b] : 0.0;
    GT[i] = (T)v;
    if (G6) G6[i] = v;
  }
  if (tid == 0) {
    c.logdet[w * 2 + sp] = s_logdet;
    c.sgn[w * 2 + sp] = (double)s_sign;
  }
}

// Re-evaluation of the mixed form's energy for walkers whose FP32 derivative
// rows could move E_L by more than a set bound.  The first-order change of
// E_L from relative errors u in the derivative rows B is bounded by
//   (u / 2) sum_i sum_j (|lap phi_j(r_i)| + 2 |grad_i J|_1 |grad phi_j(r_i)|_1) |G_ji|,
// with G the FP64 inverse.  Walkers above cap N_e go on a list; their
// derivative rows are then evaluated in FP64 and their E_L (and DMC weight)
// recomputed.
constexpr double ESC_U = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff
struct EscList {
  int mode;       // 0 none; 1 collect onto the list; 2 re-evaluate the listed walkers
  int *count;     // listed walkers
  int *list;      // [Wpad] walker of each list slot
  const double *gl;  // [Wpad][ne][4] FP64 (g_i, l_i) of each list slot (mode 2)
  double cap;     // bound per electron above which a walker is listed (Ha)
};

// Local energy of each walker from the cached orbital rows and inverses:
//   E_L = -1/2 sum_i [lap_i J + |grad_i J|^2 + 2 grad_i J . g_i + l_i] + V,
//   g_i = sum_j grad phi_j(r_i) A^{-1}_{j i},  l_i = sum_j lap phi_j(r_i) A^{-1}_{j i}.
// One workgroup per walker.  G64 (may be null): an FP64 copy of the inverses
// to contract with instead of GT (the mixed form's FP64 energy).
// measure_only != 0: E_L only; otherwise the end
// of a step in the run state's mode: DMC updates the log-weight
// (log w += -tau ((E_old + E_new)/2 - E_T)); e_log (may be null) receives
// E_L in row s_in_run of a table with row stride elog_stride.
// NTE threads per walker (one wave per electron at a time): 256, or 1024 for
// multideterminant systems, whose per-electron work runs over the
// determinant list.
template <typename T, int NTE = NT_AUX>
__global__ __launch_bounds__(NTE) void k_local_energy(DevCtx c, int measure_only, double *e_log,
                                                      long long elog_stride, const double *G64,
                                                      EscList esc) {
  const int mode = measure_only ? -1 : c.run->mode;
  const double e_trial = c.run->e_trial;
  double *e_log_row = (e_log && !measure_only) ? e_log + c.run->s_in_run * elog_stride : nullptr;
  __shared__ double part[NTE / 64][4];
  // MSD: w (3 rows) and y per wave; only the 1024-thread instantiation serves
  // multideterminant systems, so the others carry neither this array nor the
  // determinant-list code (fewer registers, more waves per SIMD)
  constexpr bool MSD_LE = NTE == 1024;
  __shared__ double msx_le[MSD_LE ? NTE / 64 : 1][MSD_LE ? 4 * MSD_NV_MAX : 1];
  int w = blockIdx.x;
  if (esc.mode == 2) {
    if ((int)blockIdx.x >= *esc.count) return;  // whole block
    w = esc.list[blockIdx.x];
  }
  const double *glw = esc.mode == 2 ? esc.gl + (size_t)blockIdx.x * c.ne * 4 : nullptr;
  const int tid = threadIdx.x, wid = wave_id(), lane = tid & 63;
  const int NP = c.NP;
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  // the terms linear in the pair sums (lap J, l_i, U, V) stay lane partials
  // until the end; only g_i and grad_i J, whose products enter E_L, are
  // reduced per electron
  double kin = 0.0, bound = 0.0, kin_l = 0.0, pot_l = 0.0, jv_l = 0.0;
  for (int i = wid; i < c.ne; i += NTE / 64) {
    const int sp = i < c.n_up ? 0 : 1, ii = i - sp * c.n_up;
    const T *row = (const T *)c.vglc + vglc_off(c, w, i);
    const T *gcol = (const T *)c.GT + gt_off(c, w, sp) + (size_t)ii * NP;
    const double *gcol64 = G64 ? G64 + gt_off(c, w, sp) + (size_t)ii * NP : nullptr;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0, bl = 0.0, bg = 0.0;
    if (glw) {
      if (lane == 0) {
        g0 = glw[4 * i];
        g1 = glw[4 * i + 1];
        g2 = glw[4 * i + 2];
        l = glw[4 * i + 3];
      }
    } else {
      for (int j = lane; j < NP; j += 64) {
        const double gj = gcol64 ? gcol64[j] : (double)gcol[j];
        const double r1 = (double)row[NP + j], r2 = (double)row[2 * NP + j],
                     r3 = (double)row[3 * NP + j], r4 = (double)row[4 * NP + j];
        g0 += r1 * gj;
        g1 += r2 * gj;
        g2 += r3 * gj;
        l += r4 * gj;
        if (esc.mode == 1) {
          bl += fabs(r4 * gj);
          bg += (fabs(r1) + fabs(r2) + fabs(r3)) * fabs(gj);
        }
      }
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
    g0 = sum64(g0); g1 = sum64(g1); g2 = sum64(g2);
    jg0 = sum64(jg0); jg1 = sum64(jg1); jg2 = sum64(jg2);
    double msd_k = 0.0;
    if constexpr (MSD_LE) if (c.M.on) {
      // grad_i T_hv = g_hi w_v and lap_i T_hv = g_hi y_v with
      //   w = grad m_i - T^T grad a_i,  y = lap m_i - T^T lap a_i - 2 w . grad ln D_0,
      // give grad_i S and lap_i S; per electron the kinetic sum gains
      //   2 (grad J + grad ln D_0) . grad S / S + lap S / S.
      const DevMsd &M = c.M;
      const int nsig = sp == 0 ? c.n_up : c.n_dn;
      const T *Tw = (const T *)M.Tt + ((size_t)w * 2 + sp) * NP * M.ldt;
      const double *Ro = M.Rdet + ((size_t)w * 2 + (1 - sp)) * M.n_det;
      double *sx = msx_le[wid];
      for (int q = lane; q < M.nv; q += 64) {
        const int cv = M.vcol[q];
        double w0 = (double)row[NP + cv], w1 = (double)row[2 * NP + cv], w2 = (double)row[3 * NP + cv],
               y = (double)row[4 * NP + cv];
        for (int j = 0; j < nsig; ++j) {
          const double tj = (double)Tw[(size_t)j * M.ldt + q];
          w0 -= tj * (double)row[NP + j];
          w1 -= tj * (double)row[2 * NP + j];
          w2 -= tj * (double)row[3 * NP + j];
          y -= tj * (double)row[4 * NP + j];
        }
        y -= 2.0 * (w0 * g0 + w1 * g1 + w2 * g2);
        sx[q] = w0;
        sx[MSD_NV_MAX + q] = w1;
        sx[2 * MSD_NV_MAX + q] = w2;
        sx[3 * MSD_NV_MAX + q] = y;
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      double d0 = 0.0, d1 = 0.0, d2 = 0.0, lq = 0.0;
      for (int q = lane; q < M.n_lst[sp]; q += 64) {
        const int4 e = M.lst[sp][q];
        const int n = e.y, h0 = e.z & 0xffff, h1 = (unsigned)e.z >> 16, v0 = e.w & 0xffff,
                  v1 = (unsigned)e.w >> 16;
        const double cr = M.lcoef[sp][q] * Ro[e.x];
        const double ga = (double)gcol[h0];
        if (n == 1) {
          d0 += cr * ga * sx[v0];
          d1 += cr * ga * sx[MSD_NV_MAX + v0];
          d2 += cr * ga * sx[2 * MSD_NV_MAX + v0];
          lq += cr * ga * sx[3 * MSD_NV_MAX + v0];
        } else {
          const double gb = (double)gcol[h1];
          const double t00 = (double)Tw[(size_t)h0 * M.ldt + v0], t01 = (double)Tw[(size_t)h0 * M.ldt + v1];
          const double t10 = (double)Tw[(size_t)h1 * M.ldt + v0], t11 = (double)Tw[(size_t)h1 * M.ldt + v1];
          double dr[4];
          for (int x = 0; x < 4; ++x) {
            const double a = sx[x * MSD_NV_MAX + v0], b = sx[x * MSD_NV_MAX + v1];
            // rank-one change of the 2x2 minor: the second-order cross terms cancel
            dr[x] = ga * a * t11 + t00 * gb * b - ga * b * t10 - t01 * gb * a;
          }
          d0 += cr * dr[0];
          d1 += cr * dr[1];
          d2 += cr * dr[2];
          lq += cr * dr[3];
        }
      }
      d0 = sum64(d0); d1 = sum64(d1); d2 = sum64(d2); lq = sum64(lq);
      const double iS = 1.0 / M.S[w];
      msd_k = 2.0 * ((jg0 + g0) * d0 + (jg1 + g1) * d1 + (jg2 + g2) * d2) * iS + lq * iS;
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
    }
    kin += jg0 * jg0 + jg1 * jg1 + jg2 * jg2 + 2.0 * (jg0 * g0 + jg1 * g1 + jg2 * g2) + msd_k;
    kin_l += jl + l;
    pot_l += v;
    jv_l += ju;
    if (esc.mode == 1) {
      bl = sum64(bl);
      bg = sum64(bg);
      bound += bl + 2.0 * (fabs(jg0) + fabs(jg1) + fabs(jg2)) * bg;
    }
  }
  kin += sum64(kin_l);
  const double pot = sum64(pot_l), jv = sum64(jv_l);
  if (lane == 0) { part[wid][0] = kin; part[wid][1] = pot; part[wid][2] = jv; part[wid][3] = bound; }
  __syncthreads();
  if (tid == 0) {
    double K = 0.0, V = 0.0, J = 0.0, Bd = 0.0;
    for (int q = 0; q < NTE / 64; ++q) {
      K += part[q][0]; V += part[q][1]; J += part[q][2]; Bd += part[q][3];
    }
    if (c.vps) V += c.vps[w];  // pseudopotential (local + non-local), when the system has one
    const double e = -0.5 * K + V + c.v_nn;
    if (esc.mode == 2) {
      // the walker's E_L of this step was first taken from FP32 derivative
      // rows (and entered its weight); replace it and correct the weight
      const double efirst = c.eloc[w];
      if (mode == 1) c.logw[w] += -c.tau * 0.5 * (e - efirst);
      c.eloc[w] = e;
      if (!isfinite(e)) c.flags[w] |= 1u;
      if (e_log_row && w < c.W) e_log_row[w] = e;
      return;
    }
    const double eold = c.eloc[w];
    if (mode == 1) c.logw[w] += -c.tau * (0.5 * (eold + e) - e_trial);
    c.eloc[w] = e;
    c.vpot[w] = V + c.v_nn;
    c.logpsi[w] = J + c.logdet[w * 2] + c.logdet[w * 2 + 1] + (c.M.on ? log(fabs(c.M.S[w])) : 0.0);
    if (!isfinite(e) || !isfinite(c.logpsi[w])) c.flags[w] |= 1u;
    if (e_log_row && w < c.W) e_log_row[w] = e;
    if (esc.mode == 1 && w < c.W && 0.5 * ESC_U * Bd > esc.cap * c.ne && isfinite(e))
      esc.list[atomicAdd(esc.count, 1)] = w;
  }
}

// FP64 orbital VGL of the listed walkers' electrons (TW per tile), contracted
// with their FP64 inverses into g_i = sum_j grad phi_j(r_i) G_ji and
// l_i = sum_j lap phi_j(r_i) G_ji: gl[slot][e][4].  grid: G * ceil(ne / TW)
// blocks; block b takes tile b % ntile of the slots b / ntile, + G, + 2G, ...
// up to the listed count (a few hundred blocks, not one per walker: the list
// is short and most blocks would only read the count).
template <int NOB>
__global__ __launch_bounds__(NT_TILE) void k_escalate_gl(DevCtx c, const double *G64, EscList esc) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  const int ntile = (c.ne + TW - 1) / TW;
  const int ngrp = gridDim.x / ntile, tile = blockIdx.x % ntile;
  const int count = *esc.count;
  if ((int)blockIdx.x / ntile >= count) return;  // whole block
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ double Bs0[FM * NCOL], Bs1[FM * NCOL];
  __shared__ double out[TW * 5 * NP];
  __shared__ double pts[TW][3];
  const int e0 = tile * TW;
  for (int slot = blockIdx.x / ntile; slot < count; slot += ngrp) {
    const int w = esc.list[slot];
    if (threadIdx.x < TW * 3) {
      const int e = min(e0 + (int)threadIdx.x / 3, c.ne - 1);
      pts[threadIdx.x / 3][threadIdx.x % 3] = c.R[((size_t)w * c.ne + e) * 3 + threadIdx.x % 3];
    }
    __syncthreads();
    mo_tile<double, NOB>(c, BL, pts, Bs0, Bs1, out);
    const int ws = wave_id(), t = threadIdx.x & 63;
    const int e = e0 + ws;
    if (e < c.ne) {
      const int sp = e < c.n_up ? 0 : 1, ii = e - sp * c.n_up;
      const double *gc = G64 + gt_off(c, w, sp) + (size_t)ii * NP;
      const double *o = out + ws * 5 * NP;
      double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0;
      for (int j = t; j < NP; j += 64) {
        const double gj = gc[j];
        g0 += o[NP + j] * gj;
        g1 += o[2 * NP + j] * gj;
        g2 += o[3 * NP + j] * gj;
        l += o[4 * NP + j] * gj;
      }
      g0 = sum64(g0); g1 = sum64(g1); g2 = sum64(g2); l = sum64(l);
      if (t == 0) {
        double *dst = (double *)esc.gl + ((size_t)slot * c.ne + e) * 4;
        dst[0] = g0;
        dst[1] = g1;
        dst[2] = g2;
        dst[3] = l;
      }
    }
    __syncthreads();  // pts and the tiles are rewritten by the next slot
  }
}

// One 16x16 MFMA tile in precision T: sum over k < K (multiple of 16) of A(i, k) B(k, j)
// with A(i, k) = fa(i0 + i, k) and B(k, j) = fb(k, j0 + j).  The operands of
// four K-steps are fetched before their four MFMAs, so their loads overlap.
template <typename T, typename FA, typename FB>
__device__ __forceinline__ typename Acc4<T>::type mfma_tile(int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, cl = lane & 15;
  typename Acc4<T>::type acc = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    T av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = fa(cl, k0 + 4 * u + kq);
      bv[u] = fb(k0 + 4 * u + kq, cl);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = mfma16x16x4(av[u], bv[u], acc);
  }
  return acc;
}

// Rank-k flush at the end of an electron block (delayed update).
// The block's moves were applied one by one as G_l = G_{l-1} - u_l z_l^T,
// z_l^T = Delta_l G_{l-1}, with u_l = Gb[l] (the moved electron's inverse
// column over its ratio) and Delta_l = Dl[l] (its orbital-row change, zero
// when rejected).  Expanding G_{l-1} gives z_l = Z_l - sum_{p<l} C[l][p] z_p
// with Z = Delta G0 and C[l][p] = Delta_l . u_p, so z = M Z with
// M = (I + L)^{-1} (L the strictly lower part of C).  Here: C = Dl Gb^T and
// Z = Delta G0 (MFMA GEMMs), M by forward substitution (one wave per
// walker), then Z' = M Z and G = G0 - Z'^T U (MFMA GEMMs).  A rejected move
// p leaves Gb[p] unscaled, but its C[l][p] meets only zeros: row p of M is
// e_p (Delta_p = 0) and column p of M multiplies Z[p] = 0.  Each GEMM runs
// over the tiles of all the tile's walkers at once (one barrier per phase);
// operands outside the block are read from a clamped row and zeroed by a
// select, so the K loop's loads carry no branches and can be issued ahead
// of their MFMAs.  mscr: TW K x K scratch for C and M (the sweep passes its
// free basis-tile LDS when it is large enough), or null for the global Ms.
template <typename T, int NOB>
__device__ void flush_block(const DevCtx &c, int w0, int sp, int kb, T *mscr) {
  constexpr int NP = NOB * 16;
  const int tid = threadIdx.x, wid = wave_id();
  const int lane = tid & 63, kq = lane >> 4, cl = lane & 15;
  const int K = c.K;
  const int KBP = (kb + 15) & ~15;
  const int nlt = KBP / 16;
  const int kl = kb - 1;  // last row of the block
  const int nz = nlt * NOB, nzc = nz + nlt * nlt;
  T *Mbase = mscr ? mscr : (T *)c.Ms + (size_t)w0 * K * K;
  __syncthreads();  // Dl and Gb of every walker complete
  // Z[l][b] = sum_j Dl[l][j] GT[b][j]; C[l][p] = sum_j Dl[l][j] Gb[p][j]
  // (tiles on or below the diagonal)
  for (int tt = wid; tt < TW * nzc; tt += NW_TILE) {
    const int w = w0 + tt / nzc, r = tt % nzc;
    const T *Dl = (const T *)c.Dl + blk_off(c, w);
    if (r < nz) {
      const int l0 = (r / NOB) * 16, b0 = (r % NOB) * 16;
      const T *GT = (const T *)c.GT + gt_off(c, w, sp);
      T *Zs = (T *)c.Zs + (size_t)w * c.K16 * NP;
      const auto z = mfma_tile<T>(
          NP,
          [&](int i, int k) {
            const T v = Dl[min(l0 + i, kl) * NP + k];
            return (l0 + i < kb) ? v : (T)0;
          },
          [&](int k, int j) { return GT[(size_t)(b0 + j) * NP + k]; });
#pragma unroll
      for (int q = 0; q < 4; ++q) Zs[(l0 + Acc4<T>::row(kq, q)) * NP + b0 + cl] = z[q];
    } else {
      const int l0 = ((r - nz) / nlt) * 16, p0 = ((r - nz) % nlt) * 16;
      if (p0 > l0) continue;  // wave-uniform: no barrier inside the loop
      const T *Gb = (const T *)c.Gb + blk_off(c, w);
      T *Mw = Mbase + (size_t)(w - w0) * K * K;
      const auto z = mfma_tile<T>(
          NP,
          [&](int i, int k) {
            const T v = Dl[min(l0 + i, kl) * NP + k];
            return (l0 + i < kb) ? v : (T)0;
          },
          [&](int k, int j) {
            const T v = Gb[min(p0 + j, kl) * NP + k];
            return (p0 + j < kb) ? v : (T)0;
          });
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = l0 + Acc4<T>::row(kq, q), p = p0 + cl;
        if (l < kb && p < kb) Mw[l * K + p] = z[q];
      }
    }
  }
  __syncthreads();
  // M = (I + L)^{-1} in place: wave ws takes walker w0 + ws, lane q column
  // q.  Row m needs C[m][q..m-1] and the finished rows q..m-1 of column q;
  // each lane reads only its own column of M and rows of C not yet
  // replaced, and writes row m after its reads.  Eight terms per round
  // (their loads issued together; past m the row index is clamped and the
  // weight is zero).
  {
    T *Mw = Mbase + (size_t)wid * K * K;
    const int q = lane;
    if (q < kb) Mw[q * K + q] = (T)1;
    for (int m = 1; m < kb; ++m) {
      if (q < m) {
        double s0 = 0.0, s1 = 0.0;
        for (int p0 = q; p0 < m; p0 += 8) {
          T mv[8], cv[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int pr = p0 + r < m ? p0 + r : q;
            mv[r] = Mw[pr * K + q];
            cv[r] = p0 + r < m ? Mw[m * K + pr] : (T)0;
          }
#pragma unroll
          for (int r = 0; r < 8; r += 2) {
            s0 += (double)cv[r] * (double)mv[r];
            s1 += (double)cv[r + 1] * (double)mv[r + 1];
          }
        }
        Mw[m * K + q] = (T)(-(s0 + s1));
      }
    }
  }
  __syncthreads();
  // Z'[l][b] = sum_{p <= l} M[l][p] Z[p][b]
  for (int tt = wid; tt < TW * nz; tt += NW_TILE) {
    const int w = w0 + tt / nz, r = tt % nz;
    const int l0 = (r / NOB) * 16, b0 = (r % NOB) * 16;
    const T *Ms = Mbase + (size_t)(w - w0) * K * K;
    const T *Zs = (const T *)c.Zs + (size_t)w * c.K16 * NP;
    T *Z2 = (T *)c.Vs + (size_t)w * c.K16 * NP;
    const auto z = mfma_tile<T>(
        KBP,
        [&](int i, int k) {
          const T v = Ms[min(l0 + i, kl) * K + min(k, kl)];
          return (k <= l0 + i && l0 + i < kb) ? v : (T)0;
        },
        [&](int k, int j) { return Zs[k * NP + b0 + j]; });
#pragma unroll
    for (int q = 0; q < 4; ++q) Z2[(l0 + Acc4<T>::row(kq, q)) * NP + b0 + cl] = z[q];
  }
  __syncthreads();
  // GT[b][j] -= sum_l Z'[l][b] Gb[l][j]
  for (int tt = wid; tt < TW * NOB * NOB; tt += NW_TILE) {
    const int w = w0 + tt / (NOB * NOB), r = tt % (NOB * NOB);
    const int b0 = (r / NOB) * 16, j0 = (r % NOB) * 16;
    const T *Gb = (const T *)c.Gb + blk_off(c, w);
    const T *Z2 = (const T *)c.Vs + (size_t)w * c.K16 * NP;
    T *GT = (T *)c.GT + gt_off(c, w, sp);
    const auto s = mfma_tile<T>(
        KBP, [&](int i, int k) { return Z2[k * NP + b0 + i]; },
        [&](int k, int j) {
          const T v = Gb[min(k, kl) * NP + j0 + j];
          return (k < kb) ? v : (T)0;
        });
#pragma unroll
    for (int q = 0; q < 4; ++q) GT[(size_t)(b0 + Acc4<T>::row(kq, q)) * NP + j0 + cl] -= s[q];
  }
  __syncthreads();
}

// Block update after a move of electron i (block position m of kb) of walker
// w, served by the 64 lanes t of one wave.  Accepted: Delta = a' - a_old
// enters Dl[m]; each later block row b > m is formed z_b = Delta . Gb[b] by a
// pair of lanes (one half of the row each) and takes the Sherman-Morrison
// correction Gb[b] -= z_b / rho * Gb[m]; Gb[m] becomes u_m = col / rho; the
// orbital row, position and log|D| follow.  (The coefficients
// C[m][p] = Delta_m . u_p of the earlier rows are formed at the flush, all at
// once.)  Rejected: Dl[m] = 0.
// vw: proposal VGL [5][NP]; colm: current inverse column of i (Gb[m]);
// aold: old value row of i (overwritten with Delta).
template <typename T, int NOB>
__device__ void block_accept(const DevCtx &c, int w, int t, int i, int sp, int m, int kb,
                             int accepted, double rho, const T *vw, T *colm_w, T *aold_w,
                             const double rn[3]) {
  constexpr int NP = NOB * 16;
  T *Gb = (T *)c.Gb + blk_off(c, w);
  T *Dl = (T *)c.Dl + blk_off(c, w);
  double *Rw = c.R + (size_t)w * c.ne * 3;
    if (accepted) {
      const double irho = 1.0 / rho;
      for (int j = t; j < NP; j += 64) {
        const T d = vw[j] - aold_w[j];
        aold_w[j] = d;  // aold now holds Delta (read across this walker's lanes)
        Dl[m * NP + j] = d;
      }
      // Two lanes per row: lane t takes row b0 + (t & 31), half h = t >> 5
      // (HALF entries, 16-byte loads); the half dot products meet across
      // the wave halves.  Rows of up to 64 orbitals keep their half in
      // registers between the dot product and the correction.
      constexpr int HALF = NP / 2;
      constexpr int VW = 16 / (int)sizeof(T);
      typedef T vecT __attribute__((ext_vector_type(VW)));
      constexpr bool KEEP = HALF <= 32;
      const int h = t >> 5;
      const T *dl = aold_w + h * HALF;
      const T *cm = colm_w + h * HALF;
      for (int b0 = (m + 1) & ~31; b0 < kb; b0 += 32) {
        const int b = b0 + (t & 31);
        const bool live = b < kb && b > m;
        vecT *row = (vecT *)(Gb + (size_t)(live ? b : 0) * NP + h * HALF);
        vecT keep[KEEP ? HALF / VW : 1];
        double zp = 0.0;
        if (live) {
          double za = 0.0, zb = 0.0;
#pragma unroll
          for (int q = 0; q < HALF / VW; ++q) {
            const vecT x = row[q];
            if constexpr (KEEP) keep[q] = x;
#pragma unroll
            for (int e = 0; e < VW; e += 2) {
              za += (double)dl[q * VW + e] * (double)x[e];
              zb += (double)dl[q * VW + e + 1] * (double)x[e + 1];
            }
          }
          zp = za + zb;
        }
        const double z = zp + __shfl_xor(zp, 32, 64);
        if (live) {
          const T f = (T)(z * irho);
#pragma unroll
          for (int q = 0; q < HALF / VW; ++q) {
            vecT x;
            if constexpr (KEEP) x = keep[q]; else x = row[q];
#pragma unroll
            for (int e = 0; e < VW; ++e) x[e] -= f * cm[q * VW + e];
            row[q] = x;
          }
        }
      }
      for (int j = t; j < NP; j += 64) Gb[m * NP + j] = (T)((double)colm_w[j] * irho);
      T *dst = (T *)c.vglc + vglc_off(c, w, i);
      for (int j = t; j < 5 * NP; j += 64) dst[j] = vw[j];
      if (t < 3) Rw[3 * i + t] = rn[t];
      if (t == 0) {
        c.logdet[w * 2 + sp] += log(fabs(rho));
        if (rho < 0.0) c.sgn[w * 2 + sp] = -c.sgn[w * 2 + sp];
      }
    } else {
      for (int j = t; j < NP; j += 64) Dl[m * NP + j] = (T)0;
    }
}

// Excited-determinant ratio from table entries: n = 0 -> 1, one hole -> T_hv,
// two holes -> the 2x2 minor (holes replaced in place).
__device__ __forceinline__ void msd_unpack(int4 e, int &n, int &h0, int &h1, int &v0, int &v1) {
  n = e.y;
  h0 = e.z & 0xffff;
  h1 = (unsigned)e.z >> 16;
  v0 = e.w & 0xffff;
  v1 = (unsigned)e.w >> 16;
}

// Wave-local LDS visibility: lanes of one wave read what other lanes of the
// same wave just wrote (LDS operations of a wave complete in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
}

// One full sweep: every electron of every walker in the tile proposes a
// drift-diffusion move r' = r + tau v + sqrt(tau) chi, is accepted with the
// Metropolis-Hastings probability (fixed node: DMC rejects sign changes),
// and accepted moves enter a delayed update of the inverse: within a block
// of k consecutive electrons of one spin, the block's inverse columns are
// updated by Sherman-Morrison, and at the block end the full inverse takes
// all k changes at once (rank-k Woodbury form, see flush_block).
//
// MSD (multideterminant form, Eq. 2 with M > 1): Psi = exp(J) D_0^up D_0^dn S
// with S = sum_d c_d R_d^up R_d^dn, R_d = minors of the table T = A^{-1} M.
// For a move of electron i (spin s) to r', with a', m' its occupied and
// virtual orbital rows there, g_i = column i of A^{-1} and rho_0 = a'.g_i:
//   T' = T + g_i q^T,  q = (m' - T^T a') / rho_0,
// so every R_d' follows from a few entries of T, the column g_i and q, and
// grad_{r'} T'_hv = g_hi grad q_v.  At the current position the same form
// with q = 0 gives grad_i T_hv = g_hi w_v, w = grad m_i - T^T grad a_i.
// The full ratio is rho_0 S'/S e^{dJ}; the drift adds grad S / S.  An
// accepted move applies T += g_i q^T and keeps the new R_d^s and S.
template <typename T, int NOB, bool MSD, int KS = stage_ksteps(NOB)>
__device__ __forceinline__ void sweep_body(const DevCtx &c, uint8_t *acc_log,
                                           long long acc_step_stride, int acc_w_stride,
                                           int tile) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * KS;
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Bs[2 * FM * NCOL];  // basis tiles; MSD scratch between tiles
  T *Bs0 = Bs, *Bs1 = Bs + FM * NCOL;
  __shared__ T vnew[TW * 5 * NP];
  __shared__ T colm[TW][NP];
  __shared__ T aold[TW][NP];
  __shared__ double pts[TW][3];
  __shared__ double s_v[TW][3];
  __shared__ double s_uacc[TW], s_uold[TW], s_rho[TW];
  __shared__ int s_acc[TW];
  __shared__ double s_S[TW], s_C0[TW];
  const int tid = threadIdx.x;
  const int ws = wave_id(), t = tid & 63;  // one wave per walker
  const int w = tile * TW + ws;
  double *Rw = c.R + (size_t)w * c.ne * 3;
  T *Gb = (T *)c.Gb + blk_off(c, w);
  const double tau = c.tau, sqt = sqrt(c.tau);
  const uint32_t step = (uint32_t)c.run->step;
  const int mode = c.run->mode;
  const DevMsd &M = c.M;
  // MSD scratch per walker: [4][nv] (q, grad q) or [3][nv] (w)
  T *msx = Bs + (size_t)ws * 4 * (MSD ? M.nv : 0);
  if (acc_log) acc_log += c.run->s_in_run * acc_step_stride + (long long)w * acc_w_stride;
  unsigned n_accepted = 0;  // this walker's accepted moves in the sweep
  PHASE_BEGIN();
  for (int i = 0; i < c.ne; ++i) {
    const int sp = i < c.n_up ? 0 : 1;
    const int ii = i - sp * c.n_up;
    const int nsig = sp == 0 ? c.n_up : c.n_dn;
    const int m = ii % c.K, b0 = ii - m;
    const int kb = min(c.K, nsig - b0);
    T *GT = (T *)c.GT + gt_off(c, w, sp);
    if (m == 0) {
      // block start: copy the block's inverse columns
      for (int b = 0; b < kb; ++b)
        for (int j = t; j < NP; j += 64) Gb[b * NP + j] = GT[(size_t)(b0 + b) * NP + j];
    }
    PHASE_MARK(0);
    // ---- P1: drift at the current position, proposal
    const T *row = (const T *)c.vglc + vglc_off(c, w, i);
    double gd0 = 0.0, gd1 = 0.0, gd2 = 0.0;
    for (int j = t; j < NP; j += 64) {
      const T gjt = Gb[m * NP + j];
      const double gj = (double)gjt;
      colm[ws][j] = gjt;
      aold[ws][j] = row[j];
      gd0 += (double)row[NP + j] * gj;
      gd1 += (double)row[2 * NP + j] * gj;
      gd2 += (double)row[3 * NP + j] * gj;
    }
    double ro[3] = {Rw[3 * i], Rw[3 * i + 1], Rw[3 * i + 2]};
    double uo = 0.0, gj[3] = {0.0, 0.0, 0.0};
    jastrow_one_partial<!MSD>(c, Rw, i, ro, t, 64, uo, gj);
    gd0 = sum64(gd0); gd1 = sum64(gd1); gd2 = sum64(gd2);
    uo = sum64(uo); gj[0] = sum64(gj[0]); gj[1] = sum64(gj[1]); gj[2] = sum64(gj[2]);
    double gs[3] = {0.0, 0.0, 0.0};  // grad_i S / S (MSD)
    if constexpr (MSD) {
      const T *Tw = (const T *)M.Tt + ((size_t)w * 2 + sp) * NP * M.ldt;
      const double *Ro = M.Rdet + ((size_t)w * 2 + (1 - sp)) * M.n_det;
      if (ii == 0) {
        // spin start: the determinants without an excitation of this spin
        double c0 = 0.0;
        for (int q = t; q < M.n_ref[sp]; q += 64) c0 += M.rcoef[sp][q] * Ro[M.rlst[sp][q]];
        c0 = sum64(c0);
        if (t == 0) {
          s_C0[ws] = c0;
          s_S[ws] = M.S[w];
        }
      }
      // w_v = grad m_v - sum_j T_jv grad a_j at the current position
      for (int v = t; v < M.nv; v += 64) {
        const int cv = M.vcol[v];
        double w0 = (double)row[NP + cv], w1 = (double)row[2 * NP + cv], w2 = (double)row[3 * NP + cv];
        for (int j = 0; j < nsig; ++j) {
          const double tj = (double)Tw[(size_t)j * M.ldt + v];
          w0 -= tj * (double)row[NP + j];
          w1 -= tj * (double)row[2 * NP + j];
          w2 -= tj * (double)row[3 * NP + j];
        }
        msx[v] = (T)w0;
        msx[M.nv + v] = (T)w1;
        msx[2 * M.nv + v] = (T)w2;
      }
      wave_lds_sync();
      for (int q = t; q < M.n_lst[sp]; q += 64) {
        int n, h0, h1, v0, v1;
        msd_unpack(M.lst[sp][q], n, h0, h1, v0, v1);
        const double cr = M.lcoef[sp][q] * Ro[M.lst[sp][q].x];
        const double g0 = (double)colm[ws][h0];
        double dr[3];
        if (n == 1) {
          for (int x = 0; x < 3; ++x) dr[x] = g0 * (double)msx[x * M.nv + v0];
        } else {
          const double g1 = (double)colm[ws][h1];
          const double t00 = (double)Tw[(size_t)h0 * M.ldt + v0], t01 = (double)Tw[(size_t)h0 * M.ldt + v1];
          const double t10 = (double)Tw[(size_t)h1 * M.ldt + v0], t11 = (double)Tw[(size_t)h1 * M.ldt + v1];
          for (int x = 0; x < 3; ++x) {
            const double wa = (double)msx[x * M.nv + v0], wb = (double)msx[x * M.nv + v1];
            dr[x] = g0 * wa * t11 + t00 * g1 * wb - g0 * wb * t10 - t01 * g1 * wa;
          }
        }
        for (int x = 0; x < 3; ++x) gs[x] += cr * dr[x];
      }
      gs[0] = sum64(gs[0]); gs[1] = sum64(gs[1]); gs[2] = sum64(gs[2]);
      __syncthreads();  // s_S / s_C0 of the spin start; scratch reuse below
      const double iS = 1.0 / s_S[ws];
      gs[0] *= iS; gs[1] *= iS; gs[2] *= iS;
    }
    double chi[3], ua;
    move_draws_lanes64(c.seed, step, (uint32_t)w, (uint32_t)i, t, chi, ua);
    if (t == 0) {
      const double v[3] = {gj[0] + gd0 + gs[0], gj[1] + gd1 + gs[1], gj[2] + gd2 + gs[2]};
      for (int x = 0; x < 3; ++x) {
        pts[ws][x] = ro[x] + tau * v[x] + sqt * chi[x];
        s_v[ws][x] = v[x];
      }
      s_uacc[ws] = ua;
      s_uold[ws] = uo;
    }
    __syncthreads();
    PHASE_MARK(1);
    // ---- P2: orbitals at the proposed positions (MFMA)
    mo_tile<T, NOB, KS>(c, BL, pts, Bs0, Bs1, vnew);
    PHASE_MARK(2);
    // ---- P3: ratio, new drift, Metropolis-Hastings decision
    const T *vw = vnew + ws * 5 * NP;
    double rho = 0.0, gn0 = 0.0, gn1 = 0.0, gn2 = 0.0;
    for (int j = t; j < NP; j += 64) {
      const double gjj = (double)colm[ws][j];
      rho += (double)vw[j] * gjj;
      gn0 += (double)vw[NP + j] * gjj;
      gn1 += (double)vw[2 * NP + j] * gjj;
      gn2 += (double)vw[3 * NP + j] * gjj;
    }
    const double rn[3] = {pts[ws][0], pts[ws][1], pts[ws][2]};
    double un = 0.0, gjn[3] = {0.0, 0.0, 0.0};
    jastrow_one_partial<!MSD>(c, Rw, i, rn, t, 64, un, gjn);
    rho = sum64(rho); gn0 = sum64(gn0); gn1 = sum64(gn1); gn2 = sum64(gn2);
    un = sum64(un); gjn[0] = sum64(gjn[0]); gjn[1] = sum64(gjn[1]); gjn[2] = sum64(gjn[2]);
    // rho is the reference determinant's ratio; rho_all includes S'/S (MSD)
    double rho_all = rho, gsn[3] = {0.0, 0.0, 0.0}, s_new = 0.0;
    // (MSD) a proposal where the reference determinant vanishes (every
    // orbital underflows far from the molecule) is rejected like any other
    // zero ratio; the table update would divide by it
    if constexpr (MSD) {
      const T *Tw = (const T *)M.Tt + ((size_t)w * 2 + sp) * NP * M.ldt;
      const double *Ro = M.Rdet + ((size_t)w * 2 + (1 - sp)) * M.n_det;
      const double ir = rho != 0.0 ? 1.0 / rho : 0.0;
      // q_v = (m'_v - sum_j T_jv a'_j) / rho_0, grad q_v = (grad u_v - q_v grad rho_0) / rho_0
      for (int v = t; v < M.nv; v += 64) {
        const int cv = M.vcol[v];
        double u0 = (double)vw[cv], u1 = (double)vw[NP + cv], u2 = (double)vw[2 * NP + cv],
               u3 = (double)vw[3 * NP + cv];
        for (int j = 0; j < nsig; ++j) {
          const double tj = (double)Tw[(size_t)j * M.ldt + v];
          u0 -= tj * (double)vw[j];
          u1 -= tj * (double)vw[NP + j];
          u2 -= tj * (double)vw[2 * NP + j];
          u3 -= tj * (double)vw[3 * NP + j];
        }
        const double q = u0 * ir;
        msx[v] = (T)q;
        msx[M.nv + v] = (T)((u1 - q * gn0) * ir);
        msx[2 * M.nv + v] = (T)((u2 - q * gn1) * ir);
        msx[3 * M.nv + v] = (T)((u3 - q * gn2) * ir);
      }
      wave_lds_sync();
      double sn = 0.0;
      double *Rn = M.Rnew + (size_t)w * M.max_lst;
      for (int q = t; q < M.n_lst[sp]; q += 64) {
        int n, h0, h1, v0, v1;
        msd_unpack(M.lst[sp][q], n, h0, h1, v0, v1);
        const double cr = M.lcoef[sp][q] * Ro[M.lst[sp][q].x];
        const double g0 = (double)colm[ws][h0];
        double r, dr[3];
        if (n == 1) {
          r = (double)Tw[(size_t)h0 * M.ldt + v0] + g0 * (double)msx[v0];
          for (int x = 0; x < 3; ++x) dr[x] = g0 * (double)msx[(x + 1) * M.nv + v0];
        } else {
          const double g1 = (double)colm[ws][h1];
          const double qa = (double)msx[v0], qb = (double)msx[v1];
          const double t00 = (double)Tw[(size_t)h0 * M.ldt + v0] + g0 * qa;
          const double t01 = (double)Tw[(size_t)h0 * M.ldt + v1] + g0 * qb;
          const double t10 = (double)Tw[(size_t)h1 * M.ldt + v0] + g1 * qa;
          const double t11 = (double)Tw[(size_t)h1 * M.ldt + v1] + g1 * qb;
          r = t00 * t11 - t01 * t10;
          for (int x = 0; x < 3; ++x) {
            const double da = (double)msx[(x + 1) * M.nv + v0], db = (double)msx[(x + 1) * M.nv + v1];
            dr[x] = g0 * da * t11 + t00 * g1 * db - g0 * db * t10 - t01 * g1 * da;
          }
        }
        Rn[q] = r;
        sn += cr * r;
        for (int x = 0; x < 3; ++x) gsn[x] += cr * dr[x];
      }
      s_new = s_C0[ws] + sum64(sn);
      gsn[0] = sum64(gsn[0]); gsn[1] = sum64(gsn[1]); gsn[2] = sum64(gsn[2]);
      const double iS = 1.0 / s_new;
      gsn[0] *= iS; gsn[1] *= iS; gsn[2] *= iS;
      rho_all = rho != 0.0 ? rho * (s_new / s_S[ws]) : 0.0;
    }
    int accepted = 0;
    if (!(mode == 1 && !(rho_all > 0.0))) {
      const double vn[3] = {gjn[0] + gn0 / rho + gsn[0], gjn[1] + gn1 / rho + gsn[1],
                            gjn[2] + gn2 / rho + gsn[2]};
      double fwd = 0.0, bwd = 0.0;
      for (int x = 0; x < 3; ++x) {
        const double a = rn[x] - ro[x] - tau * s_v[ws][x];
        const double b = ro[x] - rn[x] - tau * vn[x];
        fwd += a * a;
        bwd += b * b;
      }
      const double lnq = 2.0 * (log(fabs(rho_all)) + (un - s_uold[ws])) + (fwd - bwd) / (2.0 * tau);
      const double p = lnq >= 0.0 ? 1.0 : exp(lnq);
      accepted = s_uacc[ws] < p;
    }
    if (!isfinite(rho_all)) c.flags[w] |= 1u;
    PHASE_MARK(3);
    // ---- P4: delayed update of the block (lanes of this walker only)
    block_accept<T, NOB>(c, w, t, i, sp, m, kb, accepted, rho, vw, colm[ws], aold[ws], rn);
    if constexpr (MSD) {
      if (accepted) {
        // T += g_i q^T (g_i: the column before the move), keep R_d' and S'
        T *Tw = (T *)M.Tt + ((size_t)w * 2 + sp) * NP * M.ldt;
        for (int v = t; v < M.nv; v += 64) {
          const T q = msx[v];
          for (int j = 0; j < nsig; ++j) Tw[(size_t)j * M.ldt + v] += colm[ws][j] * q;
        }
        double *Rs = M.Rdet + ((size_t)w * 2 + sp) * M.n_det;
        const double *Rn = M.Rnew + (size_t)w * M.max_lst;
        for (int q = t; q < M.n_lst[sp]; q += 64) Rs[M.lst[sp][q].x] = Rn[q];
        if (t == 0) {
          s_S[ws] = s_new;
          M.S[w] = s_new;
        }
      }
    }
    if (acc_log && t == 0 && w < c.W) acc_log[i] = (uint8_t)accepted;
    n_accepted += (unsigned)accepted;
    PHASE_MARK(4);
    // ---- P5: block end -> rank-k flush of the full inverse
    // (C and M go to the basis tiles' LDS, free between moves, when they fit)
    if (m == kb - 1)
      flush_block<T, NOB>(c, tile * TW, sp, kb,
                          (size_t)TW * c.K * c.K <= (size_t)2 * FM * NCOL ? Bs : nullptr);
    PHASE_MARK(5);
    __syncthreads();
    PHASE_MARK(6);
  }
  PHASE_END();
  if (t == 0 && w < c.W) {
    c.nacc[w] += n_accepted;
    c.nprop[w] += (unsigned)c.ne;
  }
}

// The step index and mode come from the device run state; acc_log (may be
// null) receives the accept decisions at
// acc_log[s_in_run * acc_step_stride + w * acc_w_stride + i].
template <typename T, int NOB>
DMCX_TILE_KERNEL void k_sweep(DevCtx c, uint8_t *acc_log,
                                                    long long acc_step_stride, int acc_w_stride) {
  sweep_body<T, NOB, false>(c, acc_log, acc_step_stride, acc_w_stride, blockIdx.x);
}

// The FP32 single-determinant sweep (two workgroups per CU).
template <typename T, int NOB>
DMCX_TILE_KERNEL_W4 void k_sweep_w4(DevCtx c, uint8_t *acc_log, long long acc_step_stride,
                                    int acc_w_stride) {
  sweep_body<T, NOB, false, stage_ksteps_w4(NOB)>(c, acc_log, acc_step_stride, acc_w_stride,
                                                   blockIdx.x);
}

// The same sweep for a multideterminant trial function (table method).
template <typename T, int NOB>
DMCX_TILE_KERNEL void k_sweep_msd(DevCtx c, uint8_t *acc_log,
                                                        long long acc_step_stride, int acc_w_stride) {
  sweep_body<T, NOB, true>(c, acc_log, acc_step_stride, acc_w_stride, blockIdx.x);
}

// Several systems of one orbital-tile width in one launch (a group): tile t
// of the launch is walker tile tiles[t].y of system tiles[t].x, and runs
// exactly as that system's own sweep runs it.  The host lists the tiles of
// the costliest system first, so they are dispatched first.
struct SweepLog {
  uint8_t *acc;       // accept log of the system (may be null)
  long long step_ss;  // its stride between steps
  int walker_ss;      // and between walkers
};
template <typename T, int NOB, bool MSD, int KS>
__device__ __forceinline__ void sweep_multi(const DevCtx *__restrict__ cs,
                                            const int2 *__restrict__ tiles,
                                            const SweepLog *__restrict__ logs) {
  const int2 tl = tiles[blockIdx.x];
  const int sys = __builtin_amdgcn_readfirstlane(tl.x);
  const int tile = __builtin_amdgcn_readfirstlane(tl.y);
  const SweepLog lg = logs[sys];
  sweep_body<T, NOB, MSD, KS>(cs[sys], lg.acc, lg.step_ss, lg.walker_ss, tile);
}
template <typename T, int NOB>
DMCX_TILE_KERNEL void k_sweep_multi(const DevCtx *__restrict__ cs, const int2 *__restrict__ tiles,
                                    const SweepLog *__restrict__ logs) {
  sweep_multi<T, NOB, false, stage_ksteps(NOB)>(cs, tiles, logs);
}
template <typename T, int NOB>
DMCX_TILE_KERNEL_W4 void k_sweep_w4_multi(const DevCtx *__restrict__ cs,
                                          const int2 *__restrict__ tiles,
                                          const SweepLog *__restrict__ logs) {
  sweep_multi<T, NOB, false, stage_ksteps_w4(NOB)>(cs, tiles, logs);
}
template <typename T, int NOB>
DMCX_TILE_KERNEL void k_sweep_msd_multi(const DevCtx *__restrict__ cs,
                                        const int2 *__restrict__ tiles,
                                        const SweepLog *__restrict__ logs) {
  sweep_multi<T, NOB, true, stage_ksteps(NOB)>(cs, tiles, logs);
}


// ------------------------------------------- move-by-move interface ----
// The same block machinery as k_sweep, driven one call at a time by the
// caller's own proposals (dmcx_ratio_grad / dmcx_accept / dmcx_flush).

// Block start: Gb[b] = GT[b0 + b] for the block's kb electrons.
template <typename T, int NOB>
__global__ void k_block_init(DevCtx c, int sp, int b0, int kb) {
  constexpr int NP = NOB * 16;
  const int w = blockIdx.x;
  T *Gb = (T *)c.Gb + blk_off(c, w);
  const T *GT = (const T *)c.GT + gt_off(c, w, sp);
  for (int i = threadIdx.x; i < kb * NP; i += blockDim.x)
    Gb[i] = GT[(size_t)(b0 + i / NP) * NP + i % NP];
}

// Psi(R')/Psi(R) and grad_i ln|Psi(R')| for moving electron i (block
// position m) of every walker to r_new [W][3]; keeps the proposal's orbital
// VGL and determinant ratio for k_accept.
template <typename T, int NOB>
__global__ __launch_bounds__(NT_TILE) void k_ratio_grad(DevCtx c, int i, int m,
                                                        const double *r_new, double *ratio,
                                                        double *grad, T *prop, double *prop_rho) {
  constexpr int NP = NOB * 16;
  constexpr int FM = 4 * stage_ksteps(NOB);
  extern __shared__ __align__(16) char smem_basis[];
  const BasisLDS BL = stage_basis_lds(c.B, smem_basis);
  __shared__ T Bs0[FM * NCOL], Bs1[FM * NCOL];
  __shared__ T vnew[TW * 5 * NP];
  __shared__ double pts[TW][3];
  const int tid = threadIdx.x, ws = wave_id(), t = tid & 63;
  const int w = blockIdx.x * TW + ws;
  if (tid < TW * 3) {
    const int q = min((int)(blockIdx.x * TW) + tid / 3, c.W - 1);
    pts[tid / 3][tid % 3] = r_new[(size_t)q * 3 + tid % 3];
  }
  __syncthreads();
  mo_tile<T, NOB>(c, BL, pts, Bs0, Bs1, vnew);
  const T *vw = vnew + ws * 5 * NP;
  const T *col = (const T *)c.Gb + blk_off(c, w) + (size_t)m * NP;
  double rho = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int j = t; j < NP; j += 64) {
    const double cj = (double)col[j];
    rho += (double)vw[j] * cj;
    g0 += (double)vw[NP + j] * cj;
    g1 += (double)vw[2 * NP + j] * cj;
    g2 += (double)vw[3 * NP + j] * cj;
  }
  const double *Rw = c.R + (size_t)w * c.ne * 3;
  const double ro[3] = {Rw[3 * i], Rw[3 * i + 1], Rw[3 * i + 2]};
  const double rn[3] = {pts[ws][0], pts[ws][1], pts[ws][2]};
  double uo = 0.0, un = 0.0, go[3] = {0.0, 0.0, 0.0}, gn[3] = {0.0, 0.0, 0.0};
  jastrow_one_partial(c, Rw, i, ro, t, 64, uo, go);
  jastrow_one_partial(c, Rw, i, rn, t, 64, un, gn);
  rho = sum64(rho); g0 = sum64(g0); g1 = sum64(g1); g2 = sum64(g2);
  uo = sum64(uo); un = sum64(un); gn[0] = sum64(gn[0]); gn[1] = sum64(gn[1]); gn[2] = sum64(gn[2]);
  T *pw = prop + (size_t)w * 5 * NP;
  for (int j = t; j < 5 * NP; j += 64) pw[j] = vw[j];
  if (t == 0) {
    prop_rho[w] = rho;
    if (w < c.W) {
      ratio[w] = rho * exp(un - uo);
      grad[3 * w + 0] = gn[0] + g0 / rho;
      grad[3 * w + 1] = gn[1] + g1 / rho;
      grad[3 * w + 2] = gn[2] + g2 / rho;
    }
  }
}

// Apply accept[w] for the proposal of electron i (block position m of kb);
// one 64-lane block per walker.
template <typename T, int NOB>
__global__ __launch_bounds__(64) void k_accept(DevCtx c, int i, int sp, int m, int kb,
                                               const uint8_t *acc, const T *prop,
                                               const double *prop_rho, const double *r_new) {
  constexpr int NP = NOB * 16;
  __shared__ T colm[NP], aold[NP];
  const int w = blockIdx.x, t = threadIdx.x;
  const T *Gb = (const T *)c.Gb + blk_off(c, w);
  const T *row = (const T *)c.vglc + vglc_off(c, w, i);
  for (int j = t; j < NP; j += 64) {
    colm[j] = Gb[m * NP + j];
    aold[j] = row[j];
  }
  const int accepted = (w < c.W) ? (int)(acc[w] != 0) : 0;
  const double rho = prop_rho[w];
  const int q = min(w, c.W - 1);
  const double rn[3] = {r_new[3 * q], r_new[3 * q + 1], r_new[3 * q + 2]};
  if (accepted && !isfinite(rho)) c.flags[w] |= 1u;
  if (t == 0 && w < c.W) {
    c.nacc[w] += (unsigned)(accepted && rho != 0.0);
    c.nprop[w] += 1u;
  }
  block_accept<T, NOB>(c, w, t, i, sp, m, kb, accepted && rho != 0.0, rho,
                       prop + (size_t)w * 5 * NP, colm, aold, rn);
}

// Rank-k flush of the pending moves of the current block (kb of them).
template <typename T, int NOB>
__global__ __launch_bounds__(NT_TILE) void k_flush(DevCtx c, int sp, int kb, int use_lds) {
  extern __shared__ __align__(16) char smem_basis[];  // TW K x K scratch (use_lds)
  flush_block<T, NOB>(c, blockIdx.x * TW, sp, kb, use_lds ? (T *)smem_basis : nullptr);
}

}  // namespace dmcx
