// Host-side launchers of the kernels that are templated on the number of
// 16-orbital blocks (NOB).  Each working precision (and each sweep shape) is
// instantiated in a translation unit of its own (kern_f64.hip, kern_f32.hip,
// sweep_*.hip), so the builds of the many NOB variants run in parallel; the runtime (dmcx.hip) calls these
// with the context's NOB and never instantiates the kernels itself.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dmcx {

constexpr int NOB_MAX = 10;  // up to 160 orbital columns per tile

// Let a kernel use `dyn` bytes of dynamic LDS (beyond the 64 KB default).
// The launchers below launch only when this succeeds; a failure stays the
// thread's last HIP error, which the runtime's hipGetLastError() after every
// launcher call reports as DMCX_E_HIP.
template <typename K>
inline hipError_t allow_lds(K kernel, size_t dyn) {
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)dyn);
}

#define DMCX_NOB_SWITCH(nob, CALL) \
  switch (nob) {                   \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    case 8: CALL(8); break;        \
    case 9: CALL(9); break;        \
    default: CALL(10); break;      \
  }

// Tile shapes of the single-determinant sweep.  Both put 8 walkers in a
// workgroup of 8 waves; they differ in the depth of the staged basis tile
// (the K extent of the orbital GEMM per LDS stage) and with it in how many
// workgroups share a CU:
//   SHAPE_DEEP     4 stage_ksteps(NOB) functions per stage, up to 2 waves per
//                  SIMD (one workgroup per CU at the FP64 register count);
//   SHAPE_SHALLOW  half as deep, 4 waves per SIMD (two workgroups per CU).
enum SweepShape { SHAPE_DEEP = 0, SHAPE_SHALLOW = 1 };

// The sweep launchers of one working precision and shape, instantiated in
// translation units of their own (sweep_*.hip).
template <typename T, int SHAPE>
struct SweepLaunch {
  // one full sweep of the single-determinant trial function
  static void sweep(int nob, const DevCtx &c, uint8_t *acc, long long acc_ss, int acc_ws,
                    size_t lds, hipStream_t s);
  // static LDS bytes of that sweep kernel
  static size_t sweep_lds(int nob);
  // one sweep over the tiles of several systems of this width (a group)
  static void sweep_multi(int nob, const DevCtx *cs, const int2 *tiles, int ntiles,
                          const SweepLog *logs, size_t lds, hipStream_t s);
};

template <typename T>
struct NobLaunch {
  // orbital VGL rows of every electron of every walker -> vglc
  static void orbitals_all(int nob, const DevCtx &c, size_t lds, hipStream_t s);
  // orbitals at one point per walker -> dst [Wpad][5][NP]
  static void orbitals_at(int nob, const DevCtx &c, const double *pos, int npts, T *dst,
                          size_t lds, hipStream_t s);
  // per-tile determinant part of the ion derivatives
  static void ion_grad_det(int nob, const DevCtx &c, double *partial, int ntile, size_t lds,
                           hipStream_t s);
  // determinant adjoint of the Eq. 4 local-energy derivative (zero-variance forces)
  static void zv_det(int nob, const DevCtx &c, const T *xt, const double *cg, double *zpart,
                     double *zs, int ntile, size_t lds, hipStream_t s);
  // move-by-move interface
  static void block_init(int nob, const DevCtx &c, int sp, int b0, int kb, hipStream_t s);
  static void ratio_grad(int nob, const DevCtx &c, int iel, int m, const double *r_new,
                         double *ratio, double *grad, T *prop, double *prop_rho, size_t lds,
                         hipStream_t s);
  static void accept(int nob, const DevCtx &c, int iel, int sp, int m, int kb,
                     const uint8_t *acc8, const T *prop, const double *prop_rho,
                     const double *r_new, hipStream_t s);
  static void flush(int nob, const DevCtx &c, int sp, int kb, hipStream_t s);
  // FP64 orbital values of every electron -> A64 [Wpad][ne][NP], and the
  // working-precision value rows of vglc from them (mixed form only)
  static void values64(int nob, const DevCtx &c, double *A64, size_t lds, hipStream_t s);
  // FP64 (g_i, l_i) of the walkers on the re-evaluation list (mixed form only)
  static void escalate_gl(int nob, const DevCtx &c, const double *G64, const EscList &esc,
                          size_t lds, hipStream_t s);
};

// FP64 inverse with one wave per matrix (inverse.hip): value rows of
// precision S at rows + (w ne + e) rs; writes GT (precision T), log|det|,
// sign and, if G64 is not null, an FP64 copy of the inverses.  Returns false
// (nothing launched) when NP > 64: the rows do not fit one wave.
template <typename T, typename S>
bool inverse_w(const DevCtx &c, const S *rows, int rs, double *G64, int periodic, hipStream_t s);
// one padded width NR of it (instantiated in inv_*.hip)
template <typename T, typename S, int NR>
void launch_inverse_nr(const DevCtx &c, const S *rows, int rs, double *G64, int periodic,
                       hipStream_t s);

}  // namespace dmcx
