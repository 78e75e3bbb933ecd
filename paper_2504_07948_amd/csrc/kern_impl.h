// Definitions of the NobLaunch members (see launch.h); included once per
// working precision.
#pragma once
#include "forces.h"
#include "launch.h"
#include "zv.h"

namespace dmcx {

template <typename T>
void NobLaunch<T>::orbitals_all(int nob, const DevCtx &c, size_t lds, hipStream_t s) {
  const int npts = c.Wpad * c.ne;
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_orbitals_all<T, N>, lds) == hipSuccess) \
  k_orbitals_all<T, N><<<dim3((npts + TW - 1) / TW), dim3(NT_TILE), lds, s>>>(c)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::orbitals_at(int nob, const DevCtx &c, const double *pos, int npts, T *dst,
                               size_t lds, hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_orbitals_at<T, N>, lds) == hipSuccess) \
  k_orbitals_at<T, N><<<dim3((npts + TW - 1) / TW), dim3(NT_TILE), lds, s>>>(c, pos, npts, dst)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::ion_grad_det(int nob, const DevCtx &c, double *partial, int ntile, size_t lds,
                                hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_ion_grad_det<T, N>, lds) == hipSuccess) \
  k_ion_grad_det<T, N><<<dim3(c.Wpad * ntile), dim3(NT_FORCE), lds, s>>>(c, partial)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::zv_det(int nob, const DevCtx &c, const T *xt, const double *cg, double *zpart,
                          double *zs, int ntile, size_t lds, hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_zv_det<T, N>, lds) == hipSuccess) \
  k_zv_det<T, N><<<dim3(c.Wpad * ntile), dim3(NT_FORCE), lds, s>>>(c, xt, cg, zpart, zs)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::block_init(int nob, const DevCtx &c, int sp, int b0, int kb, hipStream_t s) {
#define DMCX_CALL(N) k_block_init<T, N><<<dim3(c.Wpad), dim3(256), 0, s>>>(c, sp, b0, kb)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::ratio_grad(int nob, const DevCtx &c, int iel, int m, const double *r_new,
                              double *ratio, double *grad, T *prop, double *prop_rho, size_t lds,
                              hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_ratio_grad<T, N>, lds) == hipSuccess) \
  k_ratio_grad<T, N><<<dim3(c.Wpad / TW), dim3(NT_TILE), lds, s>>>(c, iel, m, r_new, ratio, grad, \
                                                                   prop, prop_rho)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::accept(int nob, const DevCtx &c, int iel, int sp, int m, int kb,
                          const uint8_t *acc8, const T *prop, const double *prop_rho,
                          const double *r_new, hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  k_accept<T, N><<<dim3(c.Wpad), dim3(64), 0, s>>>(c, iel, sp, m, kb, acc8, prop, prop_rho, r_new)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::flush(int nob, const DevCtx &c, int sp, int kb, hipStream_t s) {
  // the coefficient and M scratch in LDS when the tile's K x K blocks fit in
  // the default 64 KB of dynamic LDS, else in the global Ms
  const size_t lds = (size_t)TW * c.K * c.K * sizeof(T);
  const int use_lds = lds <= 65536 ? 1 : 0;
#define DMCX_CALL(N) \
  k_flush<T, N><<<dim3(c.Wpad / TW), dim3(NT_TILE), use_lds ? lds : 0, s>>>(c, sp, kb, use_lds)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void NobLaunch<T>::values64(int nob, const DevCtx &c, double *A64, size_t lds, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    const int npts = c.Wpad * c.ne;
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_values64<T, N>, lds) == hipSuccess) \
  k_values64<T, N><<<dim3((npts + NPV - 1) / NPV), dim3(NT_TILE), lds, s>>>(c, A64)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  }
}

template <typename T>
void NobLaunch<T>::escalate_gl(int nob, const DevCtx &c, const double *G64, const EscList &esc,
                               size_t lds, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    const int ntile = (c.ne + TW - 1) / TW;
    // slot groups, each looping over its slots: few, because every block,
    // even one that finds no slot, holds a CU's worth of LDS while it is
    // dispatched (the list is usually a handful of walkers)
    const int ngrp = c.Wpad < 32 ? c.Wpad : 32;
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_escalate_gl<N>, lds) == hipSuccess) \
  k_escalate_gl<N><<<dim3(ngrp * ntile), dim3(NT_TILE), lds, s>>>(c, G64, esc)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  }
}

}  // namespace dmcx
