// SweepLaunch members (the single-determinant sweep in one tile shape);
// included once per (working precision, shape) translation unit.
#pragma once
#include "launch.h"

namespace dmcx {

template <typename T, int SHAPE>
void SweepLaunch<T, SHAPE>::sweep(int nob, const DevCtx &c, uint8_t *acc, long long acc_ss,
                                  int acc_ws, size_t lds, hipStream_t s) {
  if constexpr (SHAPE == SHAPE_SHALLOW) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep_w4<T, N>, lds) == hipSuccess) \
  k_sweep_w4<T, N><<<dim3(c.Wpad / TW), dim3(NT_TILE), lds, s>>>(c, acc, acc_ss, acc_ws)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  } else {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep<T, N>, lds) == hipSuccess) \
  k_sweep<T, N><<<dim3(c.Wpad / TW), dim3(NT_TILE), lds, s>>>(c, acc, acc_ss, acc_ws)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  }
}

template <typename T, int SHAPE>
void SweepLaunch<T, SHAPE>::sweep_multi(int nob, const DevCtx *cs, const int2 *tiles, int ntiles,
                                        const SweepLog *logs, size_t lds, hipStream_t s) {
  if constexpr (SHAPE == SHAPE_SHALLOW) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep_w4_multi<T, N>, lds) == hipSuccess) \
  k_sweep_w4_multi<T, N><<<dim3(ntiles), dim3(NT_TILE), lds, s>>>(cs, tiles, logs)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  } else {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep_multi<T, N>, lds) == hipSuccess) \
  k_sweep_multi<T, N><<<dim3(ntiles), dim3(NT_TILE), lds, s>>>(cs, tiles, logs)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  }
}

template <typename T, int SHAPE>
size_t SweepLaunch<T, SHAPE>::sweep_lds(int nob) {
  hipFuncAttributes a{};
  if constexpr (SHAPE == SHAPE_SHALLOW) {
#define DMCX_CALL(N) (void)hipFuncGetAttributes(&a, (const void *)k_sweep_w4<T, N>)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  } else {
#define DMCX_CALL(N) (void)hipFuncGetAttributes(&a, (const void *)k_sweep<T, N>)
    DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  }
  return a.sharedSizeBytes;
}

}  // namespace dmcx
