// MsdLaunch members (the multideterminant sweep); included once per working
// precision.
#pragma once
#include "kern_impl.h"
#include "msd.h"

namespace dmcx {

template <typename T>
void MsdLaunch<T>::sweep(int nob, const DevCtx &c, uint8_t *acc, long long acc_ss, int acc_ws,
                         size_t lds, hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep_msd<T, N>, lds) == hipSuccess) \
  k_sweep_msd<T, N><<<dim3(c.Wpad / TW), dim3(NT_TILE), lds, s>>>(c, acc, acc_ss, acc_ws)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
void MsdLaunch<T>::sweep_multi(int nob, const DevCtx *cs, const int2 *tiles, int ntiles,
                               const SweepLog *logs, size_t lds, hipStream_t s) {
#define DMCX_CALL(N)                                                                   \
  if (allow_lds(k_sweep_msd_multi<T, N>, lds) == hipSuccess) \
  k_sweep_msd_multi<T, N><<<dim3(ntiles), dim3(NT_TILE), lds, s>>>(cs, tiles, logs)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
}

template <typename T>
size_t MsdLaunch<T>::sweep_lds(int nob) {
  hipFuncAttributes a{};
#define DMCX_CALL(N) (void)hipFuncGetAttributes(&a, (const void *)k_sweep_msd<T, N>)
  DMCX_NOB_SWITCH(nob, DMCX_CALL)
#undef DMCX_CALL
  return a.sharedSizeBytes;
}

}  // namespace dmcx
