// FP64 wave-per-matrix inverse: dispatch on the padded orbital width.  The
// unrolled kernels are instantiated in inv_*.hip, several translation units
// that build in parallel.
#include "launch.h"

namespace dmcx {

template <typename T, typename S>
bool inverse_w(const DevCtx &c, const S *rows, int rs, double *G64, int periodic, hipStream_t s) {
  switch (c.NP) {
    case 16: launch_inverse_nr<T, S, 16>(c, rows, rs, G64, periodic, s); return true;
    case 32: launch_inverse_nr<T, S, 32>(c, rows, rs, G64, periodic, s); return true;
    case 48: launch_inverse_nr<T, S, 48>(c, rows, rs, G64, periodic, s); return true;
    case 64: launch_inverse_nr<T, S, 64>(c, rows, rs, G64, periodic, s); return true;
    default: return false;
  }
}

template bool inverse_w<double, double>(const DevCtx &, const double *, int, double *, int, hipStream_t);
template bool inverse_w<float, float>(const DevCtx &, const float *, int, double *, int, hipStream_t);
template bool inverse_w<float, double>(const DevCtx &, const double *, int, double *, int, hipStream_t);

}  // namespace dmcx
