// Device helpers shared by the dmcx kernels (gfx950 / CDNA4).
//
// - MFMA wrappers for the 16x16x4 FP64 and FP32 matrix-core instructions.
//   Operand layout per 64-lane wave (checked by dmcx_selftest):
//     A (16x4): lane l holds A[l % 16][l / 16]
//     B (4x16): lane l holds B[l / 16][l % 16]
//     D (16x16): lane l, element r holds D[Acc4<T>::row(l / 16, r)][l % 16]
//   with row = l/16 + 4 r for FP64 and row = 4 (l/16) + r for FP32.
// - Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
//   per-move draws: counter = (electron, walker, step, draw), key = seed.
// - Wave reductions: 64 lanes (one walker per wave in the tile kernels) and
//   32-lane halves (two points per wave in the force kernel).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmcx {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16x16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc4;
template <> struct Acc4<double> {
  typedef v4d type;
  __device__ __host__ static constexpr int row(int q, int r) { return q + 4 * r; }
};
template <> struct Acc4<float> {
  typedef v4f type;
  __device__ __host__ static constexpr int row(int q, int r) { return 4 * q + r; }
};

// ------------------------------------------------------------- Philox ----
struct Philox4 {
  uint32_t x[4];
};

__device__ __host__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
  // Ten rounds; each round multiplies words 0 and 2 by the Philox constants,
  // mixes the high halves with words 1 and 3 and the round key, and bumps the
  // key by the golden-ratio Weyl increments.
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t y0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
    const uint32_t y1 = (uint32_t)m1;
    const uint32_t y2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
    const uint32_t y3 = (uint32_t)m0;
    c0 = y0;
    c1 = y1;
    c2 = y2;
    c3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 o;
  o.x[0] = c0;
  o.x[1] = c1;
  o.x[2] = c2;
  o.x[3] = c3;
  return o;
}

// Two 53-bit uniforms in [0, 1) from one Philox block.
__device__ inline void uniform_pair(uint64_t seed, uint32_t step, uint32_t walker, uint32_t elec,
                                    uint32_t draw, double &u0, double &u1) {
  const Philox4 p = philox4x32_10(elec, walker, step, draw, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)p.x[0] << 32) | p.x[1];
  const uint64_t b = ((uint64_t)p.x[2] << 32) | p.x[3];
  u0 = (double)(a >> 11) * 0x1.0p-53;
  u1 = (double)(b >> 11) * 0x1.0p-53;
}

// Gaussian displacement chi (3 normals, Box-Muller on 1-u) and the
// acceptance uniform of one proposed move, computed by lanes 0, 1, 2 of the
// 64-lane wave that serves the walker (lane d evaluates draw d: draw 0 gives
// chi_x, chi_y; draw 1 chi_z; draw 2 the uniform) and broadcast to the wave.
__device__ inline void move_draws_lanes64(uint64_t seed, uint32_t step, uint32_t walker,
                                          uint32_t elec, int t, double chi[3], double &uacc) {
  const double two_pi = 6.283185307179586476925286766559;
  double u0, u1;
  uniform_pair(seed, step, walker, elec, t < 2 ? (uint32_t)t : 2u, u0, u1);
  const double rad = sqrt(-2.0 * log(1.0 - u0));
  const double cs = rad * cos(two_pi * u1);
  const double sn = rad * sin(two_pi * u1);
  chi[0] = __shfl(cs, 0, 64);
  chi[1] = __shfl(sn, 0, 64);
  chi[2] = __shfl(cs, 1, 64);
  uacc = __shfl(u0, 2, 64);
}

// Index of the calling wave within its workgroup, as a scalar (wave-uniform
// tests on it compile to scalar branches, addresses built from it to scalar
// arithmetic).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------- reductions ----
// Sum over one aligned 32-lane half of a wave.
__device__ __forceinline__ double sum32(double v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
  return v;
}
// A 64-bit value moved between lanes with one DPP control (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// Sum over the 64 lanes of a wave; every lane must be active.  Within each
// 16-lane row: quad permutations (lane ^ 1, lane ^ 2), then row rotations by
// 4 and 8, after which every lane holds its row's sum; the four row sums are
// read out and added (a wave-uniform result).
__device__ __forceinline__ double sum64(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x124>(v);  // row_ror 4
  v += dpp_f64<0x128>(v);  // row_ror 8
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Pade factor u(r) = a r / (1 + b r) and its first two radial derivatives.
struct Pade {
  double u, d1, d2;
};
__device__ __forceinline__ Pade pade(double a, double b, double r) {
  const double q = 1.0 / (1.0 + b * r);
  Pade p;
  p.u = a * r * q;
  p.d1 = a * q * q;
  p.d2 = -2.0 * a * b * q * q * q;
  return p;
}

}  // namespace dmcx
