// Counter-based Gaussian noise for the Brown thermal field (device code).
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds on a
// 4 x 32-bit counter with a 2 x 32-bit key; each round forms the two 64-bit
// products of counter words 0 and 2 with the published multipliers, mixes
// their high halves with the other counter words and the round key, and the
// key is advanced by the published Weyl constants between rounds.
// Key = replica seed (low, high); counter = (cell, step low, step high, g),
// g = trial generation (0 except for refilled retire/refill trials).
// Uniforms (x + 1/2) 2^-32, Box-Muller on (u0, u1) and (u2, u3); the first
// three normals are the x, y, z components.
#pragma once
#include "common.h"

namespace mmx {

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 each instead of a mul_hi /
    // mul_lo pair
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += W0;
    k1 += W1;
  }
}

template <typename T>
struct BoxMuller;

template <>
struct BoxMuller<double> {
  static __device__ inline void eta(const uint32_t w[4], double out[3]) {
    const double s = 2.3283064365386962890625e-10;  // 2^-32
    const double u0 = ((double)w[0] + 0.5) * s, u1 = ((double)w[1] + 0.5) * s;
    const double u2 = ((double)w[2] + 0.5) * s, u3 = ((double)w[3] + 0.5) * s;
    const double r01 = sqrt(-2.0 * log(u0));
    const double r23 = sqrt(-2.0 * log(u2));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    out[0] = r01 * cs;
    out[1] = r01 * sn;
    out[2] = r23 * cospi(2.0 * u3);
  }
};

// FP32: the hardware transcendental units do Box-Muller directly: v_log_f32
// is log2 and v_sin_f32 / v_cos_f32 take their argument in turns, so
// sin(2 pi u) is one instruction (u in (0, 1); results within a few ulp).
template <>
struct BoxMuller<float> {
  static __device__ inline void eta(const uint32_t w[4], float out[3]) {
    const float s = 2.3283064365386962890625e-10f;
    const float u0 = fmaf((float)w[0], s, 0.5f * s), u1 = fmaf((float)w[1], s, 0.5f * s);
    const float u2 = fmaf((float)w[2], s, 0.5f * s), u3 = fmaf((float)w[3], s, 0.5f * s);
    const float m2ln2 = -1.38629436111989061883f;  // -2 ln 2
    const float r01 = sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float r23 = sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    out[0] = r01 * __builtin_amdgcn_cosf(u1);
    out[1] = r01 * __builtin_amdgcn_sinf(u1);
    out[2] = r23 * __builtin_amdgcn_cosf(u3);
  }
};

template <typename T>
__device__ inline void thermal_eta(uint64_t seed, uint32_t cell, uint64_t step, T out[3],
                                   uint32_t gen = 0u) {
  uint32_t c[4] = {cell, (uint32_t)(step & 0xFFFFFFFFull), (uint32_t)(step >> 32), gen};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  BoxMuller<T>::eta(c, out);
}

}  // namespace mmx
