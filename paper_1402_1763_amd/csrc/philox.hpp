// Counter-based random numbers on the device.
//
// The paper's sampler is a sequence of independent univariate draws, and it
// recommends giving every parallel worker its own generator (Sec. 3,
// "Comments on parallelization").  Here every draw instead has an address:
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11) maps a
// 128-bit counter (element, sweep, phase, chain) and the 64-bit seed to four
// 32-bit words, so a lane computes exactly the draws of the elements it owns.
//
// Derived draws:
//   U23(x) = (floor(x / 2^9) + 1/2) 2^-23, in (0, 1), exact in FP32 and FP64;
//   Box-Muller on words (xa, xb): r = sqrt(-2 ln U23(xa)),
//   theta = 2 pi U23(xb) -> (r cos theta, r sin theta);
//   Gamma(a, 1): Marsaglia & Tsang (ACM TOMS 26(3), 2000), no squeeze step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

enum : uint32_t {
  kPhaseMessenger = 0,
  kPhaseSignal = 1,
  kPhaseGamma = 2,
  kPhaseMix = 3,
  kPhaseProbe = 4   // signs of the log-determinant estimator's probes
};
constexpr uint32_t kGammaAttempts = 1u << 16;   // counter word 0 = bin * 2^16 + attempt

struct Words4 {
  uint32_t x0, x1, x2, x3;
};

// XOR3: the two three-way XORs of a round as single gfx950 three-input
// bitwise operations (truth table 0x96) instead of pairs of XORs.
template <bool XOR3 = false>
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = XOR3 ? __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96)
                             : static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = XOR3 ? __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96)
                             : static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(p1);
    c3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

template <typename R>
__device__ __forceinline__ R u23(uint32_t x) {
  // (floor(x / 2^9) + 1/2) 2^-23 as one fused multiply-add: both forms are
  // exact (at most 24 significant bits), so they agree bit for bit
  return fma(static_cast<R>(x >> 9), R(1.1920928955078125e-07), R(5.9604644775390625e-08));
}

// Box-Muller pair from two words, in the precision R.  The FP32 form uses the
// hardware transcendentals: v_log_f32 is log2, v_sin_f32 / v_cos_f32 take
// their argument in revolutions (sin(2 pi x)), so theta = 2 pi U23 needs no
// range reduction; all are accurate to a few ulp on (0, 1).
__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, float& g0, float& g1) {
  constexpr float kMinus2Ln2 = -1.38629436111989061883f;   // -2 ln 2
  const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u23<float>(xa)));
  const float turn = u23<float>(xb);
  g0 = r * __builtin_amdgcn_cosf(turn);
  g1 = r * __builtin_amdgcn_sinf(turn);
}

__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, double& g0, double& g1) {
  const double r = sqrt(-2.0 * log(u23<double>(xa)));
  double s, c;
  sincospi(2.0 * u23<double>(xb), &s, &c);
  g0 = r * c;
  g1 = r * s;
}

// One Gamma(shape, 1) variate in FP64.  Attempt j reads the words of counter
// (bin * 2^16 + j, sweep, kPhaseGamma, chain): z = cosine normal of (x0, x1),
// u = U23(x2); candidate v = (1 + c z)^3 with d = a - 1/3, c = 1/sqrt(9 d) is
// accepted when v > 0 and ln u < z^2/2 + d - d v + d ln v.  shape < 1 draws
// Gamma(shape + 1) U^(1/shape) with U = U23(x3) of attempt 0.  Returns a
// negative value if no attempt was accepted.
__device__ inline double gamma_mt(double shape, uint32_t bin, uint32_t sweep, uint32_t chain,
                                  uint32_t k0, uint32_t k1) {
  const bool boost = shape < 1.0;
  const double a = boost ? shape + 1.0 : shape;
  const double d = a - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  double u_boost = 1.0;
  for (uint32_t j = 0; j < kGammaAttempts; ++j) {
    const Words4 w = philox4x32_10(bin * kGammaAttempts + j, sweep, kPhaseGamma, chain, k0, k1);
    if (j == 0) u_boost = u23<double>(w.x3);
    double z, unused;
    box_muller(w.x0, w.x1, z, unused);
    const double u = u23<double>(w.x2);
    const double t = 1.0 + c * z;
    const double v = t * t * t;
    if (v > 0.0 && log(u) < 0.5 * z * z + d - d * v + d * log(v)) {
      const double g = d * v;
      return boost ? g * pow(u_boost, 1.0 / shape) : g;
    }
  }
  return -1.0;
}

}  // namespace mf
