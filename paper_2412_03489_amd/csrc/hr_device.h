// hr_device.h -- device-side building blocks of the estimator (gfx950).
//
//   * Philox4x32-10 counter-based generator (Salmon et al., SC'11);
//   * open-interval uniforms, Box-Muller Gaussians (Box & Muller 1958);
//   * the one-dimensional lobe samplers of the smoothed differential kernels
//     (sections "Gradients" and "Hessians" of Wang, Fischer, Ritschel 2025),
//     the diagonal one inverted with Lambert W (Corless et al. 1996, Halley);
//   * error-free transformation TwoSum (Knuth) for compensated FP32 sums
//     (Ogita, Rump, Oishi 2005, algorithm Sum2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hr {

// ---- random-number layout ---------------------------------------------------
// key = (lo32(seed), hi32(seed)); dimension block (s, j, 0, tag); aggregate
// element selector (s, 0xFFFFFFFF, 0, tag); path-tracer pixel randomness
// (s, pixel, 16*spp + bounce, 0x80000000).  Tag: element index for
// per-element IS streams, 0x7FFFFFFF aggregate, 0x7FFFFFFE plain Gaussian.
constexpr uint32_t kTagAIS = 0x7FFFFFFFu;
constexpr uint32_t kTagGauss = 0x7FFFFFFEu;
constexpr uint32_t kTagPixel = 0x80000000u;
constexpr uint32_t kDimSelect = 0xFFFFFFFFu;

struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    // each 32 x 32 -> 64-bit product as one multiply (v_mad_u64_u32) rather
    // than separate high and low halves
    const uint64_t pa = (uint64_t)0xD2511F53u * c0, pb = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
    const uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
    uint32_t n0 = hi_b ^ c1 ^ k0;
    uint32_t n2 = hi_a ^ c3 ^ k1;
    c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ u32x4 philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1,
                                               uint32_t c2, uint32_t c3) {
  return philox10(c0, c1, c2, c3, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
}

// (w + 1/2) 2^-32: exact in FP64
__device__ __forceinline__ double u01_d(uint32_t w) { return fma((double)w, 0x1p-32, 0x1p-33); }
// the same uniform rounded to FP32 (path-tracer use)
__device__ __forceinline__ float u01_f(uint32_t w) { return (float)u01_d(w); }

// ---- one-dimensional samplers ----------------------------------------------
// Positivised derivative-of-Gaussian lobes: |u|/s^2 N(u)/Z_G, sign from xi <= 1/2,
// Rayleigh magnitude sigma sqrt(-2 ln(2 min(xi, 1 - xi))).
__device__ __forceinline__ double grad_lobe(uint32_t w, double sg) {
  if (w < 0x80000000u) {
    double t = fma((double)w, 0x1p-31, 0x1p-32);                 // 2 xi
    return -sg * sqrt(-2.0 * log(t));
  }
  double t = fma((double)(0xFFFFFFFFu - w), 0x1p-31, 0x1p-32);    // 2 (1 - xi)
  return sg * sqrt(-2.0 * log(t));
}

// W_0 / W_{-1} on [-1/e, 0): branch-point series start (p = sqrt(2(ez+1)) ),
// log asymptotics for W_{-1} near 0, then Halley steps.
__device__ inline double lambert_w(double z, bool lower) {
  const double e_hi = 2.71828182845904509080, e_lo = 1.4456468917292502e-16;
  double t = fma(e_hi, z, 1.0) + e_lo * z;   // e z + 1, kept accurate near the branch point
  if (t <= 0.0) return -1.0;
  double p = sqrt(2.0 * t);
  double w;
  if (t < 0.25) {
    double p2 = p * p, p3 = p2 * p;
    w = lower ? (-1.0 - p - p2 / 3.0 - (11.0 / 72.0) * p3) : (-1.0 + p - p2 / 3.0 + (11.0 / 72.0) * p3);
  } else if (lower) {
    double l1 = log(-z), l2 = log(-l1);
    w = l1 - l2 + l2 / l1;
  } else {
    w = z;
  }
  // Halley's step is cubically convergent: once it falls to a few ulp of w,
  // w is exact to the last ulp (a tighter test can stall on rounding noise
  // and run every iteration)
  for (int it = 0; it < 32; ++it) {
    double ew = exp(w);
    double f = w * ew - z;
    double w1 = w + 1.0;
    if (w1 == 0.0) break;
    double den = ew * w1 - (w + 2.0) * f / (2.0 * w1);
    if (den == 0.0) break;
    double dw = f / den;
    w -= dw;
    if (fabs(dw) <= 0x1p-50 * (1.0 + fabs(w))) break;
  }
  return w;
}

// Positivised second derivative of the 1-D Gaussian (three branches split at
// -sigma and +sigma, CDF 1/4 and 3/4 there); s = u^2/sigma^2 solves
// s e^{-s} = 16 y^2/e, hence s = -W(-16 y^2/e) with W_{-1} on the tails.
__device__ inline double hdiag_lobe(uint32_t w, double sg) {
  const double inv_e = 0.36787944117144233;
  if (w < 0x40000000u) {
    double xi = u01_d(w);
    double s = -lambert_w(-16.0 * xi * xi * inv_e, true);
    return -sg * sqrt(s);
  }
  if (w >= 0xC0000000u) {
    double om = fma((double)(0xFFFFFFFFu - w), 0x1p-32, 0x1p-33);
    double s = -lambert_w(-16.0 * om * om * inv_e, true);
    return sg * sqrt(s);
  }
  double d = u01_d(w) - 0.5;
  double s = -lambert_w(-16.0 * d * d * inv_e, false);
  s = s < 0.0 ? 0.0 : s;
  return d < 0.0 ? -sg * sqrt(s) : sg * sqrt(s);
}

// upper-triangle element m -> (i, j), i <= j, enumerated row by row
__device__ __forceinline__ void tri_ij(int n, int m, int& i, int& j) {
  int row = 0, start = 0;
  while (start + (n - row) <= m) { start += n - row; ++row; }
  i = row;
  j = row + (m - start);
}

// ---- compensated FP32 accumulation ------------------------------------------
struct fsum2 { float hi, lo; };
__device__ __forceinline__ void two_sum_add(fsum2& a, float x) {
  float s = a.hi + x;
  float bp = s - a.hi;
  float err = (a.hi - (s - bp)) + (x - bp);
  a.hi = s;
  a.lo += err;
}

}  // namespace hr
