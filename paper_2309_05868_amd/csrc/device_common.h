// Device-side helpers shared by the rcqr kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcqr {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): round multipliers and Weyl key increments.
// ---------------------------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kTagCountSketch = 1;
constexpr uint64_t kTagGaussian = 2;

struct Block4 {
  uint64_t y0, y1, y2, y3;
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0;
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t block_word(const Block4& b, int i) {
  return i == 0 ? b.y0 : i == 1 ? b.y1 : i == 2 ? b.y2 : b.y3;
}

// CountSketch code of one row: (bucket << 1) | signbit, bucket = floor(w s1 / 2^64), signbit = w & 1.
__device__ __forceinline__ uint32_t countsketch_code(uint64_t w, uint64_t s1) {
  const uint64_t bucket = __umul64hi(w, s1);
  return (uint32_t)((bucket << 1) | (w & 1ull));
}

// Box-Muller on two Philox words: u1 in (0, 1], u2 in [0, 1).
__device__ __forceinline__ void box_muller(uint64_t ya, uint64_t yb, double& z0, double& z1) {
  const double u1 = (double)((ya >> 11) + 1ull) * 0x1.0p-53;
  const double u2 = (double)(yb >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586 * u2;  // the double nearest to 2*pi
  double s, c;
  sincos(t, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// Order LDS traffic between the lanes of one wave (no cross-wave barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ double shfl_xor_d(double v, int mask) { return __shfl_xor(v, mask, kWave); }

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, kWave); }

// The same for the FP32 sketch kernels (overloads, so templates over the element type use one name).
__device__ __forceinline__ float shfl_xor_d(float v, int mask) { return __shfl_xor(v, mask, kWave); }

__device__ __forceinline__ float shfl_d(float v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

}  // namespace rcqr
