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

// Upper 16x16 block (a, b), a <= b, of an nb x nb block grid, numbered row by row.
__host__ __device__ constexpr int upper_blk(int a, int b, int nb) { return a * nb - a * (a - 1) / 2 + (b - a); }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ double shfl_xor_d(double v, int mask) { return __shfl_xor(v, mask, kWave); }

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, kWave); }

// The same for the FP32 sketch kernels (overloads, so templates over the element type use one name).
__device__ __forceinline__ float shfl_xor_d(float v, int mask) { return __shfl_xor(v, mask, kWave); }

__device__ __forceinline__ float shfl_d(float v, int src) { return __shfl(v, src, kWave); }

// Read a lane's value (lane index uniform across the wave, may be a runtime value).
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float readlane_d(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// One DPP lane move of a 64-bit value (lanes outside ROW_MASK, or with no source, get 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave, returned to every lane (uniform): DPP partial sums within
// quads, half rows, rows, then row broadcasts 15 and 31 gather the total in lane 63.  The
// summation order is fixed, so the result is deterministic.
template <class T>
__device__ __forceinline__ T wave_reduce_sum(T v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror
  v += dpp_move<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return readlane_d(v, kWave - 1);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

}  // namespace rcqr
