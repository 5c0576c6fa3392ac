// Streaming passes for 65..128 columns (rows padded to 128).
//
// A 128-double row does not fit a lane's registers next to the solve's working set, so the
// row solve x R = v runs as a 2 x 2 block forward substitution (Section 5.2's row-wise
// substitution, reordered by blocks):
//     x_lo = v_lo R00^{-1}                       (registers, then written to the output row)
//     x_hi = (v_hi - x_lo R01) R11^{-1}          (x_lo read back from the output row, an L2 hit,
//                                                 one entry at a time)
// Every entry of x is still produced by the same sequence of FMAs as a plain row substitution
// in increasing column order.  Q0 = V R0^{-1} is written into the Q buffer (the caller's
// output), the Gram matrix G = Q0^T Q0 is accumulated by a separate FP64-MFMA pass over Q0, and
// the final pass turns Q0 into Q = Q0 R1^{-1} in place.
//
// Factor format for 128 columns ("blocked packed"): [R00 packed | R01 dense row-major | R11 packed],
// each packed block the upper triangle row by row with 1/R_kk on the diagonal: 2080 + 4096 + 2080
// doubles.
#include "device_common.h"
#include "launch.h"

namespace rcqr {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kH = 64;            // half width
constexpr int kPk = kH * (kH + 1) / 2;

__device__ __forceinline__ int opaque_zero128(double after) {
  int z = 0;
  asm volatile("" : "+s"(z) : "v"(after));
  return z;
}

// x R = v for 64 columns, R packed (reciprocal diagonal); coefficients streamed through SGPRs.
__device__ __forceinline__ void solve64(double (&x)[kH], const double* __restrict__ Rpk) {
  constexpr int NV = kPk, NCH = (NV + 7) / 8, PD = 2;
  double buf[PD + 1][8];
#pragma unroll
  for (int ch = 0; ch < PD; ++ch) {
#pragma unroll
    for (int e = 0; e < 8; ++e) buf[ch][e] = Rpk[8 * ch + e];
  }
  int v = 0;
  double last = x[0];
#pragma unroll
  for (int k = 0; k < kH; ++k) {
#pragma unroll
    for (int j = k; j < kH; ++j) {
      if ((v & 7) == 0) {
        __builtin_amdgcn_sched_barrier(0);
        const int nxt = (v >> 3) + PD;
        if (nxt < NCH) {
          const double* src = Rpk + opaque_zero128(last);
#pragma unroll
          for (int e = 0; e < 8; ++e) buf[nxt % (PD + 1)][e] = (8 * nxt + e < NV) ? src[8 * nxt + e] : 0.0;
        }
      }
      const double c = buf[(v >> 3) % (PD + 1)][v & 7];
      if (j == k) {
        x[k] = x[k] * c;
        last = x[k];
      } else {
        x[j] = __builtin_fma(-x[k], c, x[j]);
        last = x[j];
      }
      ++v;
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// v_hi -= x_lo R01 (R01 dense 64 x 64 row-major).  x_lo[k] is read back from xlo (the row
// just written) through an offset the compiler cannot see is zero, so it is a real load and
// x_lo does not stay live in registers; loads run two entries ahead of use.
__device__ __forceinline__ void update64(double (&x)[kH], const double* xlo, const double* __restrict__ R01) {
  constexpr int NV = kH * kH, NCH = NV / 8, PD = 2;
  double buf[PD + 1][8];
#pragma unroll
  for (int ch = 0; ch < PD; ++ch) {
#pragma unroll
    for (int e = 0; e < 8; ++e) buf[ch][e] = R01[8 * ch + e];
  }
  double last = x[0];
  const double* xl = xlo + opaque_zero128(last);
  double xq[3];
  xq[0] = xl[0];
  xq[1] = xl[1];
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    if (k + 2 < kH) xq[(k + 2) % 3] = xl[k + 2];
    const double xk = xq[k % 3];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      const int v = k * kH + j;
      if ((v & 7) == 0) {
        __builtin_amdgcn_sched_barrier(0);
        const int nxt = (v >> 3) + PD;
        if (nxt < NCH) {
          const double* src = R01 + opaque_zero128(last);
#pragma unroll
          for (int e = 0; e < 8; ++e) buf[nxt % (PD + 1)][e] = src[8 * nxt + e];
        }
      }
      x[j] = __builtin_fma(-xk, buf[(v >> 3) % (PD + 1)][v & 7], x[j]);
      last = x[j];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <bool FULL>
__device__ __forceinline__ void load_half(double (&x)[kH], const double* __restrict__ row_ptr, int c0, int n) {
  if constexpr (FULL) {
    const double2* s2 = reinterpret_cast<const double2*>(row_ptr + c0);
#pragma unroll
    for (int c = 0; c < kH / 2; ++c) {
      const double2 v = s2[c];
      x[2 * c] = v.x;
      x[2 * c + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kH; ++c) x[c] = (c0 + c < n) ? row_ptr[c0 + c] : 0.0;
  }
}

template <bool FULL>
__device__ __forceinline__ void store_half(const double (&x)[kH], double* __restrict__ row_ptr, int c0, int n) {
  if constexpr (FULL) {
    double2* d2 = reinterpret_cast<double2*>(row_ptr + c0);
#pragma unroll
    for (int c = 0; c < kH / 2; ++c) d2[c] = double2{x[2 * c], x[2 * c + 1]};
  } else {
#pragma unroll
    for (int c = 0; c < kH; ++c)
      if (c0 + c < n) row_ptr[c0 + c] = x[c];
  }
}

}  // namespace

// One lane per row: out row = in row R^{-1} with the blocked packed factor.  `out` may alias
// `in` (same leading dimension): the lane reads each half of its row before writing it.
template <bool FULL>
__global__ __launch_bounds__(256) void solve128_kernel(const double* in, int64_t m, int n, int64_t ldin, const double* __restrict__ Rbk,
                                                       const int32_t* __restrict__ info, double* out, int64_t ldout) {
  if (info[0] != 0) return;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= m) return;
  const double* src = in + row * ldin;
  double* dst = out + row * ldout;
  double x[kH];
  load_half<FULL>(x, src, 0, n);
  solve64(x, Rbk);
  store_half<FULL>(x, dst, 0, n);
  load_half<FULL>(x, src, kH, n);
  update64(x, dst, Rbk + kPk);
  solve64(x, Rbk + kPk + kH * kH);
  store_half<FULL>(x, dst, kH, n);
}

// G partial = Q0^T Q0 over this workgroup's rows: the 36 upper 16x16 blocks of the 128 x 128
// matrix on FP64 MFMA.  Waves 2p and 2p+1 read the same 4-row K-steps and accumulate blocks
// 0..17 and 18..35 respectively (144 accumulator registers each); fixed grid, fixed order.
template <bool FULL>
__global__ __launch_bounds__(256) void syrk128_kernel(const double* __restrict__ Q0, int64_t m, int n, int64_t ldq,
                                                      const int32_t* __restrict__ info, double* __restrict__ gpart) {
  constexpr int NB = 8, NBU = NB * (NB + 1) / 2, HALF = NBU / 2;  // 36 blocks, 18 per wave
  __shared__ double gl[NBU * 256];
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int set = wave & 1, pair = wave >> 1;
  d4 acc[HALF];
#pragma unroll
  for (int i = 0; i < HALF; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = (m + 3) / 4;  // 4-row MFMA K-steps
  const int rsub = lane >> 4, csub = lane & 15;
  for (int64_t st = (int64_t)blockIdx.x * 2 + pair; st < nsteps; st += (int64_t)gridDim.x * 2) {
    const int64_t row = 4 * st + rsub;
    double F[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int c = 16 * a + csub;
      F[a] = (row < m && (FULL || c < n)) ? Q0[row * ldq + c] : 0.0;
    }
    if (set == 0) {
      int ab = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = a; b < NB; ++b) {
          if (ab < HALF) acc[ab] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[a], F[b], acc[ab], 0, 0, 0);
          ++ab;
        }
      }
    } else {
      int ab = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = a; b < NB; ++b) {
          if (ab >= HALF) acc[ab - HALF] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[a], F[b], acc[ab - HALF], 0, 0, 0);
          ++ab;
        }
      }
    }
  }
  for (int p = 0; p < 2; ++p) {
    if (pair == p) {
#pragma unroll
      for (int i = 0; i < HALF; ++i) {
        const int ab = set * HALF + i;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = ab * 256 + ((lane >> 4) + 4 * e) * 16 + (lane & 15);
          gl[idx] = (p == 0) ? acc[i][e] : gl[idx] + acc[i][e];
        }
      }
    }
    __syncthreads();
  }
  double* outp = gpart + (int64_t)blockIdx.x * (NBU * 256);
  for (int i = threadIdx.x; i < NBU * 256; i += 256) outp[i] = gl[i];
}

static bool full128(int n, const void* a, int64_t lda, const void* b, int64_t ldb) {
  return n == 128 && reinterpret_cast<uintptr_t>(a) % 16 == 0 && lda % 2 == 0 && reinterpret_cast<uintptr_t>(b) % 16 == 0 &&
         ldb % 2 == 0;
}

hipError_t launch_solve128(const double* in, int64_t m, int n, int64_t ldin, const double* rbk, const int32_t* info, double* out,
                           int64_t ldout, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + 255) / 256)), block(256);
  if (full128(n, in, ldin, out, ldout))
    hipLaunchKernelGGL(solve128_kernel<true>, grid, block, 0, s, in, m, n, ldin, rbk, info, out, ldout);
  else
    hipLaunchKernelGGL(solve128_kernel<false>, grid, block, 0, s, in, m, n, ldin, rbk, info, out, ldout);
  return hipGetLastError();
}

hipError_t launch_syrk128(const double* Q0, int64_t m, int n, int64_t ldq, const int32_t* info, double* gpart, hipStream_t s) {
  const dim3 grid(kGramBlocks), block(256);
  if (n == 128)
    hipLaunchKernelGGL(syrk128_kernel<true>, grid, block, 0, s, Q0, m, n, ldq, info, gpart);
  else
    hipLaunchKernelGGL(syrk128_kernel<false>, grid, block, 0, s, Q0, m, n, ldq, info, gpart);
  return hipGetLastError();
}

}  // namespace rcqr
