// Gram pass for 65..128 columns (rows padded to 128): G = Q0^T Q0 over the stored Q0 on FP64
// MFMA.  The 65..128-column row solves are in stream.hip (a 2 x 2 block substitution).
#include "device_common.h"
#include "launch.h"

namespace rcqr {

typedef double d4 __attribute__((ext_vector_type(4)));

// G partial = Q0^T Q0 over this workgroup's rows on FP64 MFMA, in the 36 upper 16x16 blocks of
// the 128 x 128 matrix.  This kernel forms the 26 blocks that involve columns 64..127; the 10
// blocks of columns 0..63 come from the pass that solved those columns (the 64-column Gram pass,
// which stores x_lo): workgroup b copies that pass's partial b into its slots (zeros past its
// grid), so one fixed-order reduction over the partials still gives G.  Four wave pairs per
// workgroup; waves 2p and 2p+1 read the same 4-row K-steps and accumulate 13 blocks each.  The
// operands of the next kSyrkAhead K-steps are in flight while a step's MFMAs run.  Fixed grid,
// fixed order.
constexpr int kSyrkPairs = 4;
constexpr int kSyrkAhead = 5;  // K-steps whose operands are loaded ahead of use

// Operands of one 4-row K-step: F[a] = Q0[row][16 a + csub] for the column blocks a >= a0 this
// wave multiplies (the others are not loaded).
template <bool FULL>
__device__ __forceinline__ void syrk_operands(double (&F)[8], const double* __restrict__ Q0, int64_t row, int64_t m, int n,
                                              int64_t ldq, int csub, int a0) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int c = 16 * a + csub;
    F[a] = (a >= a0 && row < m && (FULL || c < n)) ? Q0[row * ldq + c] : 0.0;
  }
}

template <bool FULL, bool BATCH>
__global__ __launch_bounds__(2 * kSyrkPairs * kWave) void syrk128_kernel(const double* __restrict__ Q0, int64_t m, int n, int64_t ldq,
                                                                       const int32_t* __restrict__ info, double* __restrict__ gpart,
                                                                       const double* __restrict__ gplo, int64_t nblo,
                                                                       MemberStride ms) {
  constexpr int NB = 8, NBU = NB * (NB + 1) / 2;  // 36 upper blocks
  constexpr int NL = 4, NLU = NL * (NL + 1) / 2;  // 10 of them within columns 0..63
  constexpr int HALF = (NBU - NLU) / 2;           // 13 blocks per wave
  __shared__ double gl[NBU * 256];
  if constexpr (BATCH) {  // batch member: its stored Q0 (in its Q) and workspace slice
    const int64_t mb = blockIdx.y, off = mb * ms.ws;
    info += off / (int64_t)sizeof(int32_t);
    gpart += off / (int64_t)sizeof(double);
    gplo += off / (int64_t)sizeof(double);
    if (ms.info != nullptr) {
      const MemberInfo& mi = member_info(ms, mb);
      Q0 = mi.Q;
      ldq = mi.ldq;
      m = mi.m;
      nblo = mi.gblocks;
    } else {
      Q0 += mb * ms.q;
    }
  }
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int set = wave & 1, pair = wave >> 1;
  {  // the blocks of columns 0..63: this workgroup's partial from the 64-column pass
    const bool have = (int64_t)blockIdx.x < nblo;
    const double* src = gplo + (int64_t)blockIdx.x * (NLU * 256);
    for (int i = threadIdx.x; i < NLU * 256; i += 2 * kSyrkPairs * kWave) {
      const int k = i / 256;
      const int a = k < 4 ? 0 : (k < 7 ? 1 : (k < 9 ? 2 : 3));
      const int b = a + (k - upper_blk(a, a, NL));
      gl[upper_blk(a, b, NB) * 256 + (i & 255)] = have ? src[i] : 0.0;
    }
  }
  d4 acc[HALF];
#pragma unroll
  for (int i = 0; i < HALF; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = (m + 3) / 4;  // 4-row MFMA K-steps
  const int rsub = lane >> 4, csub = lane & 15;
  const int64_t stride = (int64_t)gridDim.x * kSyrkPairs;
  int64_t st = (int64_t)blockIdx.x * kSyrkPairs + pair;
  // operands of the next kSyrkAhead K-steps in flight (a ring, unrolled so every index is fixed);
  // steps at or past nsteps read rows past m, which load as zeros and add exact zeros
  // set 0 multiplies column blocks 0..7 (blocks (0..2, 4..7) and (3, 4)), set 1 blocks 3..7
  const int a0 = set == 0 ? 0 : 3;
  double Fq[kSyrkAhead][NB];
#pragma unroll
  for (int k = 0; k < kSyrkAhead; ++k) syrk_operands<FULL>(Fq[k], Q0, 4 * (st + k * stride) + rsub, m, n, ldq, csub, a0);
  for (; st < nsteps; st += kSyrkAhead * stride) {
#pragma unroll
    for (int k = 0; k < kSyrkAhead; ++k) {
      double F[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) F[a] = Fq[k][a];
      syrk_operands<FULL>(Fq[k], Q0, 4 * (st + (k + kSyrkAhead) * stride) + rsub, m, n, ldq, csub, a0);
      int ab = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = a < NL ? NL : a; b < NB; ++b) {
          if (set == 0 && ab < HALF) acc[ab] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[a], F[b], acc[ab], 0, 0, 0);
          if (set == 1 && ab >= HALF) acc[ab - HALF] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[a], F[b], acc[ab - HALF], 0, 0, 0);
          ++ab;
        }
      }
    }
  }
  // fixed-order sum over the pairs; element e of lane l is D[l/16 + 4e][l%16]
  __syncthreads();
  for (int p = 0; p < kSyrkPairs; ++p) {
    if (pair == p) {
      auto put = [&](int blk, const d4& v) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = blk * 256 + ((lane >> 4) + 4 * e) * 16 + (lane & 15);
          gl[idx] = (p == 0) ? v[e] : gl[idx] + v[e];
        }
      };
      int ab = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = a < NL ? NL : a; b < NB; ++b) {
          if (set == 0 && ab < HALF) put(upper_blk(a, b, NB), acc[ab]);
          if (set == 1 && ab >= HALF) put(upper_blk(a, b, NB), acc[ab - HALF]);
          ++ab;
        }
      }
    }
    __syncthreads();
  }
  double* outp = gpart + (int64_t)blockIdx.x * (NBU * 256);
  for (int i = threadIdx.x; i < NBU * 256; i += 2 * kSyrkPairs * kWave) outp[i] = gl[i];
}

hipError_t launch_syrk128(const double* Q0, int64_t m, int n, int64_t ldq, const int32_t* info, double* gpart, const double* gplo,
                          int64_t nblo, hipStream_t s, const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  const dim3 grid(kGramBlocks, ms.count), block(2 * kSyrkPairs * kWave);
  const bool batch = ms.count > 1 || ms.info != nullptr;
  if (batch) {
    if (n == 128)
      hipLaunchKernelGGL((syrk128_kernel<true, true>), grid, block, 0, s, Q0, m, n, ldq, info, gpart, gplo, nblo, ms);
    else
      hipLaunchKernelGGL((syrk128_kernel<false, true>), grid, block, 0, s, Q0, m, n, ldq, info, gpart, gplo, nblo, ms);
  } else {
    if (n == 128)
      hipLaunchKernelGGL((syrk128_kernel<true, false>), grid, block, 0, s, Q0, m, n, ldq, info, gpart, gplo, nblo, ms);
    else
      hipLaunchKernelGGL((syrk128_kernel<false, false>), grid, block, 0, s, Q0, m, n, ldq, info, gpart, gplo, nblo, ms);
  }
  return hipGetLastError();
}

}  // namespace rcqr
