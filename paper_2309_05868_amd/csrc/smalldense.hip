// Single-workgroup dense kernels on n x n and (<= 256) x n matrices.
//
//  qr_block_kernel   Householder QR, R factor only (Algorithm 1, step 2; Section 5.1 notes
//                    only R is needed).  Applied to blocks of <= 256 rows of W; when s2 > 256
//                    the blocks' R factors are stacked and factored again (a TSQR tree), which
//                    is still a product of Householder reflections applied to W.
//  finalize_r0       positive diagonal (rows of R scaled by the sign of their diagonal, which
//                    makes R0 the unique R of W), rank check, and the packed padded copy the
//                    streaming passes read (upper triangle row by row, reciprocal diagonal).
//  cholesky_kernel   R1 = chol(G) (Algorithm 2, step 2) and R = R1 R0 (Algorithm 3, step 3).
#include "device_common.h"
#include "launch.h"

#include "../../include/rcqr.h"

namespace rcqr {

// ------------------------------------------------------------------------------------------
// Householder QR of a p x n block (p <= 256), matrix held in registers.
// Thread layout: column c = t / TPC, row group rg = t % TPC; a thread owns rows rg + TPC*e.
// The TPC threads of one column are consecutive lanes of one wave (TPC <= 64, power of two),
// so reductions over a column are wave shuffles; one barrier per reflector publishes v.
// ------------------------------------------------------------------------------------------
constexpr int kQrMaxRows = 256;

template <int NPAD>
__global__ __launch_bounds__(NPAD * (1024 / NPAD < 64 ? 1024 / NPAD : 64)) void qr_block_kernel(const double* __restrict__ in, int64_t ldin,
                                                                                                  int64_t p_total, int64_t rows_per_block, int n,
                                                                                                  double* __restrict__ out) {
  constexpr int TPC = 1024 / NPAD < 64 ? 1024 / NPAD : 64;
  constexpr int EPT = kQrMaxRows / TPC;
  __shared__ double vbuf[2][kQrMaxRows];
  __shared__ double taub[2];
  const int t = threadIdx.x;
  const int c = t / TPC, rg = t % TPC;
  const int64_t r_beg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p64 = p_total - r_beg < rows_per_block ? p_total - r_beg : rows_per_block;
  const int p = (int)p64;
  const double* A0 = in + r_beg * ldin;
  double a[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int r = rg + TPC * e;
    a[e] = (r < p && c < n) ? A0[(int64_t)r * ldin + c] : 0.0;
  }
  const int lane = lane_id();
  const int group_base = lane & ~(TPC - 1);
  const int steps = n < p ? n : p;
  for (int j = 0; j < steps; ++j) {
    const int buf = j & 1;
    if (c == j) {
      double ss = 0.0, alpha = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int r = rg + TPC * e;
        if (r > j) ss = __builtin_fma(a[e], a[e], ss);
        if (r == j) alpha = a[e];
      }
      for (int off = TPC / 2; off > 0; off >>= 1) {
        ss += shfl_xor_d(ss, off);
        alpha += shfl_xor_d(alpha, off);  // only the owner of row j holds a nonzero term
      }
      const double xnorm = sqrt(ss);
      double tau = 0.0, beta = alpha, denom = 1.0;
      if (xnorm != 0.0) {
        beta = -copysign(hypot(alpha, xnorm), alpha);
        tau = (beta - alpha) / beta;
        denom = alpha - beta;
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int r = rg + TPC * e;
        if (r == j) {
          vbuf[buf][r] = 1.0;
          a[e] = beta;
        } else if (r > j) {
          vbuf[buf][r] = xnorm != 0.0 ? a[e] / denom : 0.0;
          a[e] = 0.0;
        }
      }
      if (rg == 0) taub[buf] = tau;
    }
    (void)group_base;
    __syncthreads();
    if (c > j && c < n) {
      const double tau = taub[buf];
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int r = rg + TPC * e;
        if (r >= j && r < p) d = __builtin_fma(vbuf[buf][r], a[e], d);
      }
      for (int off = TPC / 2; off > 0; off >>= 1) d += shfl_xor_d(d, off);
      const double tw = tau * d;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int r = rg + TPC * e;
        if (r >= j && r < p) a[e] = __builtin_fma(-tw, vbuf[buf][r], a[e]);
      }
    }
  }
  double* R = out + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int r = rg + TPC * e;
    if (r < n && c < n) R[r * n + c] = (c >= r) ? a[e] : 0.0;
  }
}

hipError_t launch_qr_blocks(const double* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, double* out,
                            int nblocks, hipStream_t s) {
  if (rows_per_block > kQrMaxRows || n > RCQR_MAX_N || n < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks);
  if (n <= 8)
    hipLaunchKernelGGL(qr_block_kernel<8>, grid, dim3(8 * 64), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 16)
    hipLaunchKernelGGL(qr_block_kernel<16>, grid, dim3(1024), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 32)
    hipLaunchKernelGGL(qr_block_kernel<32>, grid, dim3(1024), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 64)
    hipLaunchKernelGGL(qr_block_kernel<64>, grid, dim3(1024), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else
    hipLaunchKernelGGL(qr_block_kernel<128>, grid, dim3(1024), 0, s, in, ldin, p_total, rows_per_block, n, out);
  return hipGetLastError();
}

// Offset of row k in the packed np x np upper-triangular format.
__device__ __forceinline__ int packed_row(int k, int np) { return k * np - k * (k - 1) / 2; }

// Position of entry (r, c), c >= r, of an np x np factor in the layout the streaming passes
// read: packed rows for np <= 64; for np = 128 the blocked layout
// [R00 packed (64) | R01 dense 64 x 64 row-major | R11 packed (64)].
__device__ __forceinline__ int factor_index(int np, int r, int c) {
  if (np <= 64) return packed_row(r, np) + (c - r);
  constexpr int H = 64, PK = H * (H + 1) / 2;
  if (r < H && c < H) return packed_row(r, H) + (c - r);
  if (r < H) return PK + r * H + (c - H);
  return PK + H * H + packed_row(r - H, H) + (c - r);
}

// Write entry (r, c), c >= r, of the identity-padded factor: v is R[r][c] for r, c < n; the
// diagonal is stored as its reciprocal.
__device__ __forceinline__ void put_packed(double* pk, int np, int n, int r, int c, double v) {
  double out;
  if (r < n && c < n)
    out = (r == c) ? 1.0 / v : v;
  else
    out = (r == c) ? 1.0 : 0.0;
  pk[factor_index(np, r, c)] = out;
}

// ------------------------------------------------------------------------------------------
// R0: positive diagonal, rank check, packed padded copy.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_r0_kernel(const double* __restrict__ rin, int n, int np, int32_t* __restrict__ info,
                                                          double* __restrict__ r0, double* __restrict__ r0pk) {
  __shared__ int bad;
  if (threadIdx.x == 0) {
    bad = 0;
    for (int j = 0; j < n; ++j) {
      const double d = rin[j * n + j];
      if (!(d != 0.0) || !isfinite(d)) {
        bad = j + 1;
        break;
      }
    }
    if (bad) {
      info[0] = RCQR_E_RANK;
      info[1] = bad;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < np * np; i += blockDim.x) {
    const int r = i / np, c = i % np;
    double v = 0.0;
    if (r < n && c < n) {
      const double d = rin[r * n + r];
      v = c >= r ? (d < 0.0 ? -rin[r * n + c] : rin[r * n + c]) : 0.0;
      r0[r * n + c] = v;
    }
    if (c >= r) put_packed(r0pk, np, n, r, c, v);
  }
}

hipError_t launch_finalize_r0(const double* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s) {
  hipLaunchKernelGGL(finalize_r0_kernel, dim3(1), dim3(256), 0, s, rin, n, np, info, r0, r0pk);
  return hipGetLastError();
}

__global__ void identity_factor_kernel(int n, int np, double* r0, double* r0pk) {
  for (int i = threadIdx.x; i < np * np; i += blockDim.x) {
    const int r = i / np, c = i % np;
    const double v = r == c ? 1.0 : 0.0;
    if (r < n && c < n) r0[r * n + c] = v;
    if (c >= r) put_packed(r0pk, np, n, r, c, v);
  }
}

hipError_t launch_identity_factor(int n, int np, double* r0, double* r0pk, hipStream_t s) {
  hipLaunchKernelGGL(identity_factor_kernel, dim3(1), dim3(256), 0, s, n, np, r0, r0pk);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Cholesky of G (compact upper 16x16 blocks of an np x np matrix), then R = R1 Rprev.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int upper_block_index(int a, int b, int nb) {
  // blocks (a, b), a <= b, numbered row by row
  return a * nb - a * (a - 1) / 2 + (b - a);
}

__global__ __launch_bounds__(256) void cholesky_kernel(const double* __restrict__ gc, int n, int np, const double* __restrict__ rprev,
                                                       int32_t* __restrict__ info, double* __restrict__ g_out, double* __restrict__ r1,
                                                       double* __restrict__ r1pk, double* __restrict__ r_out, int64_t ldr) {
  extern __shared__ double g[];  // n x n
  __shared__ int fail;
  if (info[0] != 0) return;
  const int nb = np / 16;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double v = 0.0;
    if (c >= r) {
      const int a = r / 16, b = c / 16;
      v = gc[upper_block_index(a, b, nb) * 256 + (r % 16) * 16 + (c % 16)];
    }
    g[i] = v;
    g_out[i] = v;
  }
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = g[j * n + j];
    if (!(d > 0.0)) {  // NaN fails too
      if (threadIdx.x == 0) {
        info[0] = RCQR_E_CHOL;
        info[1] = j + 1;
        fail = 1;
      }
      break;  // uniform: every thread read the same d
    }
    const double rjj = sqrt(d);
    __syncthreads();
    for (int c = j + 1 + threadIdx.x; c < n; c += blockDim.x) g[j * n + c] = g[j * n + c] / rjj;
    if (threadIdx.x == 0) g[j * n + j] = rjj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int a = j + 1 + idx / rem, b = j + 1 + idx % rem;
      if (b >= a) g[a * n + b] = __builtin_fma(-g[j * n + a], g[j * n + b], g[a * n + b]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) return;
  // R1 and its packed padded form
  for (int i = threadIdx.x; i < np * np; i += blockDim.x) {
    const int r = i / np, c = i % np;
    double v = 0.0;
    if (r < n && c < n) {
      v = c >= r ? g[r * n + c] : 0.0;
      r1[r * n + c] = v;
    }
    if (c >= r) put_packed(r1pk, np, n, r, c, v);
  }
  // R = R1 Rprev (both upper triangular): R[i][k] = sum_{l=i..k} R1[i][l] Rprev[l][k]
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double acc = 0.0;
    if (c >= r) {
      for (int l = r; l <= c; ++l) acc = __builtin_fma(g[r * n + l], rprev[l * n + c], acc);
    }
    r_out[(int64_t)r * ldr + c] = acc;
  }
}

hipError_t launch_cholesky(const double* gcompact, int n, int np, const double* rprev, int32_t* info, double* g_out,
                           double* r1, double* r1pk, double* r_out, int64_t ldr, hipStream_t s) {
  const size_t lds = (size_t)n * n * sizeof(double);
  static bool attr_set = false;  // G of 128 x 128 needs 128 KiB of dynamic LDS
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)cholesky_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             RCQR_MAX_N * RCQR_MAX_N * (int)sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(256), lds, s, gcompact, n, np, rprev, info, g_out, r1, r1pk, r_out, ldr);
  return hipGetLastError();
}

}  // namespace rcqr
