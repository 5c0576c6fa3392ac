// Single-workgroup dense kernels on n x n and (<= 256) x n matrices.
//
//  qr_block_kernel   Householder QR, R factor only (Algorithm 1, step 2; Section 5.1 notes
//                    only R is needed).  Applied to blocks of <= 256 rows of W; when s2 > 256
//                    the blocks' R factors are stacked and factored again (a TSQR tree), which
//                    is still a product of Householder reflections applied to W.
//  finalize_r0       positive diagonal (rows of R scaled by the sign of their diagonal, which
//                    makes R0 the unique R of W), rank check, and the packed padded copy the
//                    streaming passes read (upper triangle row by row, reciprocal diagonal).
//  cholesky_kernel   R1 = chol(G) (Algorithm 2, step 2) and R = R1 R0 (Algorithm 3, step 3);
//                    with a nonzero shift coefficient c, chol(G + c trace(G) I), the first step
//                    of shifted CholeskyQR3 (trace(G) = ||V||_F^2 when G = V^T V).
#include "device_common.h"
#include "launch.h"

#include "../../include/rcqr.h"

namespace rcqr {

// ------------------------------------------------------------------------------------------
// Householder QR of a p x n block (p <= 256), matrix held in registers.
// Thread layout: column c = t / TPC, row group rg = t % TPC; a thread owns rows rg + TPC*e.
// The TPC threads of a column are consecutive lanes of one wave, so column reductions are wave
// shuffles, and the CPW = 64 / TPC columns of a wave form a panel.  Panel by panel: the owning
// wave computes the panel's reflectors one after another (each applied at once to the panel's
// later columns), with only wave-level LDS ordering; after one workgroup barrier every later
// column applies the panel's reflectors in order.  Reflector j maps column j's x = A[j:, j] to
// beta e1 with beta = -sign(x0) ||x||, H = I - tau v v^T, v[0] = 1.
// ------------------------------------------------------------------------------------------
constexpr int kQrMaxRows = 256;

template <int TPC, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = TPC / 2; off > 0; off >>= 1) v += shfl_xor_d(v, off);
  return v;
}

template <int NPAD, int TPC, class T>
__global__ __launch_bounds__(NPAD * TPC) void qr_block_kernel(const T* __restrict__ in, int64_t ldin, int64_t p_total,
                                                             int64_t rows_per_block, int n, T* __restrict__ out) {
  static_assert(TPC <= 64 && (64 % TPC) == 0, "a column's threads must sit in one wave");
  constexpr int EPT = kQrMaxRows / TPC;
  constexpr int CPW = 64 / TPC;  // columns per wave = panel width
  __shared__ T vbuf[2][CPW][kQrMaxRows];
  __shared__ T taub[2][CPW];
  const int t = threadIdx.x;
  const int c = t / TPC, rg = t % TPC;
  const int wave = t / kWave;
  const int64_t r_beg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p64 = p_total - r_beg < rows_per_block ? p_total - r_beg : rows_per_block;
  const int p = (int)p64;
  const T* A0 = in + r_beg * ldin;
  T a[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int r = rg + TPC * e;
    a[e] = (r < p && c < n) ? A0[(int64_t)r * ldin + c] : T(0);
  }
  const int steps = n < p ? n : p;
  // apply reflector (vb, tau) with leading row j to this thread's column
  auto apply = [&](const T* vb, T tau, int j) {
    T d = T(0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int r = rg + TPC * e;
      if (r >= j && r < p) d = fma_t(vb[r], a[e], d);
    }
    d = group_sum<TPC>(d);
    const T tw = tau * d;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int r = rg + TPC * e;
      if (r >= j && r < p) a[e] = fma_t(-tw, vb[r], a[e]);
    }
  };
  for (int q = 0, pi = 0; q < steps; q += CPW, ++pi) {
    const int buf = pi & 1;
    const int qend = q + CPW < steps ? q + CPW : steps;
    if (wave == q / CPW) {
      for (int j = q; j < qend; ++j) {
        const int jj = j - q;
        if (c == j) {
          T ss = T(0), alpha = T(0);
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int r = rg + TPC * e;
            if (r > j) ss = fma_t(a[e], a[e], ss);
            if (r == j) alpha = a[e];
          }
          ss = group_sum<TPC>(ss);
          alpha = group_sum<TPC>(alpha);  // only the owner of row j holds a nonzero term
          T tau = T(0), beta = alpha, scal = T(0);
          if (ss != T(0)) {
            beta = -copysign(sqrt(fma_t(alpha, alpha, ss)), alpha);
            tau = (beta - alpha) / beta;
            scal = T(1) / (alpha - beta);
          }
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int r = rg + TPC * e;
            if (r == j) {
              vbuf[buf][jj][r] = T(1);
              a[e] = beta;
            } else if (r > j) {
              vbuf[buf][jj][r] = a[e] * scal;
              a[e] = T(0);
            }
          }
          if (rg == 0) taub[buf][jj] = tau;
        }
        wave_lds_sync();
        if (c > j && c < qend) apply(vbuf[buf][jj], taub[buf][jj], j);
      }
    }
    __syncthreads();
    if (c >= qend && c < n) {
      for (int j = q; j < qend; ++j) apply(vbuf[buf][j - q], taub[buf][j - q], j);
    }
  }
  T* R = out + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int r = rg + TPC * e;
    if (r < n && c < n) R[r * n + c] = (c >= r) ? a[e] : T(0);
  }
}

template <class T>
static hipError_t qr_blocks_any(const T* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, T* out, int nblocks,
                                hipStream_t s) {
  if (rows_per_block > kQrMaxRows || n > RCQR_MAX_N || n < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks);
  if (n <= 8)
    hipLaunchKernelGGL((qr_block_kernel<8, 64, T>), grid, dim3(8 * 64), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 16)
    hipLaunchKernelGGL((qr_block_kernel<16, 16, T>), grid, dim3(16 * 16), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 32)
    hipLaunchKernelGGL((qr_block_kernel<32, 32, T>), grid, dim3(32 * 32), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 64)
    hipLaunchKernelGGL((qr_block_kernel<64, 16, T>), grid, dim3(64 * 16), 0, s, in, ldin, p_total, rows_per_block, n, out);
  else
    hipLaunchKernelGGL((qr_block_kernel<128, 8, T>), grid, dim3(128 * 8), 0, s, in, ldin, p_total, rows_per_block, n, out);
  return hipGetLastError();
}

hipError_t launch_qr_blocks(const double* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, double* out,
                            int nblocks, hipStream_t s) {
  return qr_blocks_any(in, ldin, p_total, rows_per_block, n, out, nblocks, s);
}

hipError_t launch_qr_blocks(const float* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, float* out,
                            int nblocks, hipStream_t s) {
  return qr_blocks_any(in, ldin, p_total, rows_per_block, n, out, nblocks, s);
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
template <class T>
__global__ __launch_bounds__(256) void finalize_r0_kernel(const T* __restrict__ rin, int n, int np, int32_t* __restrict__ info,
                                                          double* __restrict__ r0, double* __restrict__ r0pk) {
  __shared__ int bad;  // first failing column (1-based), or a value > n
  if (info[0] != 0) return;  // an earlier step failed: keep its status
  if (threadIdx.x == 0) bad = n + 1;
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double d = (double)rin[j * n + j];
    if (!(d != 0.0) || !isfinite(d)) atomicMin(&bad, j + 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad <= n) {
    info[0] = RCQR_E_RANK;
    info[1] = bad;
  }
  for (int i = threadIdx.x; i < np * np; i += blockDim.x) {
    const int r = i / np, c = i % np;
    double v = 0.0;
    if (r < n && c < n) {
      const double d = (double)rin[r * n + r];
      const double x = (double)rin[r * n + c];
      v = c >= r ? (d < 0.0 ? -x : x) : 0.0;
      r0[r * n + c] = v;
    }
    if (c >= r) put_packed(r0pk, np, n, r, c, v);
  }
}

hipError_t launch_finalize_r0(const double* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s) {
  hipLaunchKernelGGL(finalize_r0_kernel<double>, dim3(1), dim3(256), 0, s, rin, n, np, info, r0, r0pk);
  return hipGetLastError();
}

hipError_t launch_finalize_r0(const float* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s) {
  hipLaunchKernelGGL(finalize_r0_kernel<float>, dim3(1), dim3(256), 0, s, rin, n, np, info, r0, r0pk);
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

// trace of an LDS matrix with row stride ld, summed in index order
static __device__ double diag_sum(const double* a, int n, int ld) {
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += a[i * ld + i];
  return tr;
}

__global__ __launch_bounds__(256) void cholesky_kernel(const double* __restrict__ gc, int n, int np, const double* __restrict__ rprev,
                                                       double shift_coef, int32_t* __restrict__ info, double* __restrict__ g_out,
                                                       double* __restrict__ r1, double* __restrict__ r1pk, double* __restrict__ r_out,
                                                       int64_t ldr) {
  extern __shared__ double g[];  // n x n
  __shared__ int fail;
  __shared__ double shift;
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
  if (shift_coef != 0.0) {
    if (threadIdx.x == 0) shift = shift_coef * diag_sum(g, n, n);
    __syncthreads();
    if (threadIdx.x < n) g[threadIdx.x * n + threadIdx.x] += shift;
    __syncthreads();
  }
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

// Cholesky for np <= 64 with short, rolled loops (a fully unrolled single-wave factorization
// is tens of KB of straight-line code that runs once and is bound by instruction fetch).
// G lives in LDS (row-major, upper triangle; the lower triangle is scratch).  Wave 0 factors:
// step j divides row j by sqrt(G[j][j]) and lane c updates column c below row j,
// G[i][c] -= R1[j][i] R1[j][c] for j < i <= c.  Then all four waves form R = R1 Rprev.
template <int NP>
__global__ __launch_bounds__(256) void cholesky_small_kernel(const double* __restrict__ gc, int n, const double* __restrict__ rprev,
                                                             double shift_coef, int32_t* __restrict__ info, double* __restrict__ g_out,
                                                             double* __restrict__ r1, double* __restrict__ r1pk, double* __restrict__ r_out,
                                                             int64_t ldr) {
  __shared__ double G[NP * NP];
  __shared__ double P[NP * NP];  // Rprev, zero-padded
  __shared__ int fail;
  __shared__ double shift;
  if (info[0] != 0) return;
  constexpr int NB = NP / 16;
  const int t = threadIdx.x;
  for (int idx = t; idx < NP * NP; idx += blockDim.x) {
    const int i = idx / NP, c = idx % NP;
    double v = 0.0, pv = 0.0;
    if (i <= c && c < n) {
      v = gc[upper_block_index(i / 16, c / 16, NB) * 256 + (i % 16) * 16 + (c % 16)];
      pv = rprev[i * n + c];
    }
    G[idx] = v;
    P[idx] = pv;
    if (i < n && c < n) g_out[i * n + c] = v;
  }
  if (t == 0) fail = 0;
  __syncthreads();
  if (shift_coef != 0.0) {
    if (t == 0) shift = shift_coef * diag_sum(G, n, NP);
    __syncthreads();
    if (t < n) G[t * NP + t] += shift;
    __syncthreads();
  }
  if (t < kWave) {
    const int c = t;
    for (int j = 0; j < n; ++j) {
      const double d = G[j * NP + j];
      if (!(d > 0.0)) {  // NaN fails too; uniform across the wave
        if (c == 0) fail = j + 1;
        break;
      }
      const double rjj = sqrt(d);
      const double inv = 1.0 / rjj;
      if (c > j && c < n) G[j * NP + c] *= inv;
      if (c == j) G[j * NP + j] = rjj;
      wave_lds_sync();
      if (c > j && c < n) {
        const double rjc = G[j * NP + c];
        for (int i = j + 1; i <= c; ++i) G[i * NP + c] = __builtin_fma(-G[j * NP + i], rjc, G[i * NP + c]);
      }
      wave_lds_sync();
    }
  }
  __syncthreads();
  if (fail) {
    if (t == 0) {
      info[0] = RCQR_E_CHOL;
      info[1] = fail;
    }
    return;
  }
  // R1, its packed padded form, and R = R1 Rprev: R[i][c] = sum_{l = i..c} R1[i][l] Rprev[l][c]
  for (int idx = t; idx < NP * NP; idx += blockDim.x) {
    const int i = idx / NP, c = idx % NP;
    const double v = (i <= c && c < n) ? G[idx] : 0.0;
    if (i < n && c < n) r1[i * n + c] = v;
    if (c >= i) put_packed(r1pk, NP, n, i, c, v);
    if (i < n && c < n) {
      double acc = 0.0;
      if (i <= c)
        for (int l = i; l <= c; ++l) acc = __builtin_fma(G[i * NP + l], P[l * NP + c], acc);
      r_out[(int64_t)i * ldr + c] = acc;
    }
  }
}

hipError_t launch_cholesky(const double* gcompact, int n, int np, const double* rprev, double shift_coef, int32_t* info,
                           double* g_out, double* r1, double* r1pk, double* r_out, int64_t ldr, hipStream_t s) {
  if (np == 16) {
    hipLaunchKernelGGL(cholesky_small_kernel<16>, dim3(1), dim3(256), 0, s, gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr);
    return hipGetLastError();
  }
  if (np == 32) {
    hipLaunchKernelGGL(cholesky_small_kernel<32>, dim3(1), dim3(256), 0, s, gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr);
    return hipGetLastError();
  }
  if (np == 64) {
    hipLaunchKernelGGL(cholesky_small_kernel<64>, dim3(1), dim3(256), 0, s, gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr);
    return hipGetLastError();
  }
  const size_t lds = (size_t)n * n * sizeof(double);
  static bool attr_set = false;  // G of 128 x 128 needs 128 KiB of dynamic LDS
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)cholesky_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             RCQR_MAX_N * RCQR_MAX_N * (int)sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(256), lds, s, gcompact, n, np, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr);
  return hipGetLastError();
}

}  // namespace rcqr
