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
// Householder QR of a p x n block (p <= 256, n <= 128), R factor only, matrix in registers.
// Sixteen waves; wave w owns columns w, w + 16, ... (NC of them) and lane l owns rows l, l + 64,
// l + 128, l + 192, so every column reduction is one wave's butterfly.  Reflector j is built by
// the owner of column j: it maps x = A[j:, j] to beta e1, beta = -sign(x0) ||x||,
// H = I - tau v v^T with v[0] = 1; v and tau go through LDS (double-buffered, so one workgroup
// barrier per reflector) and every wave applies H to its columns right of j.
// ------------------------------------------------------------------------------------------
constexpr int kQrMaxRows = 256;
constexpr int kQrWaves = 16;


template <int NC, class T>
__global__ __launch_bounds__(kQrWaves * kWave) void qr_block_kernel(const T* __restrict__ in, int64_t ldin, int64_t p_total,
                                                                    int64_t rows_per_block, int n, T* __restrict__ out) {
  constexpr int ER = kQrMaxRows / kWave;  // rows per lane
  __shared__ T vbuf[2][kQrMaxRows];
  __shared__ T taub[2];
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t r_beg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p64 = p_total - r_beg < rows_per_block ? p_total - r_beg : rows_per_block;
  const int p = (int)p64;
  const T* A0 = in + r_beg * ldin;
  T a[NC][ER];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = wave + kQrWaves * q;
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int r = lane + kWave * e;
      a[q][e] = (r < p && c < n) ? A0[(int64_t)r * ldin + c] : T(0);
    }
  }
  const int steps = n < p ? n : p;
  for (int j = 0; j < steps; ++j) {
    const int buf = j & 1;
    if (wave == (j % kQrWaves)) {
      const int oq = j / kQrWaves;
      T x[ER];
#pragma unroll
      for (int e = 0; e < ER; ++e) x[e] = T(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q == oq) {
#pragma unroll
          for (int e = 0; e < ER; ++e) x[e] = a[q][e];
        }
      T ss = T(0);
#pragma unroll
      for (int e = 0; e < ER; ++e) {
        const int r = lane + kWave * e;
        if (r > j) ss = fma_t(x[e], x[e], ss);
      }
      ss = wave_reduce_sum(ss);
      T xsel = T(0);
#pragma unroll
      for (int e = 0; e < ER; ++e) xsel = (e == (j / kWave)) ? x[e] : xsel;
      const T alpha = readlane_d(xsel, j % kWave);
      T tau = T(0), beta = alpha, scal = T(0);
      if (ss != T(0)) {
        beta = -copysign(sqrt(fma_t(alpha, alpha, ss)), alpha);
        tau = (beta - alpha) / beta;
        scal = T(1) / (alpha - beta);
      }
#pragma unroll
      for (int e = 0; e < ER; ++e) {
        const int r = lane + kWave * e;
        vbuf[buf][r] = (r == j) ? T(1) : (r > j ? x[e] * scal : T(0));
        x[e] = (r == j) ? beta : (r > j ? T(0) : x[e]);
      }
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q == oq) {
#pragma unroll
          for (int e = 0; e < ER; ++e) a[q][e] = x[e];
        }
      if (lane == 0) taub[buf] = tau;
    }
    __syncthreads();
    const T tau = taub[buf];
    if (tau != T(0)) {
      T v[ER];
#pragma unroll
      for (int e = 0; e < ER; ++e) v[e] = vbuf[buf][lane + kWave * e];
      T d[NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        d[q] = T(0);
        const int c = wave + kQrWaves * q;
        if (c > j && c < n) {
#pragma unroll
          for (int e = 0; e < ER; ++e) d[q] = fma_t(v[e], a[q][e], d[q]);
          d[q] = wave_reduce_sum(d[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int c = wave + kQrWaves * q;
        if (c > j && c < n) {
          const T tw = tau * d[q];
#pragma unroll
          for (int e = 0; e < ER; ++e) a[q][e] = fma_t(-tw, v[e], a[q][e]);
        }
      }
    }
  }
  T* R = out + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = wave + kQrWaves * q;
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int r = lane + kWave * e;
      if (r < n && c < n) R[r * n + c] = (c >= r) ? a[q][e] : T(0);
    }
  }
}

template <class T>
static hipError_t qr_blocks_any(const T* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, T* out, int nblocks,
                                hipStream_t s) {
  if (rows_per_block > kQrMaxRows || n > RCQR_MAX_N || n < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks), block(kQrWaves * kWave);
  if (n <= 16)
    hipLaunchKernelGGL((qr_block_kernel<1, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 32)
    hipLaunchKernelGGL((qr_block_kernel<2, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out);
  else if (n <= 64)
    hipLaunchKernelGGL((qr_block_kernel<4, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out);
  else
    hipLaunchKernelGGL((qr_block_kernel<8, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out);
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

// Cholesky for 65..128 columns: four waves; thread t holds rows 64h .. 64h+63 (h = t / 128) of
// column c = t % 128 of G in registers.  Per step j the pivot and row j of R1 are exchanged
// through LDS (three barriers per step).  G and R1 sit in dynamic LDS (n x n) for loading and
// for R = R1 Rprev.
constexpr int kChol128Threads = 256;

__global__ __launch_bounds__(kChol128Threads) void cholesky_kernel(const double* __restrict__ gc, int n, int np,
                                                                   const double* __restrict__ rprev, double shift_coef,
                                                                   int32_t* __restrict__ info, double* __restrict__ g_out,
                                                                   double* __restrict__ r1, double* __restrict__ r1pk,
                                                                   double* __restrict__ r_out, int64_t ldr) {
  constexpr int NPX = 128, HR = 64;
  extern __shared__ double g[];  // n x n
  __shared__ double rowb[NPX];
  __shared__ double pivb;
  __shared__ double shift;
  if (info[0] != 0) return;
  const int t = threadIdx.x;
  const int nb = np / 16;
  for (int i = t; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double v = 0.0;
    if (c >= r) {
      const int a = r / 16, b = c / 16;
      v = gc[upper_block_index(a, b, nb) * 256 + (r % 16) * 16 + (c % 16)];
    }
    g[i] = v;
    g_out[i] = v;
  }
  __syncthreads();
  if (shift_coef != 0.0) {
    if (t == 0) shift = shift_coef * diag_sum(g, n, n);
    __syncthreads();
    if (t < n) g[t * n + t] += shift;
    __syncthreads();
  }
  const int c = t % NPX, h = t / NPX, r0 = HR * h;
  double col[HR];  // G[r0 + i][c]
#pragma unroll
  for (int i = 0; i < HR; ++i) {
    const int r = r0 + i;
    col[i] = (r < n && c < n && r <= c) ? g[(r < n ? r : 0) * n + (c < n ? c : 0)] : 0.0;
  }
  constexpr int CK = 8;
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    const bool mine = (j / HR) == h;  // this thread's half holds row j
    const int jl = j - r0;            // row j's index in this half (valid when mine)
    double gjc = 0.0;
    if (mine) {
#pragma unroll
      for (int i0 = 0; i0 < HR; i0 += CK) {
        if (jl >= i0 && jl < i0 + CK) {
#pragma unroll
          for (int i = i0; i < i0 + CK; ++i) gjc = (i == jl) ? col[i] : gjc;
        }
      }
      if (c == j) pivb = gjc;
    }
    __syncthreads();
    const double d = pivb;
    if (!(d > 0.0)) {  // NaN fails too; every thread read the same pivot
      bad = j + 1;
      break;
    }
    if (mine) {
      const double rjj = sqrt(d);
      const double inv = 1.0 / rjj;
      const double rjc = (c == j) ? rjj : (c > j ? gjc * inv : 0.0);
#pragma unroll
      for (int i0 = 0; i0 < HR; i0 += CK) {
        if (jl >= i0 && jl < i0 + CK) {
#pragma unroll
          for (int i = i0; i < i0 + CK; ++i) col[i] = (i == jl) ? rjc : col[i];
        }
      }
      rowb[c] = rjc;
    }
    __syncthreads();
    const double rjc = rowb[c];
#pragma unroll
    for (int i0 = 0; i0 < HR; i0 += CK) {
      if (r0 + i0 + CK - 1 > j) {
#pragma unroll
        for (int i = i0; i < i0 + CK; ++i) {
          const int r = r0 + i;
          const double rji = rowb[r];
          const double upd = __builtin_fma(-rji, rjc, col[i]);
          col[i] = (r > j && c >= r) ? upd : col[i];
        }
      }
    }
    __syncthreads();  // rowb and pivb are rewritten by the next step
  }
  if (bad) {
    if (t == 0) {
      info[0] = RCQR_E_CHOL;
      info[1] = bad;
    }
    return;  // uniform: every thread saw the same pivot
  }
  if (c < n) {
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int r = r0 + i;
      if (r < n) g[r * n + c] = (r <= c) ? col[i] : 0.0;
    }
  }
  __syncthreads();
  // R1 and its packed padded form
  for (int i = t; i < np * np; i += blockDim.x) {
    const int r = i / np, cc = i % np;
    double v = 0.0;
    if (r < n && cc < n) {
      v = cc >= r ? g[r * n + cc] : 0.0;
      r1[r * n + cc] = v;
    }
    if (cc >= r) put_packed(r1pk, np, n, r, cc, v);
  }
  // R = R1 Rprev (both upper triangular): R[i][k] = sum_{l=i..k} R1[i][l] Rprev[l][k]
  for (int i = t; i < n * n; i += blockDim.x) {
    const int r = i / n, cc = i % n;
    double acc = 0.0;
    if (cc >= r) {
      for (int l = r; l <= cc; ++l) acc = __builtin_fma(g[r * n + l], rprev[l * n + cc], acc);
    }
    r_out[(int64_t)r * ldr + cc] = acc;
  }
}

// Cholesky for np <= 64.  Wave 0 factors with column c of G in lane c's registers (the step
// loop is rolled, the loop over rows unrolled, so the code stays small); R1 goes back to LDS and
// all four waves form R = R1 Rprev.
template <int NP>
__global__ __launch_bounds__(256) void cholesky_small_kernel(const double* __restrict__ gc, int n, const double* __restrict__ rprev,
                                                             double shift_coef, int32_t* __restrict__ info, double* __restrict__ g_out,
                                                             double* __restrict__ r1, double* __restrict__ r1pk, double* __restrict__ r_out,
                                                             int64_t ldr) {
  __shared__ double G[NP * NP];
  __shared__ double P[NP * NP];  // Rprev, zero-padded
  __shared__ double rowb[NP];
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
    // lane c holds column c of G in registers; step j: row j of R1 is R1[j][c] = G[j][c] / r_jj,
    // then G[i][c] -= R1[j][i] R1[j][c] for j < i <= c with R1[j][i] broadcast through LDS.
    // Rows go in chunks of 8: a chunk wholly at or above row j is skipped (uniform branch), the
    // rest is branch-free so the LDS reads pipeline.
    constexpr int CK = 8;
    const int c = t;
    double g[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) g[i] = (c < NP) ? G[i * NP + (c < NP ? c : 0)] : 0.0;
    int bad = 0;
    for (int j = 0; j < n; ++j) {
      double gjc = 0.0;
#pragma unroll
      for (int i0 = 0; i0 < NP; i0 += CK) {
        if (j >= i0 && j < i0 + CK) {
#pragma unroll
          for (int i = i0; i < i0 + CK; ++i) gjc = (i == j) ? g[i] : gjc;
        }
      }
      const double d = readlane_d(gjc, j);
      if (!(d > 0.0)) {  // NaN fails too; uniform across the wave
        bad = j + 1;
        break;
      }
      const double rjj = sqrt(d);
      const double inv = 1.0 / rjj;
      const double rjc = (c == j) ? rjj : (c > j ? gjc * inv : 0.0);
#pragma unroll
      for (int i0 = 0; i0 < NP; i0 += CK) {
        if (j >= i0 && j < i0 + CK) {
#pragma unroll
          for (int i = i0; i < i0 + CK; ++i) g[i] = (i == j) ? rjc : g[i];
        }
      }
      if (c < NP) rowb[c] = rjc;
      wave_lds_sync();
#pragma unroll
      for (int i0 = 0; i0 < NP; i0 += CK) {
        if (i0 + CK - 1 > j) {
#pragma unroll
          for (int i = i0; i < i0 + CK; ++i) {
            const double rji = rowb[i];
            const double upd = __builtin_fma(-rji, rjc, g[i]);
            g[i] = (i > j && c >= i) ? upd : g[i];
          }
        }
      }
      wave_lds_sync();
    }
    if (c == 0) fail = bad;
    if (c < NP) {
#pragma unroll
      for (int i = 0; i < NP; ++i) G[i * NP + c] = (i <= c) ? g[i] : 0.0;
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
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(kChol128Threads), lds, s, gcompact, n, np, rprev, shift_coef, info, g_out, r1,
                     r1pk, r_out, ldr);
  return hipGetLastError();
}

}  // namespace rcqr
