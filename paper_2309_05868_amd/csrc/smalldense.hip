// Single-workgroup dense kernels on n x n and (<= 256) x n matrices.
//
//  qr_block_kernel   Householder QR, R factor only (Algorithm 1, step 2; Section 5.1 notes
//                    only R is needed).  Applied to blocks of <= 256 rows of W; when s2 > 256
//                    the blocks' R factors are stacked and factored again (a TSQR tree), which
//                    is still a product of Householder reflections applied to W.  The last
//                    level also makes R0 of its R: positive diagonal (rows scaled by the sign of
//                    their diagonal, which makes R0 the unique R of W), rank check, and the packed
//                    padded copy the streaming passes read (upper triangle row by row, reciprocal
//                    diagonal).
//  finalize_r0       the same for an R held in memory (the second Cholesky QR's R1 R0).
//  cholesky_kernel   R1 = chol(G) (Algorithm 2, step 2) and R = R1 R0 (Algorithm 3, step 3);
//                    with a nonzero shift coefficient c, chol(G + c trace(G) I), the first step
//                    of shifted CholeskyQR3 (trace(G) = ||V||_F^2 when G = V^T V).
#include "device_common.h"
#include "launch.h"

#include "../../include/rcqr.h"

namespace rcqr {

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
// Householder QR of a p x n block (p <= 256, n <= 128), R factor only, matrix in registers.
// Sixteen waves; lane l owns rows l, l + 64, l + 128, l + 192, so every column reduction is one
// wave's butterfly.  Reflector j maps x = A[j:, j] to beta e1, beta = -sign(x0) ||x||,
// H = I - tau v v^T with v[0] = 1.  Reflectors are made two at a time: wave w owns the column
// pairs (2w, 2w + 1), (2w + 32, 2w + 33), ...; the owner of pair (j, j + 1) builds H_j, applies it
// to column j + 1 and builds H_{j+1}, and both go through LDS (double-buffered) behind one
// workgroup barrier, after which every wave applies H_j and then H_{j+1} to its columns right of
// j + 1.  Look-ahead: the owner of the next pair updates that pair first and publishes its two
// reflectors before its other columns, at raised wave priority.  Every column still receives
// H_0, H_1, ... in order through the same operations, so the factor is the same as with one
// reflector per barrier; only the number of barriers halves.
// ------------------------------------------------------------------------------------------
constexpr int kQrMaxRows = 256;
constexpr int kQrWaves = 16;

//
// Last level of the tree (fin.r0 set, one block): instead of R the kernel writes what R0 is used
// as, from its registers: R0 with a positive diagonal (rows of R with a negative diagonal entry
// negated) into fin.r0, its packed padded form into fin.r0pk, and the rank check into info (a
// zero or non-finite diagonal entry: RCQR_E_RANK and the first such column, unless an earlier
// step already failed, in which case nothing is written) -- the work of finalize_r0_kernel
// without a launch of its own.
struct QrFinal {
  double* r0;
  double* r0pk;
  int32_t* info;
  int np;
};

template <int NC, class T>
__global__ __launch_bounds__(kQrWaves * kWave) void qr_block_kernel(const T* __restrict__ in, int64_t ldin, int64_t p_total,
                                                                    int64_t rows_per_block, int n, T* __restrict__ out,
                                                                    int64_t member_bytes, QrFinal fin) {
  static_assert(NC % 2 == 0, "columns are owned in pairs");
  constexpr int ER = kQrMaxRows / kWave;  // rows per lane
  in = member_ptr(in, (int64_t)blockIdx.y * member_bytes);  // batch member
  out = member_ptr(out, (int64_t)blockIdx.y * member_bytes);
  const bool final_level = fin.r0 != nullptr;
  int32_t status0 = 0;
  if (final_level) {
    fin.r0 = member_ptr(fin.r0, (int64_t)blockIdx.y * member_bytes);
    fin.r0pk = member_ptr(fin.r0pk, (int64_t)blockIdx.y * member_bytes);
    fin.info = member_ptr(fin.info, (int64_t)blockIdx.y * member_bytes);
    status0 = fin.info[0];  // read early; used at the end
  }
  __shared__ T vbuf[2][2][kQrMaxRows];  // [pair parity][first / second reflector of the pair]
  __shared__ T taub[2][2];
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t r_beg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p64 = p_total - r_beg < rows_per_block ? p_total - r_beg : rows_per_block;
  const int p = (int)p64;
  const T* A0 = in + r_beg * ldin;
  // slot q of wave w holds column 32 (q / 2) + 2 w + (q % 2)
  auto col_of = [&](int q) { return 32 * (q / 2) + 2 * wave + (q % 2); };
  T a[NC][ER];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = col_of(q);
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int r = lane + kWave * e;
      a[q][e] = (r < p && c < n) ? A0[(int64_t)r * ldin + c] : T(0);
    }
  }
  // Reflector j from the owner's (fully updated) column j, in slot oq: into vbuf[buf][half] /
  // taub[buf][half] and into v (this lane's entries), tau.
  auto make_reflector = [&](int j, int oq, int buf, int half, T (&v)[ER], T& tau_out) {
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
      v[e] = (r == j) ? T(1) : (r > j ? x[e] * scal : T(0));
      vbuf[buf][half][r] = v[e];
      x[e] = (r == j) ? beta : (r > j ? T(0) : x[e]);
    }
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (q == oq) {
#pragma unroll
        for (int e = 0; e < ER; ++e) a[q][e] = x[e];
      }
    if (lane == 0) taub[buf][half] = tau;
    tau_out = tau;
  };
  // H applied to the wave's slot q: a -= tau (v . a) v
  auto apply = [&](int q, T tau, const T (&v)[ER]) {
    if (tau != T(0)) {
      T d = T(0);
#pragma unroll
      for (int e = 0; e < ER; ++e) d = fma_t(v[e], a[q][e], d);
      d = wave_reduce_sum(d);
      const T tw = tau * d;
#pragma unroll
      for (int e = 0; e < ER; ++e) a[q][e] = fma_t(-tw, v[e], a[q][e]);
    }
  };
  const int steps = n < p ? n : p;
  const int npairs = (steps + 1) / 2;
  // Pair pp, made by its owner (wave pp % 16, slots 2 (pp / 16) and 2 (pp / 16) + 1).
  auto make_pair = [&](int pp) {
    const int j = 2 * pp, q0 = 2 * (pp / kQrWaves), buf = pp & 1;
    T v0[ER], tau0;
    make_reflector(j, q0, buf, 0, v0, tau0);
    if (j + 1 < steps) {
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q == q0 + 1) apply(q, tau0, v0);
      T v1[ER], tau1;
      make_reflector(j + 1, q0 + 1, buf, 1, v1, tau1);
    } else if (lane == 0) {
      taub[buf][1] = T(0);  // odd number of steps: the pair has one reflector
    }
  };
  if (npairs > 0 && wave == 0) make_pair(0);
  for (int pp = 0; pp < npairs; ++pp) {
    __syncthreads();  // pair pp published; every read of pair pp - 1 is done
    const int j = 2 * pp, buf = pp & 1;
    const T tau0 = taub[buf][0], tau1 = taub[buf][1];
    T v0[ER], v1[ER];
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      v0[e] = vbuf[buf][0][lane + kWave * e];
      v1[e] = vbuf[buf][1][lane + kWave * e];
    }
    // columns right of j + 1 take H_j, then H_{j+1}
    auto update = [&](int q) {
      const int c = col_of(q);
      if (c > j + 1 && c < n) {
        apply(q, tau0, v0);
        apply(q, tau1, v1);
      }
    };
    const int nxt = pp + 1;
    if (nxt < npairs && wave == nxt % kQrWaves) {
      const int nq = 2 * (nxt / kQrWaves);
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q == nq || q == nq + 1) update(q);
      make_pair(nxt);
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q != nq && q != nq + 1) update(q);
    } else {
#pragma unroll
      for (int q = 0; q < NC; ++q) update(q);
    }
  }
  if (!final_level) {
    T* R = out + (int64_t)blockIdx.x * n * n;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = col_of(q);
#pragma unroll
      for (int e = 0; e < ER; ++e) {
        const int r = lane + kWave * e;
        if (r < n && c < n) R[r * n + c] = (c >= r) ? a[q][e] : T(0);
      }
    }
    return;
  }
  if (status0 != 0) return;  // an earlier step failed: keep its status (uniform)
  __shared__ double dg[kQrMaxRows];
  __shared__ int bad;  // first failing column (1-based), or a value > n
  if (threadIdx.x == 0) bad = n + 1;
  // the diagonal entry of column c sits in its owner's lane c % 64, row slot c / 64
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = col_of(q);
    if (c < n && lane == c % kWave) {
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < ER; ++e) d = (e == c / kWave) ? (double)a[q][e] : d;
      dg[c] = d;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double d = dg[j];
    if (!(d != 0.0) || !isfinite(d)) atomicMin(&bad, j + 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad <= n) {
    fin.info[0] = RCQR_E_RANK;
    fin.info[1] = bad;
  }
  const int np = fin.np;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = col_of(q);
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int r = lane + kWave * e;
      if (r < np && c < np) {
        double v = 0.0;
        if (r < n && c < n) {
          const double x = (double)a[q][e];
          v = c >= r ? (dg[r] < 0.0 ? -x : x) : 0.0;
          fin.r0[r * n + c] = v;
        }
        if (c >= r) put_packed(fin.r0pk, np, n, r, c, v);
      }
    }
  }
}

template <class T>
static hipError_t qr_blocks_any(const T* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, T* out, int nblocks,
                                hipStream_t s, const MemberStride& ms, QrFinal fin) {
  if (rows_per_block > kQrMaxRows || n > RCQR_MAX_N || n < 1 || ms.count < 1) return hipErrorInvalidValue;
  if (fin.r0 != nullptr && (nblocks != 1 || fin.np < n || fin.np > 16 * (n <= 32 ? 2 : (n <= 64 ? 4 : 8))))
    return hipErrorInvalidValue;  // the last level is one block, and its column slots cover np
  const dim3 grid((unsigned)nblocks, ms.count), block(kQrWaves * kWave);
  const int64_t mbytes = ms.ws;
  if (n <= 32)
    hipLaunchKernelGGL((qr_block_kernel<2, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out, mbytes, fin);
  else if (n <= 64)
    hipLaunchKernelGGL((qr_block_kernel<4, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out, mbytes, fin);
  else
    hipLaunchKernelGGL((qr_block_kernel<8, T>), grid, block, 0, s, in, ldin, p_total, rows_per_block, n, out, mbytes, fin);
  return hipGetLastError();
}

hipError_t launch_qr_blocks(const double* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, double* out,
                            int nblocks, hipStream_t s, const MemberStride& ms, double* r0, double* r0pk, int32_t* info, int np) {
  return qr_blocks_any(in, ldin, p_total, rows_per_block, n, out, nblocks, s, ms, QrFinal{r0, r0pk, info, np});
}

hipError_t launch_qr_blocks(const float* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, float* out,
                            int nblocks, hipStream_t s, const MemberStride& ms, double* r0, double* r0pk, int32_t* info, int np) {
  return qr_blocks_any(in, ldin, p_total, rows_per_block, n, out, nblocks, s, ms, QrFinal{r0, r0pk, info, np});
}

// ------------------------------------------------------------------------------------------
// R0: positive diagonal, rank check, packed padded copy.
// ------------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void finalize_r0_kernel(const T* __restrict__ rin, int n, int np, int32_t* __restrict__ info,
                                                          double* __restrict__ r0, double* __restrict__ r0pk, int64_t member_bytes) {
  __shared__ int bad;  // first failing column (1-based), or a value > n
  {
    const int64_t off = (int64_t)blockIdx.y * member_bytes;  // batch member
    rin = member_ptr(rin, off);
    info = member_ptr(info, off);
    r0 = member_ptr(r0, off);
    r0pk = member_ptr(r0pk, off);
  }
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

hipError_t launch_finalize_r0(const double* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s,
                              const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_r0_kernel<double>, dim3(1, ms.count), dim3(256), 0, s, rin, n, np, info, r0, r0pk, ms.ws);
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

// Cholesky of G (np <= 128 padded columns) by one workgroup of NWV waves, in the LDL^T order
// and by blocks of four rows.  Thread (wave w, lane l) keeps G[i][c] in registers for the rows
// of its row blocks, i = 4 (w + NWV kb) + r, and for columns c = l + 64 q, so no register is ever
// indexed by a run-time value.  Step J (rows 4J .. 4J+3): the wave owning that block eliminates
// inside it on its own (pivots and coupling coefficients read from the owning lanes; no workgroup
// barrier), writes the four rows G[4J + r][.] and 1/pivot to LDS and, after one barrier, every
// thread applies the rank-4 update G[i][c] -= sum_r (G[4J+r][i] / d_r) G[4J+r][c] to its rows
// below the block (j < i <= c, branch-free).  Look-ahead: the owner of block J + 1 updates that
// block first and publishes it, at raised wave priority, before its other rows (the operations
// on every row are unchanged, only their order across rows).  A pivot that is not > 0 (NaN included) stops every
// thread at the same step.  R1[j][j] = sqrt(d_j), R1[j][c] = G[j][c] / sqrt(d_j) are formed at
// the end for all rows at once.
template <int NP>
struct CholShape {
  static constexpr int NWV = NP >= 64 ? 16 : 4;  // waves (one 4-row block per wave at 64, two at 128)
  static constexpr int CPL = NP > 64 ? 2 : 1;   // columns per lane
  static constexpr int BR = 4;                  // rows per block
  static constexpr int NBT = NP / (NWV * BR);   // row blocks per thread
};

template <int NP>
__global__ __launch_bounds__(CholShape<NP>::NWV * kWave) void cholesky_kernel(const double* __restrict__ gc, int n,
                                                                              const double* __restrict__ rprev, double shift_coef,
                                                                              int32_t* __restrict__ info, double* __restrict__ g_out,
                                                                              double* __restrict__ r1, double* __restrict__ r1pk,
                                                                              double* __restrict__ r_out, int64_t ldr, MemberStride ms) {
  constexpr int NWV = CholShape<NP>::NWV, CPL = CholShape<NP>::CPL, BR = CholShape<NP>::BR, NBT = CholShape<NP>::NBT;
  {
    const int64_t mb = blockIdx.y, off = mb * ms.ws;  // batch member
    gc = member_ptr(gc, off);
    rprev = member_ptr(rprev, off);
    info = member_ptr(info, off);
    g_out = member_ptr(g_out, off);
    r1 = member_ptr(r1, off);
    r1pk = member_ptr(r1pk, off);
    if (ms.info != nullptr) {  // ragged batch: the member's own R
      const MemberInfo& mi = member_info(ms, mb);
      r_out = mi.R;
      ldr = mi.ldr;
    } else {
      r_out += mb * ms.r;
    }
  }
  constexpr int NB = NP / 16;
  extern __shared__ double Rl[];  // NP x NP, the rows of the LDL^T elimination; then Rprev (NP <= 64)
  double* rp = Rl + NP * NP;
  __shared__ double sdiag[NP];
  __shared__ double dinvb[2][BR];
  __shared__ int failb[2];
  __shared__ double wsum[NWV];
  if (info[0] != 0) return;
  const int t = threadIdx.x, w = t / kWave, l = lane_id();
  double g[NBT][BR][CPL];
  double diag = 0.0;
#pragma unroll
  for (int kb = 0; kb < NBT; ++kb)
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int i = BR * (w + NWV * kb) + r;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = l + kWave * q;
        double v = 0.0;
        if (i <= c && c < n) v = gc[upper_block_index(i / 16, c / 16, NB) * 256 + (i % 16) * 16 + (c % 16)];
        g[kb][r][q] = v;
        if (i == c) diag += v;
        if (i < n && c < n) g_out[i * n + c] = v;
      }
    }
  if (shift_coef != 0.0) {  // G + shift_coef * trace(G) * I; the trace summed in a fixed order
    const double ws = wave_reduce_sum(diag);
    if (l == 0) wsum[w] = ws;
    __syncthreads();
    double tr = 0.0;
    for (int k = 0; k < NWV; ++k) tr += wsum[k];
    const double shift = shift_coef * tr;
#pragma unroll
    for (int kb = 0; kb < NBT; ++kb)
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int q = 0; q < CPL; ++q)
          if (BR * (w + NWV * kb) + r == l + kWave * q && l + kWave * q < n) g[kb][r][q] += shift;
  }
  int bad = 0;
  const int nblk = (n + BR - 1) / BR;
  // In-block elimination of row block J by its owner (rows already updated by every earlier
  // block): pivots and coupling coefficients from the owning lanes, rows to LDS.
  auto eliminate = [&](int J) {
    const int buf = J & 1;
    const int j0 = BR * J;
    const int kJ = J / NWV;
    double rows[BR][CPL];
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        double v = 0.0;
#pragma unroll
        for (int kb = 0; kb < NBT; ++kb) v = (kb == kJ) ? g[kb][r][q] : v;
        rows[r][q] = v;
      }
    // column j0 + r lives in lane (j0 + r) % 64 of part (j0 + r) / 64 (the same part for the block)
    const int qj = (CPL > 1 && j0 >= kWave) ? 1 : 0;
    int fail = 0;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int j = j0 + r;
      const double d = readlane_d(qj ? rows[r][CPL - 1] : rows[r][0], j % kWave);
      const bool live = j < n;
      if (live && !(d > 0.0) && fail == 0) fail = j + 1;
      const double dinv = 1.0 / d;
      if (l == 0) dinvb[buf][r] = live ? dinv : 0.0;
#pragma unroll
      for (int r2 = r + 1; r2 < BR; ++r2) {
        const double coef = readlane_d(qj ? rows[r][CPL - 1] : rows[r][0], (j0 + r2) % kWave) * dinv;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          const int c = l + kWave * q;
          const double upd = __builtin_fma(-coef, rows[r][q], rows[r2][q]);
          rows[r2][q] = (live && c >= j0 + r2) ? upd : rows[r2][q];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = l + kWave * q;
        if (c < NP && j0 + r < NP) Rl[(j0 + r) * NP + c] = (c >= j0 + r) ? rows[r][q] : 0.0;
      }
    if (l == 0) failb[buf] = fail;
  };
  // Rank-BR update of the thread's row block kb by row block J (rows below the block only).
  auto update = [&](int kb, int j0, const double (&gj)[BR][CPL], const double (&di)[BR]) {
#pragma unroll
    for (int r2 = 0; r2 < BR; ++r2) {
      const int i = BR * (w + NWV * kb) + r2;
      double lij[BR];
#pragma unroll
      for (int r = 0; r < BR; ++r) lij[r] = Rl[(j0 + r) * NP + i] * di[r];
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = l + kWave * q;
        double upd = g[kb][r2][q];
#pragma unroll
        for (int r = 0; r < BR; ++r) upd = __builtin_fma(-lij[r], gj[r][q], upd);
        g[kb][r2][q] = (i >= j0 + BR && i <= c) ? upd : g[kb][r2][q];
      }
    }
  };
  if (nblk > 0 && w == 0) eliminate(0);
  for (int J = 0; J < nblk; ++J) {
    const int buf = J & 1;
    const int j0 = BR * J;
    __syncthreads();  // block J published; every read of block J - 1 is done
    const int f = failb[buf];
    if (f) {  // every thread read the same flag
      bad = f;
      break;
    }
    double gj[BR][CPL], di[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      di[r] = dinvb[buf][r];
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = l + kWave * q;
        gj[r][q] = (c < NP) ? Rl[(j0 + r) * NP + (c < NP ? c : 0)] : 0.0;
      }
    }
    const int nx = J + 1;
    if (nx < nblk && w == nx % NWV) {
      // look-ahead: the owner of block J + 1 brings that block up to date and publishes it first
      // (the only work on the path to the next barrier), at raised priority
      const int nkb = nx / NWV;
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int kb = 0; kb < NBT; ++kb)
        if (kb == nkb) update(kb, j0, gj, di);
      eliminate(nx);
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int kb = 0; kb < NBT; ++kb)
        if (kb != nkb) update(kb, j0, gj, di);
    } else {
#pragma unroll
      for (int kb = 0; kb < NBT; ++kb) update(kb, j0, gj, di);
    }
  }
  if (bad) {
    if (t == 0) {
      info[0] = RCQR_E_CHOL;
      info[1] = bad;
    }
    return;
  }
  __syncthreads();
  // rows of R1 from the stored rows of the LDL^T factorization
  for (int r = t; r < n; r += blockDim.x) sdiag[r] = sqrt(Rl[r * NP + r]);
  __syncthreads();
  for (int idx = t; idx < n * NP; idx += blockDim.x) {
    const int r = idx / NP, c = idx % NP;
    const double sr = sdiag[r];
    Rl[idx] = (c == r) ? sr : ((c > r && c < n) ? Rl[idx] / sr : 0.0);
  }
  __syncthreads();
  // R1, its packed padded form, and R = R1 Rprev: R[i][k] = sum_{m = i..k} R1[i][m] Rprev[m][k]
  for (int idx = t; idx < NP * NP; idx += blockDim.x) {
    const int r = idx / NP, c = idx % NP;
    const double v = (r < n && c < n && c >= r) ? Rl[r * NP + c] : 0.0;
    if (r < n && c < n) r1[r * n + c] = v;
    if (c >= r) put_packed(r1pk, NP, n, r, c, v);
  }
  if constexpr (NP <= 64) {
    // Rprev staged in LDS (one coalesced read), then the same sums in the same order
    for (int idx = t; idx < n * n; idx += blockDim.x) rp[idx] = rprev[idx];
    __syncthreads();
  }
  const double* rpv = NP <= 64 ? rp : rprev;
  // R = R1 Rprev (Algorithm 3, step 3) on the matrix cores: each wave takes 16 x 16 output blocks
  // (a, b); an upper block sums only the K-steps where both triangles are nonzero (rows 16a to
  // 16b + 15 of Rprev), a lower block is zero.  Operand lanes as in the streaming passes:
  // A[l % 16][l / 16], B[l / 16][l % 16], result element e of lane l at row l / 16 + 4e, column l % 16.
  {
    typedef double d4 __attribute__((ext_vector_type(4)));
    const int li = l & 15, lq = l >> 4;
    const int nbn = (n + 15) / 16;
    for (int blk = w; blk < nbn * nbn; blk += NWV) {
      const int a = blk / nbn, b = blk % nbn;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
      if (a <= b) {
        const int ra = 16 * a + li, cb = 16 * b + li;
        for (int ks = 4 * a; ks < 4 * b + 4; ++ks) {
          const int kk = 4 * ks + lq;
          const double av = (ra < n && kk < n) ? Rl[ra * NP + kk] : 0.0;
          const double bv = (kk < n && cb < n) ? rpv[kk * n + cb] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * a + lq + 4 * e, c = 16 * b + li;
        if (r < n && c < n) r_out[(int64_t)r * ldr + c] = (c >= r) ? acc[e] : 0.0;
      }
    }
  }
}

// Dynamic LDS: the NP x NP rows of the elimination, and up to 64 padded columns a second NP x NP
// area that stages Rprev for the final product.
template <int NP>
constexpr size_t cholesky_lds() {
  return (size_t)NP * NP * sizeof(double) * (NP <= 64 ? 2 : 1);
}

template <int NP>
static hipError_t cholesky_prepare() {
  constexpr size_t lds = cholesky_lds<NP>();
  if constexpr (lds > 32 * 1024) {
    static bool attr_set = false;  // 64 KiB (64 columns) and 128 KiB (128 columns) of dynamic LDS
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute((const void*)cholesky_kernel<NP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
  }
  return hipSuccess;
}

hipError_t prepare_cholesky(int np) {
  return np == 128 ? cholesky_prepare<128>() : np == 64 ? cholesky_prepare<64>() : hipSuccess;
}

template <int NP>
static hipError_t cholesky_any(const double* gcompact, int n, const double* rprev, double shift_coef, int32_t* info, double* g_out,
                               double* r1, double* r1pk, double* r_out, int64_t ldr, hipStream_t s, const MemberStride& ms) {
  const hipError_t e = cholesky_prepare<NP>();
  if (e != hipSuccess) return e;
  if (ms.count < 1) return hipErrorInvalidValue;
  const size_t lds = cholesky_lds<NP>();
  hipLaunchKernelGGL(cholesky_kernel<NP>, dim3(1, ms.count), dim3(CholShape<NP>::NWV * kWave), lds, s, gcompact, n, rprev, shift_coef,
                     info, g_out, r1, r1pk, r_out, ldr, ms);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* gcompact, int n, int np, const double* rprev, double shift_coef, int32_t* info,
                           double* g_out, double* r1, double* r1pk, double* r_out, int64_t ldr, hipStream_t s, const MemberStride& ms) {
  switch (np) {
    case 16: return cholesky_any<16>(gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr, s, ms);
    case 32: return cholesky_any<32>(gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr, s, ms);
    case 64: return cholesky_any<64>(gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr, s, ms);
    case 128: return cholesky_any<128>(gcompact, n, rprev, shift_coef, info, g_out, r1, r1pk, r_out, ldr, s, ms);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rcqr
