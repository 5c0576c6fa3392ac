// The two streaming passes over V.
//
//  trsm_gram_kernel  Q0 = V R0^{-1} (Algorithm 1, step 3) fused with the Gram matrix
//                    G = Q0^T Q0 (Algorithm 2, step 1 applied to Q0).  One lane owns one row of
//                    V and solves x R0 = v by forward substitution (Section 5.2 analyses this
//                    row by row; an explicit inverse of R0 is not used).  The wave's 64 solved
//                    rows are transposed through LDS into FP64 MFMA operands and
//                    G += X^T X is accumulated with v_mfma_f64_16x16x4f64 on the upper 16x16
//                    blocks.  Each workgroup sums its waves in fixed order and writes one
//                    partial; the workgroup count is fixed, so the summation order is too.
//  final_mfma_kernel Q = Q0 R1^{-1} (Algorithm 2, step 3 on Q0): recomputes the same Q0 row with
//                    the same device function (bitwise identical to the Gram pass: explicit
//                    FMAs, no implicit contraction) and applies R1^{-1} on the matrix cores.
//  final_kernel      Q0 = V R0^{-1} alone (one substitution), for the paths that need only that.
//
// Rows are padded to NP columns; the padded R has an identity block, so padded columns stay
// zero and contribute nothing.
#include "device_common.h"
#include "launch.h"

namespace rcqr {

typedef double d4 __attribute__((ext_vector_type(4)));

// Returns 0, but the compiler cannot see that, and cannot compute it before `after` is
// ready: a load at p + opaque_zero(after) is issued after the arithmetic that produced
// `after` (no hoisting of the coefficient loads ahead of the work that precedes them), while p
// keeps its address space and read-only provenance, so the load is still a scalar load.
__device__ __forceinline__ int opaque_zero(double after) {
  int z = 0;
  asm volatile("" : "+s"(z) : "v"(after));
  return z;
}

// x R = v for one row, R upper triangular and padded to NP columns, stored packed row by row
// with the reciprocal of each diagonal entry in place of the entry:
//   Rpk = [1/R00, R01, ..., R0,NP-1, 1/R11, R12, ..., 1/R(NP-1)(NP-1)].
// Column-oriented forward substitution: x_k = v_k * (1/R_kk), then v_j -= x_k R_kj (j > k),
// k ascending.  The coefficients are uniform across the wave and are streamed into scalar
// registers eight at a time, PD chunks ahead of use; a scheduling barrier per chunk keeps
// the compiler from hoisting all of them at once.  PD changes only the load schedule, never
// the arithmetic, so every caller gets bitwise the same x.
template <int NP, int PD = 4>
__device__ __forceinline__ void rowsolve(double (&x)[NP], const double* __restrict__ Rpk) {
  constexpr int NV = NP * (NP + 1) / 2;
  constexpr int NCH = (NV + 7) / 8;
  double buf[PD + 1][8];
#pragma unroll
  for (int ch = 0; ch < PD; ++ch) {
    if (ch < NCH) {
#pragma unroll
      for (int e = 0; e < 8; ++e) buf[ch][e] = (8 * ch + e < NV) ? Rpk[8 * ch + e] : 0.0;
    }
  }
  int v = 0;
  double last = x[0];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
#pragma unroll
    for (int j = k; j < NP; ++j) {
      if ((v & 7) == 0) {
        __builtin_amdgcn_sched_barrier(0);
        const int nxt = (v >> 3) + PD;
        if (nxt < NCH) {
          const double* src = Rpk + opaque_zero(last);
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

int packed_len(int np) { return np * (np + 1) / 2; }

// FULL: n == NP and rows are 16-byte aligned (V, Q aligned, even leading dimensions), so a row
// moves as NP/2 unguarded 16-byte accesses.  Otherwise every column is guarded by c < n.
template <int NP, bool FULL>
__device__ __forceinline__ void load_row(double (&x)[NP], const double* __restrict__ V, int64_t row, int64_t m, int n,
                                         int64_t ldv) {
  const double* src = V + row * ldv;
  if (row >= m) {
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = 0.0;
    return;
  }
  if constexpr (FULL) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int c = 0; c < NP / 2; ++c) {
      const double2 v = s2[c];
      x[2 * c] = v.x;
      x[2 * c + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = c < n ? src[c] : 0.0;
  }
}

template <int NP, bool FULL>
__device__ __forceinline__ void store_row(const double (&x)[NP], double* __restrict__ Q, int64_t row, int n, int64_t ldq) {
  double* dst = Q + row * ldq;
  if constexpr (FULL) {
    double2* d2 = reinterpret_cast<double2*>(dst);
#pragma unroll
    for (int c = 0; c < NP / 2; ++c) d2[c] = double2{x[2 * c], x[2 * c + 1]};
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c)
      if (c < n) dst[c] = x[c];
  }
}

int gram_compact_len(int np) {
  const int nb = np / 16;
  return nb * (nb + 1) / 2 * 256;
}

template <int NP, bool FULL, bool STORE, bool BATCH>
__global__ __launch_bounds__(kGramThreads, 1) void trsm_gram_kernel(const double* __restrict__ V, int64_t m, int n, int64_t ldv,
                                                                    const double* __restrict__ R0pk,
                                                                    const int32_t* __restrict__ info, double* __restrict__ gpart,
                                                                    double* __restrict__ q0, int64_t ldq, MemberStride ms) {
  constexpr int NB = NP / 16;
  constexpr int NBU = NB * (NB + 1) / 2;
  constexpr int NW = kGramThreads / kWave;
  int64_t nblk = gridDim.x;  // workgroups of this member
  if constexpr (BATCH) {
    // batch member: workspace pointers move by whole doubles / ints (the workspace stride is a
    // multiple of 256 bytes), keeping them typed so the factor still streams through scalar loads
    const int64_t mb = blockIdx.y, off = mb * ms.ws;
    member_v(ms, mb, V, m, ldv);
    R0pk += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    gpart += off / (int64_t)sizeof(double);
    if (ms.info != nullptr) {  // ragged batch: the member's own Gram grid and Q
      const MemberInfo& mi = member_info(ms, mb);
      nblk = mi.gblocks;
      if (q0 != nullptr) {
        q0 = mi.Q;
        ldq = mi.ldq;
      }
    } else if (q0 != nullptr) {
      q0 += mb * ms.q;
    }
    if ((int64_t)blockIdx.x >= nblk) return;
  }
  __shared__ double xs[NW][16][kWave + 1];
  __shared__ double gl[NBU * 256];
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  d4 acc[NBU];
#pragma unroll
  for (int i = 0; i < NBU; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t ntiles = (m + kWave - 1) / kWave;
  for (int64_t t = (int64_t)blockIdx.x * NW + wave; t < ntiles; t += nblk * NW) {
    const int64_t row = t * kWave + lane;
    double x[NP];
    load_row<NP, FULL>(x, V, row, m, n, ldv);
    rowsolve<NP>(x, R0pk);
    // when Q0 is stored, each lane writes its solved row from registers (the lines of a row are
    // completed by consecutive stores and merge in L2; no extra registers for a staged copy)
    if constexpr (STORE) {
      if (row < m) store_row<NP, FULL>(x, q0, row, n, ldq);
    }
    // transpose 16-column blocks through LDS into MFMA operands:
    // F[a][s] (lane l) = X[4s + l/16][16a + l%16]
    double F[NB][16];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
#pragma unroll
      for (int c = 0; c < 16; ++c) xs[wave][c][lane] = x[16 * a + c];
      wave_lds_sync();
#pragma unroll
      for (int s = 0; s < 16; ++s) F[a][s] = xs[wave][lane & 15][4 * s + (lane >> 4)];
      wave_lds_sync();
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int ab = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = a; b < NB; ++b) {
          acc[ab] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[a][s], F[b][s], acc[ab], 0, 0, 0);
          ++ab;
        }
      }
    }
  }
  // fixed-order sum of the waves' blocks; MFMA output element e of lane l is D[l/16 + 4e][l%16]
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ab = 0; ab < NBU; ++ab) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = ab * 256 + ((lane >> 4) + 4 * e) * 16 + (lane & 15);
          gl[idx] = (w == 0) ? acc[ab][e] : gl[idx] + acc[ab][e];
        }
      }
    }
    __syncthreads();
  }
  double* out = gpart + (int64_t)blockIdx.x * (NBU * 256);
  for (int i = threadIdx.x; i < NBU * 256; i += kGramThreads) out[i] = gl[i];
}

// Persistent and phase-aligned: workgroup b takes tiles b*NW + w + k*gridDim.x*NW; in every
// round all its waves solve with R0, meet at a barrier, then solve with R1.  The two packed
// factors (16.6 KB each at 64 columns) do not fit the scalar data cache together, so keeping
// the waves of a CU on the same factor at the same time keeps the coefficient stream hitting.
// Batch member (BATCH): factor pointers move by the workspace stride; the input rows are the
// member's V, or (src_q) its Q holding a stored Q0; the output is the member's Q.
template <bool BATCH, class PI, class PO>
__device__ __forceinline__ void member_rows(const MemberStride& ms, int src_q, PI& in, int64_t& m, int64_t& ldin, PO& out, int64_t& ldout) {
  if constexpr (BATCH) {
    const int64_t mb = blockIdx.y;
    if (ms.info != nullptr) {
      const MemberInfo& mi = member_info(ms, mb);
      m = mi.m;
      out = mi.Q;
      ldout = mi.ldq;
      in = src_q ? mi.Q : mi.V;
      ldin = src_q ? mi.ldq : mi.ldv;
    } else {
      out += mb * ms.q;
      in += mb * (src_q ? ms.q : ms.v);
    }
  }
}

template <int NP, bool APPLY_R1, bool FULL, int NW, bool BATCH = false>
__global__ __launch_bounds__(NW * kWave) void final_kernel(const double* __restrict__ V, int64_t m, int n, int64_t ldv,
                                                          const double* __restrict__ R0pk, const double* __restrict__ R1pk,
                                                          const int32_t* __restrict__ info, double* __restrict__ Q, int64_t ldq,
                                                          MemberStride ms, int src_q) {
  if constexpr (BATCH) {
    const int64_t off = (int64_t)blockIdx.y * ms.ws;
    R0pk += off / (int64_t)sizeof(double);
    R1pk += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    member_rows<BATCH>(ms, src_q, V, m, ldv, Q, ldq);
  }
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t ntiles = (m + kWave - 1) / kWave;
  const int64_t per_round = (int64_t)gridDim.x * NW;
  const int64_t rounds = (ntiles + per_round - 1) / per_round;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t row = (r * per_round + (int64_t)blockIdx.x * NW + wave) * kWave + lane;
    double x[NP];
    load_row<NP, FULL>(x, V, row, m, n, ldv);
    rowsolve<NP>(x, R0pk);
    if constexpr (APPLY_R1) {
      __syncthreads();
      rowsolve<NP>(x, R1pk);
    }
    if (row < m) store_row<NP, FULL>(x, Q, row, n, ldq);
    if constexpr (APPLY_R1) __syncthreads();
  }
}

// Row i of R^{-1} in lane i (x R = e_i by the row substitution), stored as the upper 16 x 16
// blocks of R^{-1} (row-major blocks, upper_blk order) in rib.  One wave.
template <int NP>
__device__ __forceinline__ void build_rinv_blocks(const double* __restrict__ Rpk, double* rib, int lane) {
  constexpr int NB = NP / 16;
  double x[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) x[c] = (c == lane) ? 1.0 : 0.0;
  rowsolve<NP>(x, Rpk);
  if (lane < NP) {
    const int a = lane / 16;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      if (cb >= a) {
#pragma unroll
        for (int j = 0; j < 16; ++j) rib[upper_blk(a, cb, NB) * 256 + (lane & 15) * 16 + j] = x[16 * cb + j];
      }
    }
  }
}

// Q = (V R0^{-1}) R1^{-1} with the second step on the matrix cores.  R1 is the Cholesky factor
// of the Gram matrix of Q0, whose condition number is that of Q0, O(1) (Section 4's remark on
// kappa of randQR's Q); its inverse is formed accurately and applied as a product, while the
// solve with the ill-conditioned R0 stays a row-wise substitution (Section 5.2).
//   * wave 0 of each workgroup forms row i of R1^{-1} in lane i by the same substitution
//     (x R1 = e_i) and stores its upper 16x16 blocks in LDS;
//   * per tile of 64 rows: x = v R0^{-1} (lane = row), then 16 rows at a time go through LDS
//     into MFMA operands, Q[16 rows] = X[16 rows] R1^{-1} on v_mfma_f64_16x16x4f64
//     (upper blocks only), written straight from the accumulators.
// Only R0 streams through the scalar data cache (R0 and R1 together would not fit it).
template <int NP, bool FULL, int NW, bool BATCH>
__global__ __launch_bounds__(NW * kWave) void final_mfma_kernel(const double* __restrict__ V, int64_t m, int n, int64_t ldv,
                                                               const double* __restrict__ R0pk, const double* __restrict__ R1pk,
                                                               const int32_t* __restrict__ info, double* __restrict__ Q,
                                                               int64_t ldq, MemberStride ms) {
  constexpr int NB = NP / 16;
  constexpr int NBU = NB * (NB + 1) / 2;
  if constexpr (BATCH) {
    const int64_t mb = blockIdx.y, off = mb * ms.ws;  // batch member (typed offsets, as above)
    member_v(ms, mb, V, m, ldv);
    R0pk += off / (int64_t)sizeof(double);
    R1pk += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    if (ms.info != nullptr) {
      const MemberInfo& mi = member_info(ms, mb);
      Q = mi.Q;
      ldq = mi.ldq;
    } else {
      Q += mb * ms.q;
    }
  }
  __shared__ double rib[NBU * 256];
  __shared__ double st[NW][16][NP + 1];
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int li = lane & 15, lq = lane >> 4;
  if (wave == 0) build_rinv_blocks<NP>(R1pk, rib, lane);
  __syncthreads();
  double (*s)[NP + 1] = st[wave];
  const int64_t ntiles = (m + kWave - 1) / kWave;
  for (int64_t t = (int64_t)blockIdx.x * NW + wave; t < ntiles; t += (int64_t)gridDim.x * NW) {
    const int64_t row = t * kWave + lane;
    double x[NP];
    load_row<NP, FULL>(x, V, row, m, n, ldv);
    rowsolve<NP>(x, R0pk);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (lq == rb) {
#pragma unroll
        for (int c = 0; c < NP; ++c) s[li][c] = x[c];
      }
      wave_lds_sync();
      d4 acc[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < NP / 4; ++k) {
        const double a = s[li][4 * k + lq];
#pragma unroll
        for (int cb = k / 4; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rib[upper_blk(k / 4, cb, NB) * 256 + (4 * (k % 4) + lq) * 16 + li],
                                                         acc[cb], 0, 0, 0);
      }
      wave_lds_sync();
      // accumulator element e of lane l holds row l/16 + 4e, column l%16 of the 16 x 16 block
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int col = 16 * cb + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t r = t * kWave + 16 * rb + lq + 4 * e;
          if (r < m && (FULL || col < n)) Q[r * ldq + col] = acc[cb][e];
        }
      }
    }
  }
}

// 65..128 columns: a row does not fit a lane's registers next to the solve's working set, so
// x R = v runs as a 2 x 2 block substitution over 64-column halves (Section 5.2's row-wise
// substitution on the diagonal blocks, a product for the coupling block):
//     x_lo = v_lo R00^{-1}                  written to the output row: in the Gram phase by the
//                                           64-column Gram pass, which also forms the Gram blocks
//                                           of columns 0..63; elsewhere by final_kernel<64>
//     x_hi = (v_hi - x_lo R01) R11^{-1}     solve_hi_kernel
// The factor is in the blocked packed format [R00 packed | R01 dense row-major | R11 packed]
// (2080 + 4096 + 2080 doubles).  In solve_hi_kernel the coupling product runs on the matrix
// cores: R01 sits in LDS, x_lo is read back from the output rows as MFMA operands (16 rows x 4
// columns per K-step), and each 16-row block of x_lo R01 goes through LDS to the lanes that own
// those rows.  Only R11 streams through the scalar data cache.
template <bool FULL, int NW, bool BATCH = false>
__global__ __launch_bounds__(NW * kWave) void solve_hi_kernel(const double* in, int64_t m, int n, int64_t ldin,
                                                             const double* __restrict__ Rbk, const int32_t* __restrict__ info,
                                                             double* out, int64_t ldout, MemberStride ms, int src_q) {
  constexpr int H = 64, PK = H * (H + 1) / 2;
  __shared__ double r01[H][H + 1];
  __shared__ double ust[NW][16][H + 1];
  if constexpr (BATCH) {
    const int64_t off = (int64_t)blockIdx.y * ms.ws;
    Rbk += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    member_rows<BATCH>(ms, src_q, in, m, ldin, out, ldout);
  }
  if (info[0] != 0) return;
  for (int i = threadIdx.x; i < H * H; i += NW * kWave) r01[i / H][i % H] = Rbk[PK + i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int li = lane & 15, lq = lane >> 4;
  const int nh = n - H;
  double (*u)[H + 1] = ust[wave];
  const int64_t ntiles = (m + kWave - 1) / kWave;
  for (int64_t t = (int64_t)blockIdx.x * NW + wave; t < ntiles; t += (int64_t)gridDim.x * NW) {
    const int64_t row = t * kWave + lane;
    double x[H];
    if (row < m) {
      const double* src = in + row * ldin + H;
      if constexpr (FULL) {
        const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
        for (int c = 0; c < H / 2; ++c) {
          const double2 v = s2[c];
          x[2 * c] = v.x;
          x[2 * c + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int c = 0; c < H; ++c) x[c] = c < nh ? src[c] : 0.0;
      }
    } else {
#pragma unroll
      for (int c = 0; c < H; ++c) x[c] = 0.0;
    }
    // x_lo operands in halves of eight K-steps, two halves in flight: while one half of a 16-row
    // block is multiplied, the same half of the next 16-row block is loaded
    auto load_half = [&](int rb, int h, double (&a)[8]) {
      const int64_t arow = t * kWave + 16 * rb + li;
      const double* xl = out + arow * ldout;
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = arow < m ? xl[4 * (8 * h + k) + lq] : 0.0;
    };
    double ring[2][8];
    load_half(0, 0, ring[0]);
    load_half(0, 1, ring[1]);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      d4 acc[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int ks = 8 * h + k;
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ring[h][k], r01[4 * ks + lq][16 * cb + li], acc[cb], 0, 0, 0);
        }
        if (rb + 1 < 4) load_half(rb + 1, h, ring[h]);
      }
      // element e of lane l: row 16 rb + l/16 + 4e, column 16 cb + l%16 of x_lo R01
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) u[lq + 4 * e][16 * cb + li] = acc[cb][e];
      wave_lds_sync();
      if (lq == rb) {
#pragma unroll
        for (int c = 0; c < H; ++c) x[c] -= u[li][c];
      }
      wave_lds_sync();
    }
    rowsolve<H>(x, Rbk + PK + H * H);
    if (row < m) {
      double* dst = out + row * ldout + H;
      if constexpr (FULL) {
        double2* d2 = reinterpret_cast<double2*>(dst);
#pragma unroll
        for (int c = 0; c < H / 2; ++c) d2[c] = double2{x[2 * c], x[2 * c + 1]};
      } else {
#pragma unroll
        for (int c = 0; c < H; ++c)
          if (c < nh) dst[c] = x[c];
      }
    }
  }
}

// Q = Q0 R1^{-1} in place for a stored Q0 (the materialising alternative to final_mfma_kernel,
// chosen by the tuner): the MFMA operands are read straight from the Q0 rows (16 rows x 4
// columns per K-step), the same products in the same order as final_mfma_kernel, so Q is bitwise
// the same.  Each 16-row block is read completely before it is overwritten.
template <int NP, bool FULL, int NW>
__global__ __launch_bounds__(NW * kWave) void apply_rinv_kernel(double* Q, int64_t m, int n, int64_t ldq,
                                                               const double* __restrict__ R1pk, const int32_t* __restrict__ info) {
  constexpr int NB = NP / 16;
  constexpr int NBU = NB * (NB + 1) / 2;
  __shared__ double rib[NBU * 256];
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int li = lane & 15, lq = lane >> 4;
  if (wave == 0) build_rinv_blocks<NP>(R1pk, rib, lane);
  __syncthreads();
  const int64_t nblk16 = (m + 15) / 16;
  for (int64_t b16 = (int64_t)blockIdx.x * NW + wave; b16 < nblk16; b16 += (int64_t)gridDim.x * NW) {
    const int64_t arow = b16 * 16 + li;
    // operands one 16-column block (four K-steps) at a time, the next block's loads in flight
    auto load_blk = [&](int kb, double (&a)[4]) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int col = 16 * kb + 4 * kk + lq;
        a[kk] = (arow < m && (FULL || col < n)) ? Q[arow * ldq + col] : 0.0;
      }
    };
    double a[2][4];
    load_blk(0, a[0]);
    d4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      __builtin_amdgcn_sched_barrier(0);  // keep the operand reads of one block together
      if (kb + 1 < NB) load_blk(kb + 1, a[(kb + 1) & 1]);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
        for (int cb = kb; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kb & 1][kk], rib[upper_blk(kb, cb, NB) * 256 + (4 * kk + lq) * 16 + li],
                                                         acc[cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = b16 * 16 + lq + 4 * e;
        if (r < m && (FULL || col < n)) Q[r * ldq + col] = acc[cb][e];
      }
    }
  }
}

// 65..128 columns, Algorithm 2 step 3: R1^{-1} formed once per factorization (R1 = chol(G) has the
// condition number of Q0, O(1); Section 4's remark on the conditioning of randQR's Q), then
// Q = Q0 R1^{-1} as one product on the matrix cores over the stored Q0 (apply_rinv128_kernel).
// Row i of R^{-1} solves x R = e_i by block substitution over the blocked factor
// [R00 | R01; 0 | R11]: x_lo = e_i R00^{-1} (zero below row 64), x_hi = (e_i,hi - x_lo R01) R11^{-1};
// lane i of wave 0 takes rows 0..63, lane i of wave 1 rows 64..127 (x_lo = 0, so x_hi = e_i R11^{-1}
// at once, while wave 0 solves with R00).  The coupling product x_lo R01 (64 x 64 x 64) runs on the
// matrix cores, one 16-row block per wave, with x_lo and R01 staged in LDS.  The upper 16 x 16
// blocks of R^{-1} (36 of them, row-major blocks in upper_blk order) go to rinv.
constexpr int kRinvWaves = 4;
__global__ __launch_bounds__(kRinvWaves * kWave) void rinv128_kernel(const double* __restrict__ Rbk, const int32_t* __restrict__ info,
                                                                    double* __restrict__ rinv, MemberStride ms) {
  constexpr int H = 64, PK = H * (H + 1) / 2, NB = 8;
  __shared__ double r01[H][H + 1];
  __shared__ double xs[H][H + 1];  // x_lo of rows 0..63, then x_lo R01
  {
    const int64_t off = (int64_t)blockIdx.y * ms.ws;  // batch member
    Rbk += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    rinv += off / (int64_t)sizeof(double);
  }
  if (info[0] != 0) return;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int li = lane & 15, lq = lane >> 4;
  for (int i = threadIdx.x; i < H * H; i += kRinvWaves * kWave) r01[i / H][i % H] = Rbk[PK + i];
  const int row = wave * H + lane;
  double lo[H], hi[H];
  if (wave < 2) {
#pragma unroll
    for (int c = 0; c < H; ++c) {
      lo[c] = (wave == 0 && c == lane) ? 1.0 : 0.0;
      hi[c] = (wave == 1 && c == lane) ? 1.0 : 0.0;
    }
    if (wave == 0) {
      rowsolve<H>(lo, Rbk);
#pragma unroll
      for (int c = 0; c < H; ++c) xs[lane][c] = lo[c];
    } else {
      rowsolve<H>(hi, Rbk + PK + H * H);
    }
  }
  __syncthreads();
  // x_lo R01, rows 16 w .. 16 w + 15 by wave w; element e of lane l: row 16 w + l/16 + 4e,
  // column 16 cb + l%16
  d4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < H / 4; ++ks) {
    const double a = xs[16 * wave + li][4 * ks + lq];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, r01[4 * ks + lq][16 * cb + li], acc[cb], 0, 0, 0);
  }
  __syncthreads();  // every wave has read its x_lo operands
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) xs[16 * wave + lq + 4 * e][16 * cb + li] = acc[cb][e];
  __syncthreads();
  if (wave >= 2) return;
  if (wave == 0) {
#pragma unroll
    for (int c = 0; c < H; ++c) hi[c] = -xs[lane][c];
    rowsolve<H>(hi, Rbk + PK + H * H);
  }
  const int a = row / 16;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    if (cb >= a) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int col = 16 * cb + j;
        rinv[upper_blk(a, cb, NB) * 256 + (row & 15) * 16 + j] = col < H ? lo[col] : hi[col - H];
      }
    }
  }
}

// Q = Q0 R1^{-1} in place, 65..128 columns (rows padded to 128): the upper blocks of R1^{-1} in LDS,
// the MFMA operands read straight from the stored Q0 rows (16 rows x 4 columns per K-step); each
// 16-row block is read completely before it is overwritten.
template <bool FULL, int NW, bool BATCH>
__global__ __launch_bounds__(NW * kWave) void apply_rinv128_kernel(double* Q, int64_t m, int n, int64_t ldq,
                                                                  const double* __restrict__ rinv, const int32_t* __restrict__ info,
                                                                  MemberStride ms) {
  constexpr int NP = 128, NB = 8, NBU = NB * (NB + 1) / 2;
  __shared__ double rib[NBU * 256];
  if constexpr (BATCH) {
    const int64_t mb = blockIdx.y, off = mb * ms.ws;
    rinv += off / (int64_t)sizeof(double);
    info += off / (int64_t)sizeof(int32_t);
    if (ms.info != nullptr) {
      const MemberInfo& mi = member_info(ms, mb);
      Q = mi.Q;
      ldq = mi.ldq;
      m = mi.m;
    } else {
      Q += mb * ms.q;
    }
  }
  if (info[0] != 0) return;
  for (int i = threadIdx.x; i < NBU * 256; i += NW * kWave) rib[i] = rinv[i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int li = lane & 15, lq = lane >> 4;
  const int64_t nblk16 = (m + 15) / 16;
  const int64_t tstride = (int64_t)gridDim.x * NW;
  // operands one 16-column block (four K-steps) at a time, four blocks ahead in a ring (into the
  // wave's next 16-row block near the end of one); a block's rows are all read before its
  // results are stored, and the next block's rows are other rows
  auto load_blk = [&](int64_t t, int kb, double (&a)[4]) {
    const int64_t arow = t * 16 + li;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int col = 16 * kb + 4 * kk + lq;
      a[kk] = (t < nblk16 && arow < m && (FULL || col < n)) ? Q[arow * ldq + col] : 0.0;
    }
  };
  int64_t b16 = (int64_t)blockIdx.x * NW + wave;
  double ring[4][4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) load_blk(b16, kb, ring[kb]);
  for (; b16 < nblk16; b16 += tstride) {
    d4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      double a[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) a[kk] = ring[kb % 4][kk];
      __builtin_amdgcn_sched_barrier(0);  // keep the operand reads of one block together
      if (kb + 4 < NB)
        load_blk(b16, kb + 4, ring[kb % 4]);
      else
        load_blk(b16 + tstride, kb + 4 - NB, ring[kb % 4]);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
        for (int cb = kb; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], rib[upper_blk(kb, cb, NB) * 256 + (4 * kk + lq) * 16 + li], acc[cb], 0,
                                                         0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = b16 * 16 + lq + 4 * e;
        if (r < m && (FULL || col < n)) Q[r * ldq + col] = acc[cb][e];
      }
    }
  }
}

static int final_grid();

hipError_t launch_rinv128(const double* rbk, const int32_t* info, double* rinv, hipStream_t s, const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rinv128_kernel, dim3(1, ms.count), dim3(kRinvWaves * kWave), 0, s, rbk, info, rinv, ms);
  return hipGetLastError();
}

hipError_t launch_apply_rinv128(double* Q, int64_t m, int n, int64_t ldq, const double* rinv, const int32_t* info, int grid_mult,
                                hipStream_t s, const MemberStride& ms) {
  if (m <= 0) return hipSuccess;
  if (n <= 64 || n > 128 || ms.count < 1) return hipErrorInvalidValue;
  constexpr int NW = 8;
  const int64_t blocks = (m + 15) / 16;
  int64_t g = (blocks + NW - 1) / NW;
  if (g > (int64_t)grid_mult * final_grid()) g = (int64_t)grid_mult * final_grid();
  const dim3 grid((unsigned)g, ms.count), block(NW * kWave);
  const bool batch = ms.count > 1 || ms.info != nullptr;
  const bool full = n == 128;
#define RCQR_AR128(F, B) hipLaunchKernelGGL((apply_rinv128_kernel<F, NW, B>), grid, block, 0, s, Q, m, n, ldq, rinv, info, ms);
  if (batch) {
    if (full) { RCQR_AR128(true, true) } else { RCQR_AR128(false, true) }
  } else {
    if (full) { RCQR_AR128(true, false) } else { RCQR_AR128(false, false) }
  }
#undef RCQR_AR128
  return hipGetLastError();
}

static bool full_rows(int np, int n, const void* a, int64_t lda, const void* b, int64_t ldb) {
  const bool al = (reinterpret_cast<uintptr_t>(a) % 16 == 0) && (lda % 2 == 0);
  const bool bl = b == nullptr || ((reinterpret_cast<uintptr_t>(b) % 16 == 0) && (ldb % 2 == 0));
  return n == np && al && bl;
}

hipError_t launch_trsm_gram(int np, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk, const int32_t* info,
                            double* gpart, double* q0, int64_t ldq, hipStream_t s, const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  const dim3 grid(gram_blocks(m), ms.count), block(kGramThreads);
  const bool full = ms.info != nullptr ? (n == np && ms.aligned) : (full_rows(np, n, V, ldv, q0, ldq) && ms.v % 2 == 0 && ms.q % 2 == 0);
  const bool batch = ms.count > 1 || ms.info != nullptr;
#define RCQR_GRAM_B(NPV, B)                                                                                                       \
  if (full && q0)                                                                                                                 \
    hipLaunchKernelGGL((trsm_gram_kernel<NPV, true, true, B>), grid, block, 0, s, V, m, n, ldv, r0pk, info, gpart, q0, ldq, ms);   \
  else if (full)                                                                                                                  \
    hipLaunchKernelGGL((trsm_gram_kernel<NPV, true, false, B>), grid, block, 0, s, V, m, n, ldv, r0pk, info, gpart, q0, ldq, ms);  \
  else if (q0)                                                                                                                    \
    hipLaunchKernelGGL((trsm_gram_kernel<NPV, false, true, B>), grid, block, 0, s, V, m, n, ldv, r0pk, info, gpart, q0, ldq, ms);  \
  else                                                                                                                            \
    hipLaunchKernelGGL((trsm_gram_kernel<NPV, false, false, B>), grid, block, 0, s, V, m, n, ldv, r0pk, info, gpart, q0, ldq, ms);
#define RCQR_GRAM(NPV)       \
  if (batch) {               \
    RCQR_GRAM_B(NPV, true)   \
  } else {                   \
    RCQR_GRAM_B(NPV, false)  \
  }
  switch (np) {
    case 16: RCQR_GRAM(16) break;
    case 32: RCQR_GRAM(32) break;
    case 64: RCQR_GRAM(64) break;
    default: return hipErrorInvalidValue;
  }
#undef RCQR_GRAM
#undef RCQR_GRAM_B
  return hipGetLastError();
}

static int final_grid() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  return cus;
}

hipError_t prepare_stream_launches() {
  (void)final_grid();
  return hipSuccess;
}

hipError_t launch_final(int np, bool apply_r1, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk,
                        const double* r1pk, const int32_t* info, double* Q, int64_t ldq, hipStream_t s, int grid_mult,
                        const MemberStride& ms, int src_q) {
  if (m <= 0) return hipSuccess;
  if (ms.count < 1) return hipErrorInvalidValue;
  const bool full = ms.info != nullptr ? (n == np && ms.aligned)
                                       : (full_rows(np, n, V, ldv, Q, ldq) && ms.v % 2 == 0 && ms.q % 2 == 0);
  const bool batch = ms.count > 1 || ms.info != nullptr;
  const int64_t tiles = (m + kWave - 1) / kWave;
  if (apply_r1) {
    // eight waves per workgroup, about two workgroups per CU over the whole pass
    constexpr int NW = 8;
    int64_t g = (tiles + NW - 1) / NW;
    if (g > (int64_t)grid_mult * final_grid()) g = (int64_t)grid_mult * final_grid();
    const dim3 grid((unsigned)g, ms.count), block(NW * kWave);
#define RCQR_FINAL_MFMA_B(NPV, B)                                                                                               \
  if (full)                                                                                                                     \
    hipLaunchKernelGGL((final_mfma_kernel<NPV, true, NW, B>), grid, block, 0, s, V, m, n, ldv, r0pk, r1pk, info, Q, ldq, ms);  \
  else                                                                                                                          \
    hipLaunchKernelGGL((final_mfma_kernel<NPV, false, NW, B>), grid, block, 0, s, V, m, n, ldv, r0pk, r1pk, info, Q, ldq, ms);
#define RCQR_FINAL_MFMA(NPV)       \
  if (batch) {                     \
    RCQR_FINAL_MFMA_B(NPV, true)   \
  } else {                         \
    RCQR_FINAL_MFMA_B(NPV, false)  \
  }
    switch (np) {
      case 16: RCQR_FINAL_MFMA(16) break;
      case 32: RCQR_FINAL_MFMA(32) break;
      case 64: RCQR_FINAL_MFMA(64) break;
      default: return hipErrorInvalidValue;
    }
#undef RCQR_FINAL_MFMA
#undef RCQR_FINAL_MFMA_B
    return hipGetLastError();
  }
  // one factor: Q0 = V R0^{-1} only (persistent, one workgroup per CU)
#define RCQR_FINAL_B(NPV, NWV, B)                                                                                                \
  if (full)                                                                                                                     \
    hipLaunchKernelGGL((final_kernel<NPV, false, true, NWV, B>), grid, block, 0, s, V, m, n, ldv, r0pk, r1pk, info, Q, ldq, ms, src_q); \
  else                                                                                                                          \
    hipLaunchKernelGGL((final_kernel<NPV, false, false, NWV, B>), grid, block, 0, s, V, m, n, ldv, r0pk, r1pk, info, Q, ldq, ms, src_q);
#define RCQR_FINAL(NPV, NWV)                                                                                                    \
  {                                                                                                                             \
    int64_t g = (tiles + NWV - 1) / NWV;                                                                                        \
    if (g > final_grid()) g = final_grid();                                                                                     \
    const dim3 grid((unsigned)g, ms.count), block(NWV * kWave);                                                                 \
    if (batch) {                                                                                                                \
      RCQR_FINAL_B(NPV, NWV, true)                                                                                              \
    } else {                                                                                                                    \
      RCQR_FINAL_B(NPV, NWV, false)                                                                                             \
    }                                                                                                                           \
  }
  switch (np) {
    case 16: RCQR_FINAL(16, 16) break;
    case 32: RCQR_FINAL(32, 16) break;
    case 64: RCQR_FINAL(64, 12) break;
    default: return hipErrorInvalidValue;
  }
#undef RCQR_FINAL
#undef RCQR_FINAL_B
  return hipGetLastError();
}

hipError_t launch_apply_rinv(int np, double* Q, int64_t m, int n, int64_t ldq, const double* r1pk, const int32_t* info, int grid_mult,
                             hipStream_t s) {
  if (m <= 0) return hipSuccess;
  constexpr int NW = 8;
  const bool full = full_rows(np, n, Q, ldq, nullptr, 0);
  const int64_t blocks = (m + 15) / 16;
  int64_t g = (blocks + NW - 1) / NW;
  if (g > (int64_t)grid_mult * final_grid()) g = (int64_t)grid_mult * final_grid();
  const dim3 grid((unsigned)g), block(NW * kWave);
#define RCQR_APPLY(NPV)                                                                                             \
  if (full)                                                                                                         \
    hipLaunchKernelGGL((apply_rinv_kernel<NPV, true, NW>), grid, block, 0, s, Q, m, n, ldq, r1pk, info);          \
  else                                                                                                              \
    hipLaunchKernelGGL((apply_rinv_kernel<NPV, false, NW>), grid, block, 0, s, Q, m, n, ldq, r1pk, info);
  switch (np) {
    case 16: RCQR_APPLY(16) break;
    case 32: RCQR_APPLY(32) break;
    case 64: RCQR_APPLY(64) break;
    default: return hipErrorInvalidValue;
  }
#undef RCQR_APPLY
  return hipGetLastError();
}

// x_hi = (v_hi - x_lo R01) R11^{-1} for x_lo already in the output's first 64 columns.
static hipError_t launch_solve_hi(const double* in, int64_t m, int n, int64_t ldin, const double* rbk, const int32_t* info,
                                  double* out, int64_t ldout, hipStream_t s, int grid_mult, const MemberStride& ms, int src_q) {
  constexpr int NW = 8;
  const int64_t tiles = (m + kWave - 1) / kWave;
  int64_t g = (tiles + NW - 1) / NW;
  if (g > (int64_t)grid_mult * final_grid()) g = (int64_t)grid_mult * final_grid();
  const dim3 grid((unsigned)g, ms.count), block(NW * kWave);
  const bool batch = ms.count > 1 || ms.info != nullptr;
  const bool full = n == 128 && (ms.info != nullptr ? ms.aligned : (full_rows(64, 64, in, ldin, out, ldout) && ms.v % 2 == 0 && ms.q % 2 == 0));
#define RCQR_HI(F, B) \
  hipLaunchKernelGGL((solve_hi_kernel<F, NW, B>), grid, block, 0, s, in, m, n, ldin, rbk, info, out, ldout, ms, src_q);
  if (batch) {
    if (full) { RCQR_HI(true, true) } else { RCQR_HI(false, true) }
  } else {
    if (full) { RCQR_HI(true, false) } else { RCQR_HI(false, false) }
  }
#undef RCQR_HI
  return hipGetLastError();
}

hipError_t launch_solve128(const double* in, int64_t m, int n, int64_t ldin, const double* rbk, const int32_t* info, double* out,
                           int64_t ldout, hipStream_t s, int grid_mult, const MemberStride& ms, int src_q) {
  if (m <= 0) return hipSuccess;
  if (n <= 64 || n > 128 || ms.count < 1) return hipErrorInvalidValue;
  // x_lo = v_lo R00^{-1} into the output's first 64 columns (R00 packed leads the blocked format);
  // the 64-column view of 16-byte aligned rows with even leading dimensions is aligned too
  const hipError_t e = launch_final(64, false, in, m, 64, ldin, rbk, rbk, info, out, ldout, s, 2, ms, src_q);
  if (e != hipSuccess) return e;
  return launch_solve_hi(in, m, n, ldin, rbk, info, out, ldout, s, grid_mult, ms, src_q);
}

hipError_t launch_solve128_gram(const double* V, int64_t m, int n, int64_t ldv, const double* rbk, const int32_t* info, double* Q,
                                int64_t ldq, double* gplo, hipStream_t s, int grid_mult, const MemberStride& ms) {
  if (m <= 0) return hipSuccess;
  if (n <= 64 || n > 128 || ms.count < 1) return hipErrorInvalidValue;
  // x_lo by the 64-column Gram pass (R00 packed leads the blocked format), stored in Q's first 64
  // columns, with the Gram blocks of those columns into gplo
  const hipError_t e = launch_trsm_gram(64, V, m, 64, ldv, rbk, info, gplo, Q, ldq, s, ms);
  if (e != hipSuccess) return e;
  return launch_solve_hi(V, m, n, ldv, rbk, info, Q, ldq, s, grid_mult, ms, 0);
}

}  // namespace rcqr
