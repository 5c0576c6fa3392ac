// Host-callable launchers of the rcqr kernels (one per kernel family).  Every launcher only
// enqueues work on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcqr {

// Row-count-dependent partitions of the multi-workgroup passes.  Functions of the shape only (so
// the summation orders they fix do not depend on the device or on other members of a batch), and
// computed with the same integer arithmetic on the host and on the device.
//   bucket index: chunks of at least 4096 rows, at most 256, histogram matrix <= 2^26 entries
__host__ __device__ inline int bucket_nchunk(int64_t m, int64_t s1) {
  int64_t nch = (m + 4095) / 4096;
  if (nch > 256) nch = 256;
  const int64_t cap_ch = ((int64_t)1 << 26) / s1;
  if (nch > cap_ch) nch = cap_ch;
  return nch < 1 ? 1 : (int)nch;
}
__host__ __device__ inline int64_t bucket_chunk_rows(int64_t m, int nchunk) { return ((m + nchunk - 1) / nchunk + 3) / 4 * 4; }
//   small-s1 CountSketch (per-wave LDS copies of W1 of s1 x NPL, NPL = n padded to 8, 16, 32, 64):
//   one workgroup per 256-row chunk, at most 256 x (workgroups per CU at FP64)
constexpr int kCsLdsDoubles = 4096;  // s1 * NPL limit (4 waves x 32 KiB)
constexpr int kCsChunk = 256;        // rows hashed at once by one wave
__host__ __device__ inline int npl_of(int n) {
  int p = 8;
  while (p < n) p <<= 1;
  return p;
}
__host__ __device__ inline bool countsketch_lds_fits(int64_t s1, int n) { return n <= 64 && s1 * npl_of(n) <= kCsLdsDoubles; }
// per-wave capacity of the LDS copies: the smallest of 1024, 2048, 4096 elements holding s1 x NPL
// (smaller copies let 4, 2 or 1 workgroups share a CU)
__host__ __device__ inline int cs_cap(int64_t s1, int n) {
  const int64_t need = s1 * npl_of(n);
  return need <= 1024 ? 1024 : need <= 2048 ? 2048 : 4096;
}
__host__ __device__ inline int countsketch_lds_parts(int64_t m, int64_t s1, int n) {
  const int cap = cs_cap(s1, n);
  const int64_t target = 256 * (cap == 1024 ? 4 : cap == 2048 ? 2 : 1);
  int64_t p = (m + kCsChunk - 1) / kCsChunk;
  if (p > target) p = target;
  return p < 1 ? 1 : (int)p;
}
//   Gram pass (and Gram partials): one workgroup per eight 64-row tiles (one tile per wave), at
//   most kGramBlocks
constexpr int kGramBlocks = 256;     // most workgroups of the Gram pass (the count fixes the sum order)
constexpr int kGramThreads = 512;
__host__ __device__ inline int gram_blocks(int64_t m) {
  const int64_t per = kGramThreads;  // eight waves, one 64-row tile each
  const int64_t b = (m + per - 1) / per;
  return b < 1 ? 1 : (b > kGramBlocks ? kGramBlocks : (int)b);
}

// One member of a ragged batch as the kernels see it (written into the member's workspace slice
// by the batch's first kernel from the caller's rcqr_member_t): its own V, Q, R and row count,
// its sketch seed, and the row-count-dependent partitions above.
struct MemberInfo {
  const double* V;
  double* Q;
  double* R;
  int64_t m, ldv, ldq, ldr;
  uint64_t seed;
  int64_t chunk_rows;
  int32_t nchunk, cs_parts, gblocks, pad;
};

// A batch of factorizations in one set of launches: member b of a launch is a grid index
// (blockIdx.y, or blockIdx.z where y is taken); its workspace pointers move by b * ws bytes.
//   * same-shaped batch (info == nullptr): V, Q and R move by b * v, b * q, b * r elements, and
//     the sketch seed is seeds[b] (a device array) or, without one, the plan's seed + b;
//   * ragged batch (info != nullptr): members share n, s1 and s2 but not m; member b's V, Q, R,
//     leading dimensions, row count, seed and partitions are read from the MemberInfo at
//     info + b * ws bytes, and the grids are sized for the largest member (workgroups beyond a
//     member's own partition return at once).
// All zero, one member, for a single factorization (the kernels then compute exactly what they
// did alone).
struct MemberStride {
  int64_t ws = 0, v = 0, q = 0, r = 0;
  int32_t count = 1;
  const uint64_t* seeds = nullptr;
  const MemberInfo* info = nullptr;
  bool aligned = false;  // ragged: every member's V and Q 16-byte aligned with even leading dimensions
};

__host__ __device__ inline const MemberInfo& member_info(const MemberStride& ms, int64_t b) {
  return *reinterpret_cast<const MemberInfo*>(reinterpret_cast<const char*>(ms.info) + b * ms.ws);
}

__host__ __device__ inline uint64_t member_seed(uint64_t seed, const MemberStride& ms, int64_t b) {
  if (ms.info != nullptr) return member_info(ms, b).seed;
  return ms.seeds != nullptr ? ms.seeds[b] : seed + (uint64_t)b;
}

template <class T>
__host__ __device__ inline T* member_ptr(T* p, int64_t bytes) {
  return p == nullptr ? p : (T*)((const char*)p + bytes);
}

// Member b's V, row count and leading dimension (uniform stride, or its MemberInfo).
template <class P>
__device__ inline void member_v(const MemberStride& ms, int64_t b, P& V, int64_t& m, int64_t& ldv) {
  if (ms.info != nullptr) {
    const MemberInfo& mi = member_info(ms, b);
    V = mi.V;
    m = mi.m;
    ldv = mi.ldv;
  } else {
    V += b * ms.v;
  }
}

// --- sketch.hip --------------------------------------------------------------------------
// members > 1: the same fill at p + b * member_words, b < members
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s, int members = 1, int64_t member_words = 0);
hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t s);
// dst[i] = src[i], i < count <= 256 (one workgroup; a kernel, so it can sit in a captured graph)
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int count, hipStream_t s);
// Bucket index of S1 over `nchunk` contiguous row chunks (one workgroup each):
//   hash_hist:  codes[i] = (h(i) << 1) | signbit(i); hist[chunk][b] = rows of the chunk in bucket b
//   colscan:    hist[chunk][b] <- rows of bucket b in earlier chunks; counts[b] = bucket size;
//               unsorted[b] = 0 (when non-null)
//   scan:       offsets[0..s1] = exclusive scan of counts (cursor[b] = offsets[b] if non-null)
//   scatter:    entries[offsets[b] + hist[chunk][b] + k] = (i << 1) | signbit(i)
hipError_t launch_hash_hist(int64_t m, int64_t s1, uint64_t seed, int nchunk, uint32_t* codes, uint32_t* hist, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_hist_colscan(int nchunk, int64_t s1, uint32_t* hist, uint32_t* counts, uint8_t* unsorted, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_bucket_scan(const uint32_t* counts, int64_t s1, uint32_t* offsets, uint32_t* cursor, hipStream_t s, const MemberStride& ms = MemberStride());
//              when the bucket counters fit in LDS, each chunk's segment of each bucket is then
//              sorted by row, so every bucket lists its rows in ascending order; a segment too
//              long for the in-register sort sets unsorted[b] (s1 bytes, zero on entry)
hipError_t launch_bucket_scatter(int64_t m, int64_t s1, int nchunk, const uint32_t* codes, const uint32_t* offsets, uint32_t* hist,
                                 uint32_t* entries, uint8_t* unsorted, hipStream_t s, const MemberStride& ms = MemberStride());
// True when launch_bucket_scatter leaves the buckets sorted (up to the flagged ones).
bool bucket_scatter_sorts(int64_t s1);
// W1[b, :] = sum over the bucket's rows (ascending row order) of sign * V[row, :]; the float
// overload rounds each entry of V to FP32 and accumulates in FP32 (single-precision sketch).
// unsorted == nullptr: every bucket is sorted here; otherwise only the flagged ones are.
hipError_t launch_bucket_gather(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, const uint32_t* offsets,
                                const uint32_t* entries, const uint8_t* unsorted, double* W1, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_bucket_gather(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, const uint32_t* offsets,
                                const uint32_t* entries, const uint8_t* unsorted, float* W1, hipStream_t s);
// Small-s1 CountSketch: per-wave LDS copies of W1; writes one partial W1 per workgroup.
hipError_t launch_countsketch_lds(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, uint64_t seed,
                                  double* parts, int nparts, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_countsketch_lds(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, uint64_t seed,
                                  float* parts, int nparts, hipStream_t s);
// Wpart[kc] = S2[:, kc-th chunk of KC columns] * W1[chunk, :], S2 generated on the fly.
hipError_t launch_gauss_gemm(const double* W1, int n, int64_t s1, int64_t s2, uint64_t seed, double scale, int64_t kc_len,
                             int64_t nkc, double* wpart, hipStream_t s, const MemberStride& ms = MemberStride());
// The same product in FP32 on the matrix cores (kc_len a multiple of 32): FP32 operands, or
// operands rounded to BF16 (bf16 = true); FP32 accumulation.
hipError_t launch_gauss_mfma(const float* W1, int n, int64_t s1, int64_t s2, uint64_t seed, double scale, int64_t kc_len,
                             int64_t nkc, bool bf16, float* wpart, hipStream_t s);
// out[i] = sum_{p = 0..nparts-1} parts[p * stride + i], compensated, in a fixed order that depends
// only on nparts (16 interleaved groups of parts, then the group sums in order).
// In a ragged batch the partial count is the member's own: parts_kind kPartsCountSketch (its
// CountSketch copies) or kPartsGram (its Gram pass workgroups); kPartsUniform takes nparts.
enum { kPartsUniform = 0, kPartsCountSketch = 1, kPartsGram = 2 };
hipError_t launch_reduce_parts(const double* parts, int64_t nparts, int64_t stride, int64_t len, double* out,
                               hipStream_t s, const MemberStride& ms = MemberStride(), int parts_kind = kPartsUniform);
hipError_t launch_reduce_parts(const float* parts, int64_t nparts, int64_t stride, int64_t len, float* out, hipStream_t s);
hipError_t launch_widen(const float* in, int64_t count, double* out, hipStream_t s);
hipError_t launch_hash_debug(int64_t row0, int64_t count, int64_t s1, uint64_t seed, int32_t* bucket, int8_t* sign,
                             hipStream_t s);
hipError_t launch_gaussian_block(int64_t j0, int64_t nj, int64_t k0, int64_t nk, uint64_t seed, double scale,
                                 double* out, hipStream_t s);

// --- smalldense.hip ------------------------------------------------------------------------
// R (n x n, row-major, ld n) = R factor of the p x n block `in` (ld ldin, p <= 256) by
// Householder reflections; rows of R beyond min(p, n) are zero.  One workgroup per block:
// block b reads rows [b*rows_per_block, ...) and writes out + b*n*n.  With r0 set (the last level
// of the tree: one block) it writes instead what launch_finalize_r0 would make of that R: r0, its
// packed padded form r0pk (np columns) and the rank status in info.
hipError_t launch_qr_blocks(const double* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, double* out,
                            int nblocks, hipStream_t s, const MemberStride& ms = MemberStride(), double* r0 = nullptr,
                            double* r0pk = nullptr, int32_t* info = nullptr, int np = 0);
hipError_t launch_qr_blocks(const float* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, float* out,
                            int nblocks, hipStream_t s, const MemberStride& ms = MemberStride(), double* r0 = nullptr,
                            double* r0pk = nullptr, int32_t* info = nullptr, int np = 0);
// Sign-normalise an upper-triangular R (rows scaled so the diagonal is positive), check its
// diagonal (status RANK on zero / non-finite), write R0 (n x n) and its packed padded form.
hipError_t launch_finalize_r0(const double* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s, const MemberStride& ms = MemberStride());
// Cholesky of the Gram matrix held as compact upper 16x16 blocks; writes G (n x n, upper,
// lower zero), R1 and its packed padded form, and R = R1 * Rprev into the caller's R
// (ld ldr).  A non-positive pivot sets status CHOL.
// shift_coef != 0 factors G + shift_coef * trace(G) * I instead of G.
hipError_t launch_cholesky(const double* gcompact, int n, int np, const double* rprev, double shift_coef, int32_t* info,
                           double* g_out, double* r1, double* r1pk, double* r_out, int64_t ldr, hipStream_t s, const MemberStride& ms = MemberStride());
// One-time host-side setup of the Cholesky kernel for np (its LDS limit); done before any
// stream capture so that no attribute call happens inside a captured graph.
hipError_t prepare_cholesky(int np);
// Identity (n x n) into r0 and its packed padded form into r0pk.
hipError_t launch_identity_factor(int n, int np, double* r0, double* r0pk, hipStream_t s);

// --- stream.hip ------------------------------------------------------------------------------
int gram_compact_len(int np);        // doubles per compact Gram partial
int packed_len(int np);              // doubles of a packed np x np triangular factor
// Packed factor format (R padded to np columns with an identity block): the upper triangle
// row by row, the reciprocal of each diagonal entry in place of the entry.
hipError_t launch_trsm_gram(int np, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk, const int32_t* info,
                            double* gpart, double* q0, int64_t ldq, hipStream_t s, const MemberStride& ms = MemberStride());
// Device properties the launchers read (multiprocessor count), queried once, before any capture.
hipError_t prepare_stream_launches();
// grid_mult: workgroups per CU cap of the multi-row kernels (a launch-shape knob; never changes results).
// In a batch the one-factor pass (apply_r1 = false) reads the member's V, or its Q when src_q.
hipError_t launch_final(int np, bool apply_r1, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk,
                        const double* r1pk, const int32_t* info, double* Q, int64_t ldq, hipStream_t s, int grid_mult = 2,
                        const MemberStride& ms = MemberStride(), int src_q = 0);
// Q = Q0 R1^{-1} in place for a stored Q0 (np <= 64), bitwise the same as launch_final's second step.
hipError_t launch_apply_rinv(int np, double* Q, int64_t m, int n, int64_t ldq, const double* r1pk, const int32_t* info, int grid_mult,
                             hipStream_t s);

// --- stream128.hip (65..128 columns; factor in the blocked packed format) --------------------
// out = in R^{-1} row by row (out may alias in with the same leading dimension).
// In a batch the input rows are the member's V, or its Q when src_q; the output is its Q.
hipError_t launch_solve128(const double* in, int64_t m, int n, int64_t ldin, const double* rbk, const int32_t* info, double* out,
                           int64_t ldout, hipStream_t s, int grid_mult = 2, const MemberStride& ms = MemberStride(), int src_q = 0);
// The Gram phase's solve: Q0 = V R^{-1} into Q (Q may alias V), x_lo by the 64-column Gram pass,
// which also writes the Gram partials of columns 0..63 (gram_blocks(m) compact partials of 10
// blocks) to gplo for launch_syrk128.
hipError_t launch_solve128_gram(const double* V, int64_t m, int n, int64_t ldv, const double* rbk, const int32_t* info, double* Q,
                                int64_t ldq, double* gplo, hipStream_t s, int grid_mult = 2, const MemberStride& ms = MemberStride());
// R1^{-1} of a blocked packed factor as the 36 upper 16 x 16 blocks (rinv: 36 * 256 doubles), and
// Q = Q0 R1^{-1} in place on the stored Q0 from them (65..128 columns).
hipError_t launch_rinv128(const double* rbk, const int32_t* info, double* rinv, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_apply_rinv128(double* Q, int64_t m, int n, int64_t ldq, const double* rinv, const int32_t* info, int grid_mult,
                                hipStream_t s, const MemberStride& ms = MemberStride());
// Gram partials of Q0 (kGramBlocks compact partials of 36 upper 16x16 blocks): the blocks that
// involve columns 64..127 from Q0, those of columns 0..63 copied from the nblo partials in gplo
// (launch_solve128_gram's; a ragged member's count is its own Gram grid).
hipError_t launch_syrk128(const double* Q0, int64_t m, int n, int64_t ldq, const int32_t* info, double* gpart, const double* gplo,
                          int64_t nblo, hipStream_t s, const MemberStride& ms = MemberStride());

}  // namespace rcqr
