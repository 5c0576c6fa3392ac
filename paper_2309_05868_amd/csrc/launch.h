// Host-callable launchers of the rcqr kernels (one per kernel family).  Every launcher only
// enqueues work on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcqr {

// A batch of same-shaped factorizations in one set of launches: member b of a launch is a grid
// index (blockIdx.y, or blockIdx.z where y is taken); its workspace pointers move by b * ws
// bytes, V, Q and R by b * v, b * q, b * r elements, and its sketch seed is seeds[b] (a device
// array) or, without one, the plan's seed + b.  All zero, one member, for a single
// factorization (the kernels then compute exactly what they did alone).
struct MemberStride {
  int64_t ws = 0, v = 0, q = 0, r = 0;
  int32_t count = 1;
  const uint64_t* seeds = nullptr;
};

__host__ __device__ inline uint64_t member_seed(uint64_t seed, const MemberStride& ms, int64_t b) {
  return ms.seeds != nullptr ? ms.seeds[b] : seed + (uint64_t)b;
}

template <class T>
__host__ __device__ inline T* member_ptr(T* p, int64_t bytes) {
  return p == nullptr ? p : (T*)((const char*)p + bytes);
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
int64_t bucket_chunk_rows(int64_t m, int nchunk);
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
int countsketch_lds_parts(int64_t m, int64_t s1, int n);
bool countsketch_lds_fits(int64_t s1, int n);
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
hipError_t launch_reduce_parts(const double* parts, int64_t nparts, int64_t stride, int64_t len, double* out,
                               hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_reduce_parts(const float* parts, int64_t nparts, int64_t stride, int64_t len, float* out, hipStream_t s);
hipError_t launch_widen(const float* in, int64_t count, double* out, hipStream_t s);
hipError_t launch_hash_debug(int64_t row0, int64_t count, int64_t s1, uint64_t seed, int32_t* bucket, int8_t* sign,
                             hipStream_t s);
hipError_t launch_gaussian_block(int64_t j0, int64_t nj, int64_t k0, int64_t nk, uint64_t seed, double scale,
                                 double* out, hipStream_t s);

// --- smalldense.hip ------------------------------------------------------------------------
// R (n x n, row-major, ld n) = R factor of the p x n block `in` (ld ldin, p <= 256) by
// Householder reflections; rows of R beyond min(p, n) are zero.  One workgroup per block:
// block b reads rows [b*rows_per_block, ...) and writes out + b*n*n.
hipError_t launch_qr_blocks(const double* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, double* out,
                            int nblocks, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_qr_blocks(const float* in, int64_t ldin, int64_t p_total, int64_t rows_per_block, int n, float* out,
                            int nblocks, hipStream_t s);
// Sign-normalise the Householder R (rows scaled so the diagonal is positive), check its
// diagonal (status RANK on zero / non-finite), write R0 (n x n) and its packed padded form.
// The float overload promotes an FP32 Householder R to FP64 first.
hipError_t launch_finalize_r0(const double* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s, const MemberStride& ms = MemberStride());
hipError_t launch_finalize_r0(const float* rin, int n, int np, int32_t* info, double* r0, double* r0pk, hipStream_t s);
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
constexpr int kGramBlocks = 256;     // most workgroups of the Gram pass (the count fixes the sum order)
constexpr int kGramThreads = 512;
// Workgroups of the Gram pass (and Gram partials) for m rows: one per eight 64-row tiles (one
// tile per wave), at most kGramBlocks.  A function of m alone, so the summation order is fixed
// by the shape; a small matrix does not pay for kGramBlocks partials that would hold zeros.
inline int gram_blocks(int64_t m) {
  const int64_t per = kGramThreads;  // eight waves, one 64-row tile each
  const int64_t b = (m + per - 1) / per;
  return b < 1 ? 1 : (b > kGramBlocks ? kGramBlocks : (int)b);
}
int gram_compact_len(int np);        // doubles per compact Gram partial
int packed_len(int np);              // doubles of a packed np x np triangular factor
// Packed factor format (R padded to np columns with an identity block): the upper triangle
// row by row, the reciprocal of each diagonal entry in place of the entry.
hipError_t launch_trsm_gram(int np, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk, const int32_t* info,
                            double* gpart, double* q0, int64_t ldq, hipStream_t s, const MemberStride& ms = MemberStride());
// Device properties the launchers read (multiprocessor count), queried once, before any capture.
hipError_t prepare_stream_launches();
// grid_mult: workgroups per CU cap of the multi-row kernels (a launch-shape knob; never changes results).
hipError_t launch_final(int np, bool apply_r1, const double* V, int64_t m, int n, int64_t ldv, const double* r0pk,
                        const double* r1pk, const int32_t* info, double* Q, int64_t ldq, hipStream_t s, int grid_mult = 2, const MemberStride& ms = MemberStride());
// Q = Q0 R1^{-1} in place for a stored Q0 (np <= 64), bitwise the same as launch_final's second step.
hipError_t launch_apply_rinv(int np, double* Q, int64_t m, int n, int64_t ldq, const double* r1pk, const int32_t* info, int grid_mult,
                             hipStream_t s);

// --- stream128.hip (65..128 columns; factor in the blocked packed format) --------------------
// out = in R^{-1} row by row (out may alias in with the same leading dimension).
hipError_t launch_solve128(const double* in, int64_t m, int n, int64_t ldin, const double* rbk, const int32_t* info, double* out,
                           int64_t ldout, hipStream_t s, int grid_mult = 2);
// Gram partials of Q0 (kGramBlocks compact partials of 36 upper 16x16 blocks).
hipError_t launch_syrk128(const double* Q0, int64_t m, int n, int64_t ldq, const int32_t* info, double* gpart, hipStream_t s);

}  // namespace rcqr
