// Sketch kernels: CountSketch W1 = S1 V and Gaussian sketch W = S2 W1 (Algorithm 1, step 1).
//
// The CountSketch has one +-1 per column of S1 (Section 3), so W1 = S1 V adds or subtracts
// rows of V into s1 buckets (Section 4.2).  Two strategies, both deterministic:
//   * small s1*n (<= 4096 entries): every wave keeps a private copy of W1 in LDS and streams
//     contiguous rows of V; rows of one batch that share a bucket are first combined by the
//     lowest such lane, in row order; the copies are summed in fixed order.
//   * otherwise: a bucket index (CSR of S1) is built per call -- hash codes, bucket counts,
//     exclusive scan, scatter of (row, sign) -- and one wave per bucket gathers its rows.  The
//     scatter sorts each chunk's short segment of each bucket (or the gather sorts the bucket),
//     so the sum order is ascending row order whatever order the scatter's atomics produced.
// The Gaussian sketch S2 = G / sqrt(s2) (Section 3) is never stored: each GEMM workgroup
// regenerates its 64 x 16 tiles of S2 from Philox counters in LDS.
#include "device_common.h"
#include "launch.h"

namespace rcqr {

// ------------------------------------------------------------------------------------------
// fills
// ------------------------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t* p, int64_t count, uint32_t v, int64_t member_words) {
  p += blockIdx.y * member_words;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static int grid_for(int64_t count, int threads, int cap = 4096) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s, int members, int64_t member_words) {
  if (count <= 0 || members < 1) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count, 256), members), dim3(256), 0, s, p, count, value, member_words);
  return hipGetLastError();
}
__global__ void copy_i32_kernel(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = src[i];
}

hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_i32_kernel, dim3(1), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// CountSketch hash and per-chunk bucket histograms.  Rows are split into `nchunk` contiguous
// chunks (a multiple of 4 rows each, one workgroup per chunk); one Philox block serves rows
// 4q .. 4q+3.  hist[chunk][b] = number of rows of the chunk in bucket b.
// ------------------------------------------------------------------------------------------
constexpr int kHistLds = 32768;     // buckets counted in LDS by the hash (128 KiB); above this, in the chunk's global row
constexpr int kScatterLds = 16384;  // buckets whose counters and segment starts the scatter keeps in LDS

__global__ __launch_bounds__(1024) void hash_hist_kernel(int64_t m, uint64_t s1, uint64_t seed, int64_t chunk_rows, uint32_t* __restrict__ codes,
                                                        uint32_t* __restrict__ hist, MemberStride ms) {
  __shared__ uint32_t lh[kHistLds];
  {
    const int64_t mb = blockIdx.y;  // batch member
    codes = member_ptr(codes, mb * ms.ws);
    hist = member_ptr(hist, mb * ms.ws);
    seed = member_seed(seed, ms, mb);
    if (ms.info != nullptr) {  // ragged batch: the member's rows and chunks
      const MemberInfo& mi = member_info(ms, mb);
      if ((int)blockIdx.x >= mi.nchunk) return;
      m = mi.m;
      chunk_rows = mi.chunk_rows;
    }
  }
  const bool in_lds = s1 <= (uint64_t)kHistLds;
  uint32_t* gh = hist + (int64_t)blockIdx.x * (int64_t)s1;
  if (in_lds) {
    for (int64_t b = threadIdx.x; b < (int64_t)s1; b += blockDim.x) lh[b] = 0u;
  } else {
    for (int64_t b = threadIdx.x; b < (int64_t)s1; b += blockDim.x) gh[b] = 0u;
  }
  __syncthreads();
  const int64_t r_beg = (int64_t)blockIdx.x * chunk_rows;
  const int64_t r_end = r_beg + chunk_rows < m ? r_beg + chunk_rows : m;
  for (int64_t r = r_beg + 4 * (int64_t)threadIdx.x; r < r_end; r += 4 * (int64_t)blockDim.x) {
    const Block4 y = philox4x64_10((uint64_t)(r >> 2), 0, 0, kTagCountSketch, seed, 0);
    const uint32_t c[4] = {countsketch_code(y.y0, s1), countsketch_code(y.y1, s1), countsketch_code(y.y2, s1),
                           countsketch_code(y.y3, s1)};
    if (r + 3 < r_end) {
      *reinterpret_cast<uint4*>(codes + r) = make_uint4(c[0], c[1], c[2], c[3]);
    } else {
      for (int u = 0; u < 4 && r + u < r_end; ++u) codes[r + u] = c[u];
    }
    for (int u = 0; u < 4 && r + u < r_end; ++u) {
      if (in_lds)
        atomicAdd(&lh[c[u] >> 1], 1u);
      else
        atomicAdd(&gh[c[u] >> 1], 1u);
    }
  }
  if (in_lds) {
    __syncthreads();
    for (int64_t b = threadIdx.x; b < (int64_t)s1; b += blockDim.x) gh[b] = lh[b];
  }
}

hipError_t launch_hash_hist(int64_t m, int64_t s1, uint64_t seed, int nchunk, uint32_t* codes, uint32_t* hist, hipStream_t s,
                            const MemberStride& ms) {
  if (m <= 0) return hipSuccess;
  if (ms.count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hash_hist_kernel, dim3(nchunk, ms.count), dim3(1024), 0, s, m, (uint64_t)s1, seed, bucket_chunk_rows(m, nchunk), codes,
                     hist, ms);
  return hipGetLastError();
}

// hist[chunk][b] <- rows of bucket b in earlier chunks (exclusive scan down each column);
// counts[b] <- total rows of bucket b.  Workgroup: 32 buckets x 16 chunk segments; each thread
// scans its segment of one column, the segment totals are combined through LDS.
__global__ __launch_bounds__(512) void hist_colscan_kernel(int nchunk, int64_t s1, uint32_t* __restrict__ hist, uint32_t* __restrict__ counts,
                                                           uint8_t* __restrict__ unsorted, MemberStride ms) {
  constexpr int NB = 32, NS = 16, BATCH = 8;
  {
    const int64_t off = (int64_t)blockIdx.y * ms.ws;  // batch member
    hist = member_ptr(hist, off);
    counts = member_ptr(counts, off);
    unsorted = member_ptr(unsorted, off);
    if (ms.info != nullptr) nchunk = member_info(ms, blockIdx.y).nchunk;
  }
  __shared__ uint32_t segtot[NS][NB];
  const int bl = threadIdx.x % NB, sg = threadIdx.x / NB;
  const int64_t b = (int64_t)blockIdx.x * NB + bl;
  const int per = (nchunk + NS - 1) / NS;
  const int c_beg = sg * per, c_end = c_beg + per < nchunk ? c_beg + per : nchunk;
  uint32_t v[BATCH];
  uint32_t run = 0;
  // pass 1: segment total
  if (b < s1) {
    for (int c0 = c_beg; c0 < c_end; c0 += BATCH) {
#pragma unroll
      for (int u = 0; u < BATCH; ++u) v[u] = (c0 + u < c_end) ? hist[(int64_t)(c0 + u) * s1 + b] : 0u;
#pragma unroll
      for (int u = 0; u < BATCH; ++u) run += v[u];
    }
  }
  segtot[sg][bl] = run;
  __syncthreads();
  if (b >= s1) return;
  uint32_t pre = 0;
  for (int h = 0; h < sg; ++h) pre += segtot[h][bl];
  if (sg == NS - 1) {
    counts[b] = pre + run;
    if (unsorted) unsorted[b] = 0;
  }
  // pass 2: exclusive prefix within the segment (the values are L2-resident from pass 1)
  for (int c0 = c_beg; c0 < c_end; c0 += BATCH) {
#pragma unroll
    for (int u = 0; u < BATCH; ++u) v[u] = (c0 + u < c_end) ? hist[(int64_t)(c0 + u) * s1 + b] : 0u;
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      if (c0 + u < c_end) hist[(int64_t)(c0 + u) * s1 + b] = pre;
      pre += v[u];
    }
  }
}

hipError_t launch_hist_colscan(int nchunk, int64_t s1, uint32_t* hist, uint32_t* counts, uint8_t* unsorted, hipStream_t s,
                               const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hist_colscan_kernel, dim3((unsigned)((s1 + 31) / 32), ms.count), dim3(512), 0, s, nchunk, s1, hist, counts, unsorted,
                     ms);
  return hipGetLastError();
}

// Debug: bucket and sign per row.
__global__ void hash_debug_kernel(int64_t row0, int64_t count, uint64_t s1, uint64_t seed, int32_t* bucket, int8_t* sign) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t row = (uint64_t)(row0 + i);
    const Block4 y = philox4x64_10(row >> 2, 0, 0, kTagCountSketch, seed, 0);
    const uint32_t code = countsketch_code(block_word(y, (int)(row & 3)), s1);
    bucket[i] = (int32_t)(code >> 1);
    sign[i] = (code & 1) ? (int8_t)-1 : (int8_t)1;
  }
}

hipError_t launch_hash_debug(int64_t row0, int64_t count, int64_t s1, uint64_t seed, int32_t* bucket, int8_t* sign,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(hash_debug_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, row0, count, (uint64_t)s1, seed, bucket, sign);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Bucket index: exclusive scan (one workgroup) and scatter.
// ------------------------------------------------------------------------------------------
// Tiles of 1024 x PER counts, moved between memory and LDS by coalesced loads and stores: each
// thread scans PER consecutive counts from LDS (padded by one word per 32, so the threads of a wave
// read different banks), the 1024 thread totals are scanned by waves (shuffles) and across the 16
// waves through LDS, plus the carry of earlier tiles.
template <int PER>
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const uint32_t* __restrict__ counts, int64_t s1,
                                                           uint32_t* __restrict__ offsets, uint32_t* __restrict__ cursor,
                                                           int64_t member_bytes) {
  constexpr int TILE = 1024 * PER;
  {
    const int64_t off = (int64_t)blockIdx.y * member_bytes;  // batch member
    counts = member_ptr(counts, off);
    offsets = member_ptr(offsets, off);
    cursor = member_ptr(cursor, off);
  }
  __shared__ uint32_t tile[TILE + TILE / 32];
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry_s;
  const int t = threadIdx.x, lane = lane_id(), wave = t / kWave;
  auto at = [](int i) { return i + (i >> 5); };
  uint32_t carry = 0;
  for (int64_t base = 0; base < s1; base += TILE) {
    for (int i = t; i < TILE; i += 1024) tile[at(i)] = base + i < s1 ? counts[base + i] : 0u;
    __syncthreads();
    uint32_t v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = tile[at(t * PER + u)];
    uint32_t tot = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) tot += v[u];
    // inclusive scan of the thread totals within the wave
    uint32_t inc = tot;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();  // every thread has read its counts from the tile
    uint32_t before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    uint32_t run = before + inc - tot;  // exclusive prefix of this thread's first count
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      tile[at(t * PER + u)] = run;
      run += v[u];
    }
    if (t == 1023) carry_s = run;
    __syncthreads();
    carry = carry_s;
    for (int i = t; i < TILE; i += 1024) {
      if (base + i < s1) {
        const uint32_t o = tile[at(i)];
        offsets[base + i] = o;
        if (cursor) cursor[base + i] = o;
      }
    }
    __syncthreads();  // the tile and wsum are reused by the next tile
  }
  if (t == 0) offsets[s1] = carry;
}

hipError_t launch_bucket_scan(const uint32_t* counts, int64_t s1, uint32_t* offsets, uint32_t* cursor, hipStream_t s,
                              const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  // one pass of 1024 x PER buckets at a time: eight per thread up to 8192 buckets, 32 above (one
  // pass up to 32768; the passes are bound by their shuffles and barriers, not their loads)
  if (s1 <= 8192)
    hipLaunchKernelGGL(bucket_scan_kernel<8>, dim3(1, ms.count), dim3(1024), 0, s, counts, s1, offsets, cursor, ms.ws);
  else
    hipLaunchKernelGGL(bucket_scan_kernel<32>, dim3(1, ms.count), dim3(1024), 0, s, counts, s1, offsets, cursor, ms.ws);
  return hipGetLastError();
}

// Ascending sort of p[0..len) (len <= N, distinct keys) by a bitonic network in registers.
template <int N>
__device__ __forceinline__ void sort_segment(uint32_t* p, int len) {
  uint32_t v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = i < len ? p[i] : 0xFFFFFFFFu;
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const uint32_t a = v[i], b = v[l];
          const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
          const bool up = (i & k) == 0;
          v[i] = up ? lo : hi;
          v[l] = up ? hi : lo;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < len) p[i] = v[i];
}

bool bucket_scatter_sorts(int64_t s1) { return s1 <= (int64_t)kScatterLds; }

// entries[offsets[b] + base(chunk, b) + k] = (row << 1) | signbit for the k-th row of the chunk
// in bucket b.  k comes from an LDS counter, so the order inside a chunk's segment is whatever
// the atomics give; the segment (this workgroup's rows of bucket b, typically a few) is then
// sorted in registers.  Segments follow each other in chunk order, so each bucket ends up in
// ascending row order.  A segment longer than the largest network flags its bucket for the
// gather's own sort.  With the counters in global memory (s1 above the LDS limit) the
// segments are left as they are and the gather sorts every bucket.
__global__ __launch_bounds__(1024) void bucket_scatter_kernel(int64_t m, int64_t s1, int64_t chunk_rows, const uint32_t* __restrict__ codes,
                                                             const uint32_t* __restrict__ offsets, uint32_t* __restrict__ hist,
                                                             uint32_t* entries, uint8_t* __restrict__ unsorted, MemberStride ms) {
  __shared__ uint32_t cur[kScatterLds];
  {
    const int64_t off = (int64_t)blockIdx.y * ms.ws;  // batch member
    codes = member_ptr(codes, off);
    offsets = member_ptr(offsets, off);
    hist = member_ptr(hist, off);
    entries = member_ptr(entries, off);
    unsorted = member_ptr(unsorted, off);
    if (ms.info != nullptr) {  // ragged batch: the member's rows and chunks
      const MemberInfo& mi = member_info(ms, blockIdx.y);
      if ((int)blockIdx.x >= mi.nchunk) return;
      m = mi.m;
      chunk_rows = mi.chunk_rows;
    }
  }
  __shared__ uint32_t seg0[kScatterLds];  // start of this chunk's segment of each bucket
  const bool in_lds = s1 <= (int64_t)kScatterLds;
  uint32_t* gh = hist + (int64_t)blockIdx.x * s1;
  if (in_lds) {
    for (int64_t b = threadIdx.x; b < s1; b += blockDim.x) {
      const uint32_t o = offsets[b] + gh[b];
      cur[b] = o;
      seg0[b] = o;
    }
    __syncthreads();
  }
  const int64_t r_beg = (int64_t)blockIdx.x * chunk_rows;
  const int64_t r_end = r_beg + chunk_rows < m ? r_beg + chunk_rows : m;
  for (int64_t r = r_beg + threadIdx.x; r < r_end; r += blockDim.x) {
    const uint32_t code = codes[r];
    const uint32_t b = code >> 1;
    const uint32_t pos = in_lds ? atomicAdd(&cur[b], 1u) : offsets[b] + atomicAdd(&gh[b], 1u);
    entries[pos] = ((uint32_t)r << 1) | (code & 1u);
  }
  if (!in_lds) return;
  __syncthreads();  // the workgroup's entries are written and visible to the workgroup
  for (int64_t b = threadIdx.x; b < s1; b += blockDim.x) {
    const uint32_t beg = seg0[b];
    const int len = (int)(cur[b] - beg);
    if (len <= 1) continue;
    uint32_t* seg = entries + beg;
    if (len <= 4)
      sort_segment<4>(seg, len);
    else if (len <= 8)
      sort_segment<8>(seg, len);
    else if (len <= 16)
      sort_segment<16>(seg, len);
    else if (len <= 32)
      sort_segment<32>(seg, len);
    else if (len <= 64)
      sort_segment<64>(seg, len);
    else
      unsorted[b] = 1;
  }
}

hipError_t launch_bucket_scatter(int64_t m, int64_t s1, int nchunk, const uint32_t* codes, const uint32_t* offsets, uint32_t* hist,
                                 uint32_t* entries, uint8_t* unsorted, hipStream_t s, const MemberStride& ms) {
  if (m <= 0) return hipSuccess;
  if ((bucket_scatter_sorts(s1) && unsorted == nullptr) || ms.count < 1) return hipErrorInvalidValue;
  // 16 waves per chunk with the counters in LDS (the chunk is one workgroup per CU); four with
  // global counters, whose atomics contend more with more waves (measured 99 -> 130 us at s1 = 32768)
  const int threads = bucket_scatter_sorts(s1) ? 1024 : 256;
  hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nchunk, ms.count), dim3(threads), 0, s, m, s1, bucket_chunk_rows(m, nchunk), codes, offsets,
                     hist, entries, unsorted, ms);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Bucket gather: one wave per bucket.
// ------------------------------------------------------------------------------------------
constexpr int kSortCap = 1024;  // entries one wave sorts in LDS at a time (16 KiB per workgroup: ten per CU)
constexpr int kGatherWaves = 4;

// Bitonic sort of keys[0..N) (N a power of two) by one wave.
__device__ void wave_bitonic_sort(uint32_t* keys, int N, int lane) {
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < N; i += kWave) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// Accumulate sorted entries keys[0..cnt) into acc (element type T: FP64, or FP32 for the
// single-precision sketch, where each V entry is rounded to FP32 before it is added): lane
// group g takes entries g, g+G, ...
template <int NPL, class T>
__device__ __forceinline__ void gather_rows(const uint32_t* keys, int cnt, const double* __restrict__ V, int64_t ldv, int n,
                                            int lane, T (&acc)[NPL > 64 ? 2 : 1]) {
  constexpr int G = NPL >= 64 ? 1 : 64 / NPL;
  const int g = NPL >= 64 ? 0 : lane / NPL;
  const int c = NPL >= 64 ? lane : lane % NPL;
  int e = g;
  // eight rows in flight per lane group, added in entry order
  constexpr int U = 8;
  for (; e + (U - 1) * G < cnt; e += U * G) {
    uint32_t kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) kk[u] = keys[e + u * G];
    // V is read once here: non-temporal loads (measured 5.8 -> 6.5 TB/s for this access pattern)
    if constexpr (NPL > 64) {
      double v[U][2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double* row = V + (int64_t)(kk[u] >> 1) * ldv;
        v[u][0] = c < n ? __builtin_nontemporal_load(row + c) : 0.0;
        v[u][1] = c + 64 < n ? __builtin_nontemporal_load(row + c + 64) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool neg = kk[u] & 1u;
        const T x0 = (T)v[u][0], x1 = (T)v[u][1];
        acc[0] += neg ? -x0 : x0;
        acc[1] += neg ? -x1 : x1;
      }
    } else {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = c < n ? __builtin_nontemporal_load(V + (int64_t)(kk[u] >> 1) * ldv + c) : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T x = (T)v[u];
        acc[0] += (kk[u] & 1u) ? -x : x;
      }
    }
  }
  for (; e < cnt; e += G) {
    const uint32_t k = keys[e];
    const double* row = V + (int64_t)(k >> 1) * ldv;
    const bool neg = k & 1u;
    const T v0 = (T)(c < n ? row[c] : 0.0);
    acc[0] += neg ? -v0 : v0;
    if constexpr (NPL > 64) {
      const T v1 = (T)(c + 64 < n ? row[c + 64] : 0.0);
      acc[1] += neg ? -v1 : v1;
    }
  }
}

template <int NPL, class T>
__global__ __launch_bounds__(256) void bucket_gather_kernel(const double* __restrict__ V, int64_t ldv, int64_t m, int n, int64_t s1,
                                                            const uint32_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ entries,
                                                            const uint8_t* __restrict__ unsorted, T* __restrict__ W1, MemberStride ms) {
  __shared__ uint32_t keys_all[kGatherWaves][kSortCap];
  {
    const int64_t mb = blockIdx.y, off = mb * ms.ws;  // batch member
    member_v(ms, mb, V, m, ldv);
    offsets = member_ptr(offsets, off);
    entries = member_ptr(entries, off);
    unsorted = member_ptr(unsorted, off);
    W1 = member_ptr(W1, off);
  }
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  const int64_t b = (int64_t)blockIdx.x * kGatherWaves + wave;
  if (b >= s1) return;  // whole wave leaves; no workgroup barrier below
  uint32_t* keys = keys_all[wave];
  const uint32_t beg = offsets[b];
  const int64_t L = (int64_t)offsets[b + 1] - beg;
  T acc[NPL > 64 ? 2 : 1];
  acc[0] = T(0);
  if constexpr (NPL > 64) acc[1] = T(0);

  if (unsorted != nullptr && unsorted[b] == 0) {
    // already in ascending row order: consecutive slices through LDS (one coalesced copy each,
    // so the row addresses come from LDS), no sort
    for (int64_t s0 = 0; s0 < L; s0 += kSortCap) {
      const int cnt = (int)(L - s0 < kSortCap ? L - s0 : kSortCap);
      for (int i = lane; i < cnt; i += kWave) keys[i] = entries[beg + s0 + i];
      wave_lds_sync();
      gather_rows<NPL, T>(keys, cnt, V, ldv, n, lane, acc);
      wave_lds_sync();
    }
  } else if (L <= kSortCap) {
    int N = 1;
    while (N < L) N <<= 1;
    for (int i = lane; i < N; i += kWave) keys[i] = i < L ? entries[beg + i] : 0xFFFFFFFFu;
    wave_lds_sync();
    wave_bitonic_sort(keys, N, lane);
    gather_rows<NPL, T>(keys, (int)L, V, ldv, n, lane, acc);
  } else {
    // Windows of rows [lo, hi) small enough to sort; together they visit the bucket's
    // entries in ascending row order.
    int64_t lo = 0, remaining = L;
    while (remaining > 0) {
      int64_t span = (m - lo) * (kSortCap / 2) / remaining;
      if (span < 1) span = 1;
      int64_t hi, cnt;
      for (;;) {
        hi = lo + span < m ? lo + span : m;
        cnt = 0;
        for (int64_t i = lane; i < L; i += kWave) {
          const int64_t row = entries[beg + i] >> 1;
          cnt += (row >= lo && row < hi) ? 1 : 0;
        }
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
        if (cnt <= kSortCap) break;
        span = span / 2 > 0 ? span / 2 : 1;
      }
      int base = 0;
      for (int64_t i0 = 0; i0 < L; i0 += kWave) {
        const int64_t i = i0 + lane;
        uint32_t key = 0;
        bool pred = false;
        if (i < L) {
          key = entries[beg + i];
          const int64_t row = key >> 1;
          pred = row >= lo && row < hi;
        }
        const uint64_t mask = __ballot(pred);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (pred) keys[pos] = key;
        base += __popcll(mask);
      }
      int N = 1;
      while (N < cnt) N <<= 1;
      for (int i = (int)cnt + lane; i < N; i += kWave) keys[i] = 0xFFFFFFFFu;
      wave_lds_sync();
      wave_bitonic_sort(keys, N, lane);
      gather_rows<NPL, T>(keys, (int)cnt, V, ldv, n, lane, acc);
      wave_lds_sync();
      remaining -= cnt;
      lo = hi;
    }
  }
  if constexpr (NPL < 64) {
    for (int off = NPL; off < kWave; off <<= 1) acc[0] += shfl_xor_d(acc[0], off);
    if (lane < NPL && lane < n) W1[b * n + lane] = acc[0];
  } else {
    if (lane < n) W1[b * n + lane] = acc[0];
    if constexpr (NPL > 64) {
      if (lane + 64 < n) W1[b * n + lane + 64] = acc[1];
    }
  }
}

template <class T>
static hipError_t bucket_gather_any(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, const uint32_t* offsets,
                                    const uint32_t* entries, const uint8_t* unsorted, T* W1, hipStream_t s,
                                    const MemberStride& ms) {
  if (ms.count < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((s1 + kGatherWaves - 1) / kGatherWaves), ms.count), block(256);
  if (n <= 8)
    hipLaunchKernelGGL((bucket_gather_kernel<8, T>), grid, block, 0, s, V, ldv, m, n, s1, offsets, entries, unsorted, W1, ms);
  else if (n <= 16)
    hipLaunchKernelGGL((bucket_gather_kernel<16, T>), grid, block, 0, s, V, ldv, m, n, s1, offsets, entries, unsorted, W1, ms);
  else if (n <= 32)
    hipLaunchKernelGGL((bucket_gather_kernel<32, T>), grid, block, 0, s, V, ldv, m, n, s1, offsets, entries, unsorted, W1, ms);
  else if (n <= 64)
    hipLaunchKernelGGL((bucket_gather_kernel<64, T>), grid, block, 0, s, V, ldv, m, n, s1, offsets, entries, unsorted, W1, ms);
  else
    hipLaunchKernelGGL((bucket_gather_kernel<128, T>), grid, block, 0, s, V, ldv, m, n, s1, offsets, entries, unsorted, W1, ms);
  return hipGetLastError();
}

hipError_t launch_bucket_gather(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, const uint32_t* offsets,
                                const uint32_t* entries, const uint8_t* unsorted, double* W1, hipStream_t s, const MemberStride& ms) {
  return bucket_gather_any(V, ldv, m, n, s1, offsets, entries, unsorted, W1, s, ms);
}

hipError_t launch_bucket_gather(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, const uint32_t* offsets,
                                const uint32_t* entries, const uint8_t* unsorted, float* W1, hipStream_t s) {
  return bucket_gather_any(V, ldv, m, n, s1, offsets, entries, unsorted, W1, s, MemberStride());
}

// ------------------------------------------------------------------------------------------
// Small-s1 CountSketch: per-wave LDS copies of W1 (s1 x NPL), contiguous row chunks.
// ------------------------------------------------------------------------------------------
template <int NPL, class T, int CAP>
__global__ __launch_bounds__(256) void countsketch_lds_kernel(const double* __restrict__ V, int64_t ldv, int64_t m, int n, int64_t s1,
                                                              uint64_t seed, T* __restrict__ parts, MemberStride ms) {
  __shared__ T w1[4][CAP];
  {
    const int64_t mb = blockIdx.y;  // batch member
    member_v(ms, mb, V, m, ldv);
    parts = member_ptr(parts, mb * ms.ws);
    seed = member_seed(seed, ms, mb);
  }
  // workgroups of this member (the grid is sized for the largest member of a ragged batch)
  const int64_t nparts = ms.info != nullptr ? member_info(ms, blockIdx.y).cs_parts : (int64_t)gridDim.x;
  if ((int64_t)blockIdx.x >= nparts) return;
  __shared__ uint32_t codes[4][kCsChunk];
  constexpr int RB = kWave / NPL;  // rows per batch
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int q = lane / NPL, c = lane % NPL;
  T* mine = w1[wave];
  for (int i = lane; i < s1 * NPL; i += kWave) mine[i] = T(0);
  // rows of this workgroup
  const int64_t per = ((m + nparts - 1) / nparts + kCsChunk - 1) / kCsChunk * kCsChunk;
  const int64_t r_beg = (int64_t)blockIdx.x * per;
  const int64_t r_end = r_beg + per < m ? r_beg + per : m;
  wave_lds_sync();
  for (int64_t base = r_beg + (int64_t)wave * kCsChunk; base < r_end; base += 4 * kCsChunk) {
    // hash the chunk: lane computes the Philox block of rows base + 4*lane .. +3 (base % 4 == 0)
    {
      const Block4 y = philox4x64_10((uint64_t)(base >> 2) + lane, 0, 0, kTagCountSketch, seed, 0);
      codes[wave][4 * lane + 0] = countsketch_code(y.y0, (uint64_t)s1);
      codes[wave][4 * lane + 1] = countsketch_code(y.y1, (uint64_t)s1);
      codes[wave][4 * lane + 2] = countsketch_code(y.y2, (uint64_t)s1);
      codes[wave][4 * lane + 3] = countsketch_code(y.y3, (uint64_t)s1);
    }
    wave_lds_sync();
    const int rows = (int)((r_end - base) < kCsChunk ? (r_end - base) : kCsChunk);
    // the rows of a sub-chunk are loaded together (NBS independent loads per lane in flight),
    // then added batch by batch in row order
    constexpr int SCR = NPL <= 16 ? 128 : 64;  // rows per sub-chunk
    constexpr int NBS = SCR / RB;              // batches per sub-chunk
    for (int s0 = 0; s0 < rows; s0 += SCR) {
    T vv[NBS];
#pragma unroll
    for (int k = 0; k < NBS; ++k) {
      const int rq = s0 + k * RB + q;
      vv[k] = (T)((rq < rows && c < n) ? __builtin_nontemporal_load(V + (base + rq) * ldv + c) : 0.0);
    }
#pragma unroll
    for (int k = 0; k < NBS; ++k) {
      const int b0 = s0 + k * RB;
      const int rq = b0 + q;
      const bool valid = rq < rows && c < n;
      T v = vv[k];
      const uint32_t code = rq < rows ? codes[wave][rq] : 0u;
      if (code & 1u) v = -v;
      const uint32_t bkt = code >> 1;
      if constexpr (RB > 1) {
        // combine rows of this batch with the same bucket into the lowest such row, in row order
        bool same[RB];
        bool partner = false;
#pragma unroll
        for (int q2 = 0; q2 < RB; ++q2) {
          const int rq2 = b0 + q2;
          same[q2] = rq2 < rows && (codes[wave][rq2 < rows ? rq2 : 0] >> 1) == bkt;
          if (q2 != q && same[q2] && rq < rows) partner = true;
        }
        if (__ballot(partner) == 0) {
          // no two rows of the batch share a bucket (the common case): each row is its own
          // leader and its sum is the row itself, so the shuffles below would add nothing
          if (valid) mine[bkt * NPL + c] += v;
        } else {
          bool leader = rq < rows;
          T tot = v;
#pragma unroll
          for (int q2 = 0; q2 < RB; ++q2) {
            const T v2 = shfl_d(v, q2 * NPL + c);
            if (same[q2] && q2 < q) leader = false;
            if (same[q2] && q2 > q) tot += v2;
          }
          if (leader && c < n) mine[bkt * NPL + c] += tot;
        }
      } else {
        if (valid) mine[bkt * NPL + c] += v;
      }
      wave_lds_sync();
    }
    }
  }
  __syncthreads();
  // fixed-order sum of the four wave copies -> this workgroup's partial
  T* out = parts + (int64_t)blockIdx.x * s1 * n;
  for (int64_t i = threadIdx.x; i < s1 * n; i += blockDim.x) {
    const int64_t b = i / n, cc = i % n;
    const int64_t o = b * NPL + cc;
    out[i] = ((w1[0][o] + w1[1][o]) + w1[2][o]) + w1[3][o];
  }
}

template <int NPL, class T>
static void countsketch_lds_cap(int cap, dim3 grid, hipStream_t s, const double* V, int64_t ldv, int64_t m, int n, int64_t s1,
                                uint64_t seed, T* parts, const MemberStride& ms) {
  const dim3 block(256);
  if (cap == 1024)
    hipLaunchKernelGGL((countsketch_lds_kernel<NPL, T, 1024>), grid, block, 0, s, V, ldv, m, n, s1, seed, parts, ms);
  else if (cap == 2048)
    hipLaunchKernelGGL((countsketch_lds_kernel<NPL, T, 2048>), grid, block, 0, s, V, ldv, m, n, s1, seed, parts, ms);
  else
    hipLaunchKernelGGL((countsketch_lds_kernel<NPL, T, 4096>), grid, block, 0, s, V, ldv, m, n, s1, seed, parts, ms);
}

template <class T>
static hipError_t countsketch_lds_any(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, uint64_t seed, T* parts,
                                      int nparts, hipStream_t s, const MemberStride& ms) {
  if (!countsketch_lds_fits(s1, n) || nparts < 1 || ms.count < 1) return hipErrorInvalidValue;
  const dim3 grid(nparts, ms.count);
  const int cap = cs_cap(s1, n);
  switch (npl_of(n)) {
    case 8: countsketch_lds_cap<8, T>(cap, grid, s, V, ldv, m, n, s1, seed, parts, ms); break;
    case 16: countsketch_lds_cap<16, T>(cap, grid, s, V, ldv, m, n, s1, seed, parts, ms); break;
    case 32: countsketch_lds_cap<32, T>(cap, grid, s, V, ldv, m, n, s1, seed, parts, ms); break;
    case 64: countsketch_lds_cap<64, T>(cap, grid, s, V, ldv, m, n, s1, seed, parts, ms); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_countsketch_lds(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, uint64_t seed, double* parts,
                                  int nparts, hipStream_t s, const MemberStride& ms) {
  return countsketch_lds_any(V, ldv, m, n, s1, seed, parts, nparts, s, ms);
}

hipError_t launch_countsketch_lds(const double* V, int64_t ldv, int64_t m, int n, int64_t s1, uint64_t seed, float* parts,
                                  int nparts, hipStream_t s) {
  return countsketch_lds_any(V, ldv, m, n, s1, seed, parts, nparts, s, MemberStride());
}

// ------------------------------------------------------------------------------------------
// Gaussian sketch GEMM on the matrix cores, split over s1: Wpart[kc] = S2[:, chunk] W1[chunk, :],
// the partial products of the s1 chunks summed afterwards in a fixed order.  S2 tiles are drawn
// on the fly from the counter-based generator and never stored in HBM.  Wave w owns S2 rows
// 16w..16w+15 of the workgroup's 64-row block and every 16-column block of W.  Operand lanes:
// row/column = lane % 16, k group = lane / 16 (the same k order on both operands, so any k
// permutation inside the instruction cancels).
//   * single-precision sketch: S2 entries are the FP64 contract values rounded to FP32 (for the
//     BF16 variant both operands rounded on to BF16), v_mfma_f32_16x16x4f32 (8 per 32-wide k
//     step) or v_mfma_f32_16x16x32_bf16 (one per step), FP32 accumulation; result lane l,
//     element e: row 4 (l / 16) + e, column l % 16;
//   * FP64 sketch: v_mfma_f64_16x16x4f64, FP64 throughout; result lane l, element e: row
//     l / 16 + 4e, column l % 16.
// ------------------------------------------------------------------------------------------
constexpr int kGemmRows = 64;  // rows of S2 (and W) per workgroup
constexpr int kMmK = 32;  // k step of the matrix-core kernel

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int NP, bool BF16>
__global__ __launch_bounds__(256) void gauss_mfma_kernel(const float* __restrict__ W1, int n, int64_t s1, int64_t s2, uint64_t seed,
                                                         double scale, int64_t kc_len, float* __restrict__ wpart) {
  __shared__ float st[kGemmRows][kMmK + 1];  // S2 tile, [row j][k]
  __shared__ float wt[NP][kMmK + 1];         // W1 tile transposed, [column c][k]
  constexpr int NCB = NP / 16;
  const int t = threadIdx.x, wave = t / kWave, lane = lane_id();
  const int li = lane % 16, lq = lane / 16;
  const int64_t kc = blockIdx.x, rb = blockIdx.y;
  const int64_t k_beg = kc * kc_len;
  const int64_t k_end = k_beg + kc_len < s1 ? k_beg + kc_len : s1;
  f32x4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = k_beg; k0 < k_end; k0 += kMmK) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // 512 Philox blocks: (k, block of 4 rows)
      const int idx = t + 256 * h;
      const int kk = idx % kMmK, jb = idx / kMmK;  // jb in 0..15
      const int64_t k = k0 + kk;
      const int64_t jblk = rb * (kGemmRows / 4) + jb;
      double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
      if (k < k_end) {
        const Block4 y = philox4x64_10((uint64_t)k, (uint64_t)jblk, 0, kTagGaussian, seed, 0);
        box_muller(y.y0, y.y1, z0, z1);
        box_muller(y.y2, y.y3, z2, z3);
      }
      const int64_t j = 4 * jblk;
      const bool kin = k < k_end;
      st[4 * jb + 0][kk] = (kin && j + 0 < s2) ? (float)(z0 * scale) : 0.f;
      st[4 * jb + 1][kk] = (kin && j + 1 < s2) ? (float)(z1 * scale) : 0.f;
      st[4 * jb + 2][kk] = (kin && j + 2 < s2) ? (float)(z2 * scale) : 0.f;
      st[4 * jb + 3][kk] = (kin && j + 3 < s2) ? (float)(z3 * scale) : 0.f;
    }
    for (int i = t; i < kMmK * NP; i += 256) {
      const int kk = i / NP, c = i % NP;
      const int64_t k = k0 + kk;
      wt[c][kk] = (k < k_end && c < n) ? W1[k * n + c] : 0.f;
    }
    __syncthreads();
    const float* arow = st[16 * wave + li];
    if constexpr (BF16) {
      bf16x8 a;
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = (__bf16)arow[8 * lq + q];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float* brow = wt[16 * cb + li];
        bf16x8 b;
#pragma unroll
        for (int q = 0; q < 8; ++q) b[q] = (__bf16)brow[8 * lq + q];
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < kMmK / 4; ++ks) {
        const float a = arow[4 * ks + lq];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, wt[16 * cb + li][4 * ks + lq], acc[cb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int c = 16 * cb + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t j = rb * kGemmRows + 16 * wave + 4 * lq + e;
      if (j < s2 && c < n) wpart[(kc * s2 + j) * n + c] = acc[cb][e];
    }
  }
}

hipError_t launch_gauss_mfma(const float* W1, int n, int64_t s1, int64_t s2, uint64_t seed, double scale, int64_t kc_len,
                             int64_t nkc, bool bf16, float* wpart, hipStream_t s) {
  if (kc_len % kMmK != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nkc, (unsigned)((s2 + kGemmRows - 1) / kGemmRows)), block(256);
  const int np = n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 128;
#define RCQR_GAUSS_MFMA(NP_)                                                                                          \
  if (np == NP_) {                                                                                                    \
    if (bf16)                                                                                                         \
      hipLaunchKernelGGL((gauss_mfma_kernel<NP_, true>), grid, block, 0, s, W1, n, s1, s2, seed, scale, kc_len, wpart); \
    else                                                                                                              \
      hipLaunchKernelGGL((gauss_mfma_kernel<NP_, false>), grid, block, 0, s, W1, n, s1, s2, seed, scale, kc_len, wpart); \
  }
  RCQR_GAUSS_MFMA(16)
  RCQR_GAUSS_MFMA(32)
  RCQR_GAUSS_MFMA(64)
  RCQR_GAUSS_MFMA(128)
#undef RCQR_GAUSS_MFMA
  return hipGetLastError();
}

// FP64 product: 8 v_mfma_f64_16x16x4f64 per 32-wide k step and 16-column block.
template <int NP>
__global__ __launch_bounds__(256) void gauss_mfma64_kernel(const double* __restrict__ W1, int n, int64_t s1, int64_t s2, uint64_t seed,
                                                           double scale, int64_t kc_len, double* __restrict__ wpart, MemberStride ms) {
  {
    const int64_t mb = blockIdx.z;  // batch member
    W1 = member_ptr(W1, mb * ms.ws);
    wpart = member_ptr(wpart, mb * ms.ws);
    seed = member_seed(seed, ms, mb);
  }
  __shared__ double st[kGemmRows][kMmK + 1];  // S2 tile, [row j][k]
  __shared__ double wt[NP][kMmK + 1];         // W1 tile transposed, [column c][k]
  constexpr int NCB = NP / 16;
  const int t = threadIdx.x, wave = t / kWave, lane = lane_id();
  const int li = lane % 16, lq = lane / 16;
  const int64_t kc = blockIdx.x, rb = blockIdx.y;
  const int64_t k_beg = kc * kc_len;
  const int64_t k_end = k_beg + kc_len < s1 ? k_beg + kc_len : s1;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = k_beg; k0 < k_end; k0 += kMmK) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // 512 Philox blocks: (k, block of 4 rows)
      const int idx = t + 256 * h;
      const int kk = idx % kMmK, jb = idx / kMmK;
      const int64_t k = k0 + kk;
      const int64_t jblk = rb * (kGemmRows / 4) + jb;
      double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
      if (k < k_end) {
        const Block4 y = philox4x64_10((uint64_t)k, (uint64_t)jblk, 0, kTagGaussian, seed, 0);
        box_muller(y.y0, y.y1, z0, z1);
        box_muller(y.y2, y.y3, z2, z3);
      }
      const int64_t j = 4 * jblk;
      const bool kin = k < k_end;
      st[4 * jb + 0][kk] = (kin && j + 0 < s2) ? z0 * scale : 0.0;
      st[4 * jb + 1][kk] = (kin && j + 1 < s2) ? z1 * scale : 0.0;
      st[4 * jb + 2][kk] = (kin && j + 2 < s2) ? z2 * scale : 0.0;
      st[4 * jb + 3][kk] = (kin && j + 3 < s2) ? z3 * scale : 0.0;
    }
    for (int i = t; i < kMmK * NP; i += 256) {
      const int kk = i / NP, c = i % NP;
      const int64_t k = k0 + kk;
      wt[c][kk] = (k < k_end && c < n) ? W1[k * n + c] : 0.0;
    }
    __syncthreads();
    const double* arow = st[16 * wave + li];
#pragma unroll
    for (int ks = 0; ks < kMmK / 4; ++ks) {
      const double a = arow[4 * ks + lq];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, wt[16 * cb + li][4 * ks + lq], acc[cb], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int c = 16 * cb + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t j = rb * kGemmRows + 16 * wave + lq + 4 * e;
      if (j < s2 && c < n) wpart[(kc * s2 + j) * n + c] = acc[cb][e];
    }
  }
}

template <int NP>
static void launch_gauss64(dim3 grid, const double* W1, int n, int64_t s1, int64_t s2, uint64_t seed, double scale, int64_t kc_len,
                           double* wpart, hipStream_t s, const MemberStride& ms) {
  hipLaunchKernelGGL((gauss_mfma64_kernel<NP>), grid, dim3(256), 0, s, W1, n, s1, s2, seed, scale, kc_len, wpart, ms);
}

hipError_t launch_gauss_gemm(const double* W1, int n, int64_t s1, int64_t s2, uint64_t seed, double scale, int64_t kc_len,
                             int64_t nkc, double* wpart, hipStream_t s, const MemberStride& ms) {
  if (kc_len % kMmK != 0 || ms.count < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nkc, (unsigned)((s2 + kGemmRows - 1) / kGemmRows), ms.count);
  const int np = n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 128;
  if (np == 16) launch_gauss64<16>(grid, W1, n, s1, s2, seed, scale, kc_len, wpart, s, ms);
  else if (np == 32) launch_gauss64<32>(grid, W1, n, s1, s2, seed, scale, kc_len, wpart, s, ms);
  else if (np == 64) launch_gauss64<64>(grid, W1, n, s1, s2, seed, scale, kc_len, wpart, s, ms);
  else launch_gauss64<128>(grid, W1, n, s1, s2, seed, scale, kc_len, wpart, s, ms);
  return hipGetLastError();
}

// Widen an FP32 array to FP64 (inspection of the single-precision sketch's intermediates).
__global__ void widen_kernel(const float* __restrict__ in, int64_t count, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) out[i] = in[i];
}

hipError_t launch_widen(const float* in, int64_t count, double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, in, count, out);
  return hipGetLastError();
}

// Debug: a block of S2 entries.
__global__ void gaussian_block_kernel(int64_t j0, int64_t nj, int64_t k0, int64_t nk, uint64_t seed, double scale, double* out) {
  const int64_t total = nj * nk;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = j0 + i / nk, k = k0 + i % nk;
    const Block4 y = philox4x64_10((uint64_t)k, (uint64_t)(j >> 2), 0, kTagGaussian, seed, 0);
    double z0, z1;
    if ((j & 3) < 2)
      box_muller(y.y0, y.y1, z0, z1);
    else
      box_muller(y.y2, y.y3, z0, z1);
    out[i] = ((j & 1) ? z1 : z0) * scale;
  }
}

hipError_t launch_gaussian_block(int64_t j0, int64_t nj, int64_t k0, int64_t nk, uint64_t seed, double scale, double* out,
                                 hipStream_t s) {
  if (nj * nk <= 0) return hipSuccess;
  hipLaunchKernelGGL(gaussian_block_kernel, dim3(grid_for(nj * nk, 256)), dim3(256), 0, s, j0, nj, k0, nk, seed, scale, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Fixed-order sum of partials, compensated (Neumaier's variant of Kahan summation): the
// rounding error of each addition is recovered exactly (TwoSum) and added back at the end, so
// the result does not degrade with the number of partials.
// ------------------------------------------------------------------------------------------
// Workgroup: 16 consecutive outputs x 16 groups of parts.  Group g sums parts g, g + 16, g + 32, ...
// (compensated, increasing p); the 16 group sums are then combined in g order.  The partition
// depends only on nparts, so the order of every sum is fixed.
template <class T>
__global__ __launch_bounds__(256) void reduce_parts_kernel(const T* __restrict__ parts, int64_t nparts, int64_t stride, int64_t len,
                                                           T* __restrict__ out, MemberStride ms, int parts_kind) {
  constexpr int E = 16, G = 16;
  parts = member_ptr(parts, (int64_t)blockIdx.y * ms.ws);
  out = member_ptr(out, (int64_t)blockIdx.y * ms.ws);
  if (ms.info != nullptr && parts_kind != kPartsUniform) {  // ragged batch: the member's own partial count
    const MemberInfo& mi = member_info(ms, blockIdx.y);
    nparts = parts_kind == kPartsCountSketch ? mi.cs_parts : mi.gblocks;
  }
  __shared__ T ssum[G][E], scomp[G][E];
  const int e = threadIdx.x % E, g = threadIdx.x / E;
  const int64_t i = (int64_t)blockIdx.x * E + e;
  T sum = T(0), comp = T(0);
  if (i < len) {
    int64_t p = g;
    for (; p + 3 * G < nparts; p += 4 * G) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = parts[(p + u * G) * stride + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T t = sum + v[u];
        comp += (fabs(sum) >= fabs(v[u])) ? ((sum - t) + v[u]) : ((v[u] - t) + sum);
        sum = t;
      }
    }
    for (; p < nparts; p += G) {
      const T x = parts[p * stride + i];
      const T t = sum + x;
      comp += (fabs(sum) >= fabs(x)) ? ((sum - t) + x) : ((x - t) + sum);
      sum = t;
    }
  }
  ssum[g][e] = sum;
  scomp[g][e] = comp;
  __syncthreads();
  if (g == 0 && i < len) {
    T tot = ssum[0][e], c = scomp[0][e];
    for (int h = 1; h < G; ++h) {
      const T x = ssum[h][e];
      const T t = tot + x;
      c += (fabs(tot) >= fabs(x)) ? ((tot - t) + x) : ((x - t) + tot);
      c += scomp[h][e];
      tot = t;
    }
    out[i] = tot + c;
  }
}

hipError_t launch_reduce_parts(const double* parts, int64_t nparts, int64_t stride, int64_t len, double* out, hipStream_t s,
                               const MemberStride& ms, int parts_kind) {
  if (len <= 0 || ms.count < 1) return hipSuccess;
  hipLaunchKernelGGL(reduce_parts_kernel<double>, dim3((unsigned)((len + 15) / 16), ms.count), dim3(256), 0, s, parts, nparts, stride, len,
                     out, ms, parts_kind);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const float* parts, int64_t nparts, int64_t stride, int64_t len, float* out, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_parts_kernel<float>, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, s, parts, nparts, stride, len, out,
                     MemberStride(), (int)kPartsUniform);
  return hipGetLastError();
}

}  // namespace rcqr
