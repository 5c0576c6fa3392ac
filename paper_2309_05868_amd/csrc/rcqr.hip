// Host side of the rcqr C ABI: argument checks, workspace layout, and the order of the kernel
// launches of Algorithm 3 (rand_cholQR), Algorithm 4 (cholQR2) and shifted CholeskyQR3 on the
// plan's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/rcqr.h"
#include "launch.h"

using namespace rcqr;

namespace {

constexpr size_t kAlign = 256;
constexpr int kQrRows = 256;     // rows one Householder workgroup factors
constexpr int kMaxBatch = 4096;  // members of one rcqr_factor_batch call (a grid dimension)
constexpr int kPhases = 7;
constexpr int64_t kMaxRows = (int64_t)1 << 31;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int padded_cols(int64_t n) {
  int p = 16;
  while (p < n) p <<= 1;
  return p;
}

struct Layout {
  size_t info, minfo, w1, csparts, codes, counts, offsets, hist, entries, unsorted, wpart, w, qra, qrb, r0, r0pk, gpart, gplo, gc, g, r1, r1pk,
      ra, rapk, rtmp, rtmp2, rinv, total;
};

struct Shape {
  int64_t m, n, s1, s2;
  int np;
  bool lds_cs;
  int cs_parts;
  int nchunk;  // row chunks of the bucket index build
  int64_t kc_len, nkc;
  int64_t qr_blocks0;
};

Shape make_shape(int64_t m, int64_t n, int64_t s1, int64_t s2) {
  Shape sh{};
  sh.m = m;
  sh.n = n;
  sh.s1 = s1;
  sh.s2 = s2;
  sh.np = padded_cols(n);
  sh.lds_cs = countsketch_lds_fits(s1, (int)n);
  sh.cs_parts = sh.lds_cs ? countsketch_lds_parts(m, s1, (int)n) : 0;
  sh.nchunk = bucket_nchunk(m, s1);
  // Gaussian GEMM split over s1: about 512 workgroups (two per CU, so one workgroup's S2
  // generation overlaps another's products), partials capped at 48 MiB
  const int64_t nrb = (s2 + 63) / 64;
  int64_t nkc = 512 / nrb;
  const int64_t cap = (int64_t)(48u << 20) / (s2 * n * 8);
  if (nkc > cap) nkc = cap;
  if (nkc < 1) nkc = 1;
  const int64_t maxk = (s1 + 31) / 32;
  if (nkc > maxk) nkc = maxk;
  int64_t kc = (s1 + nkc - 1) / nkc;
  kc = (kc + 31) / 32 * 32;  // whole k steps of both GEMM kernels
  sh.kc_len = kc;
  sh.nkc = (s1 + kc - 1) / kc;
  sh.qr_blocks0 = (s2 + kQrRows - 1) / kQrRows;
  return sh;
}

Layout make_layout(const Shape& sh) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + (bytes ? bytes : 1));
    return at;
  };
  const size_t n = (size_t)sh.n, np = (size_t)sh.np;
  L.info = take(16 * sizeof(int32_t));
  L.minfo = take(sizeof(MemberInfo));  // a ragged batch's member description
  L.w1 = take((size_t)sh.s1 * n * 8);
  L.csparts = take(sh.lds_cs ? (size_t)sh.cs_parts * sh.s1 * n * 8 : 0);
  const size_t mm = sh.lds_cs ? 0 : (size_t)sh.m;
  const size_t ss = sh.lds_cs ? 0 : (size_t)sh.s1;
  L.codes = take(mm * 4);
  L.counts = take(ss * 4);
  L.offsets = take(sh.lds_cs ? 0 : (ss + 1) * 4);
  L.hist = take(sh.lds_cs ? 0 : (size_t)sh.nchunk * ss * 4);
  L.entries = take(mm * 4);
  L.unsorted = take(ss);
  L.wpart = take((size_t)sh.nkc * sh.s2 * n * 8);
  L.w = take((size_t)sh.s2 * n * 8);
  L.qra = take((size_t)sh.qr_blocks0 * n * n * 8);
  L.qrb = take((size_t)sh.qr_blocks0 * n * n * 8);
  const size_t pk = (size_t)packed_len((int)np) * 8;
  L.r0 = take(n * n * 8);
  L.r0pk = take(pk);
  L.gpart = take((size_t)kGramBlocks * gram_compact_len((int)np) * 8);
  L.gplo = take(np > 64 ? (size_t)kGramBlocks * gram_compact_len(64) * 8 : 0);  // Gram partials of columns 0..63
  L.gc = take((size_t)gram_compact_len((int)np) * 8);
  L.g = take(n * n * 8);
  L.r1 = take(n * n * 8);
  L.r1pk = take(pk);
  L.ra = take(n * n * 8);
  L.rapk = take(pk);
  L.rtmp = take(n * n * 8);
  L.rtmp2 = take(n * n * 8);
  L.rinv = take(np > 64 ? (size_t)36 * 256 * 8 : 0);  // upper blocks of R1^{-1}, 65..128 columns
  L.total = off;
  return L;
}

rcqr_status_t check_shape(int64_t m, int64_t n, int64_t s1, int64_t s2) {
  if (n < 1 || m < n || s2 < n || s1 < s2) return RCQR_E_INVALID;
  if (m >= kMaxRows || s1 >= kMaxRows) return RCQR_E_INVALID;
  if (n > RCQR_MAX_N) return RCQR_E_UNSUPPORTED;
  return RCQR_OK;
}

bool flags_valid(uint32_t flags) {
  const uint32_t known = RCQR_FLAG_SKETCH_FP32 | RCQR_FLAG_GEMM_BF16 | RCQR_FLAG_REORTH | RCQR_FLAG_SKETCH_AT_PLAN;
  if (flags & ~known) return false;
  if ((flags & RCQR_FLAG_GEMM_BF16) && !(flags & RCQR_FLAG_SKETCH_FP32)) return false;
  return true;
}

const char* const kPhaseNames[kPhases] = {"countsketch", "gaussian", "householder", "trsm_gram", "cholesky", "reorth", "final"};

}  // namespace

struct rcqr_plan_s {
  Shape sh;
  Layout L;
  uint64_t seed;
  uint32_t flags;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  // launch choices that never change results (set by rcqr_tune or rcqr_set_tuning)
  int final_mode;  // RCQR_FINAL_RECOMPUTE or RCQR_FINAL_MATERIALIZE
  int grid_mult;   // workgroups-per-CU cap of the multi-row passes
  // per-phase timing: a ring of `cap` steps, kPhases + 1 events each
  int cap;
  int recorded;
  hipEvent_t* ev;
  // host staging of a ragged batch's member descriptions (copied into the workspace slices)
  MemberInfo* staged;
  int32_t staged_cap;

  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

#define RCQR_TRY(expr)                       \
  do {                                       \
    if ((expr) != hipSuccess) return RCQR_E_HIP; \
  } while (0)

// Workspace of rcqr_factor_static: a file-scope device array, one copy per GPU.  Host code uses
// the per-device address from hipGetSymbolAddress, never the array's name (which on the host
// is only a handle for the symbol lookup).
constexpr size_t kScratchBytes = RCQR_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on the stream's device (looked up once per device, with
// that device current; the caller's current device is restored).
static rcqr_status_t scratch_address(hipStream_t stream, char** out) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return RCQR_E_HIP;
  int dev = cur;
  if (stream != nullptr) {
    hipDevice_t d = 0;
    if (hipStreamGetDevice(stream, &d) != hipSuccess) return RCQR_E_HIP;
    dev = (int)d;
  }
  if (dev < 0 || dev >= kMaxDevices) return RCQR_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return RCQR_E_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur && hipSetDevice(cur) != hipSuccess) return RCQR_E_HIP;
    if (e != hipSuccess || ptr == nullptr) return RCQR_E_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return RCQR_OK;
}

static rcqr_status_t mark(rcqr_plan_t p, int i) {
  if (p->cap > 0) {
    const int slot = p->recorded % p->cap;
    RCQR_TRY(hipEventRecord(p->ev[slot * (kPhases + 1) + i], p->stream));
  }
  return RCQR_OK;
}

static void free_events(rcqr_plan_t p) {
  if (p->ev) {
    for (int i = 0; i < p->cap * (kPhases + 1); ++i)
      if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    delete[] p->ev;
  }
  p->ev = nullptr;
  p->cap = 0;
  p->recorded = 0;
}

// R0 = Householder R of W (s2 x n): TSQR over 256-row blocks, then sign normalisation.
// R0 of W (element type T: FP64, or FP32 for the single-precision sketch, promoted to FP64 by
// the finalize step).
template <class T>
static rcqr_status_t run_householder(rcqr_plan_t p) {
  const Shape& sh = p->sh;
  const int n = (int)sh.n;
  hipStream_t s = p->stream;
  const T* in = p->at<T>(p->L.w);
  int64_t rows = sh.s2, rpb = kQrRows;
  T* bufs[2] = {p->at<T>(p->L.qra), p->at<T>(p->L.qrb)};
  int which = 0;
  for (;;) {
    const int64_t nblocks = (rows + rpb - 1) / rpb;
    if (nblocks == 1) {  // the last level writes R0, its packed form and the rank status itself
      RCQR_TRY(launch_qr_blocks(in, n, rows, rpb, n, bufs[which], 1, s, MemberStride(), p->at<double>(p->L.r0),
                                p->at<double>(p->L.r0pk), p->at<int32_t>(p->L.info), sh.np));
      break;
    }
    RCQR_TRY(launch_qr_blocks(in, n, rows, rpb, n, bufs[which], (int)nblocks, s));
    in = bufs[which];
    which ^= 1;
    rows = nblocks * n;
    rpb = (kQrRows / n) * n;
  }
  return RCQR_OK;
}

// The CountSketch S1 (Section 3) as a bucket index: each row's bucket and sign, then the rows of
// every bucket listed in ascending order.  A function of (m, s1, seed) only.
static rcqr_status_t build_bucket_index(rcqr_plan_t p) {
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  hipStream_t s = p->stream;
  uint32_t* counts = p->at<uint32_t>(L.counts);
  uint32_t* offsets = p->at<uint32_t>(L.offsets);
  uint32_t* hist = p->at<uint32_t>(L.hist);
  uint32_t* codes = p->at<uint32_t>(L.codes);
  uint32_t* entries = p->at<uint32_t>(L.entries);
  uint8_t* unsorted = p->at<uint8_t>(L.unsorted);
  RCQR_TRY(launch_hash_hist(sh.m, sh.s1, p->seed, sh.nchunk, codes, hist, s));
  RCQR_TRY(launch_hist_colscan(sh.nchunk, sh.s1, hist, counts, unsorted, s));
  RCQR_TRY(launch_bucket_scan(counts, sh.s1, offsets, nullptr, s));
  RCQR_TRY(launch_bucket_scatter(sh.m, sh.s1, sh.nchunk, codes, offsets, hist, entries, unsorted, s));
  return RCQR_OK;
}

// Algorithm 1, step 1: W1 = S1 V, then W = S2 W1, in FP64 or (single-precision sketch) FP32.
template <class T>
static rcqr_status_t run_sketch(rcqr_plan_t p, const double* V, int64_t ldv) {
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  const int n = (int)sh.n;
  hipStream_t s = p->stream;
  T* W1 = p->at<T>(L.w1);
  if (sh.lds_cs) {
    T* parts = p->at<T>(L.csparts);
    RCQR_TRY(launch_countsketch_lds(V, ldv, sh.m, n, sh.s1, p->seed, parts, sh.cs_parts, s));
    RCQR_TRY(launch_reduce_parts(parts, sh.cs_parts, sh.s1 * sh.n, sh.s1 * sh.n, W1, s));
  } else {
    if (!(p->flags & RCQR_FLAG_SKETCH_AT_PLAN) && build_bucket_index(p) != RCQR_OK) return RCQR_E_HIP;
    const uint8_t* unsorted = p->at<uint8_t>(L.unsorted);
    RCQR_TRY(launch_bucket_gather(V, ldv, sh.m, n, sh.s1, p->at<uint32_t>(L.offsets), p->at<uint32_t>(L.entries),
                                  bucket_scatter_sorts(sh.s1) ? unsorted : nullptr, W1, s));
  }
  if (mark(p, 1) != RCQR_OK) return RCQR_E_HIP;
  const double scale = 1.0 / std::sqrt((double)sh.s2);
  T* wpart = p->at<T>(L.wpart);
  if constexpr (sizeof(T) == 8) {
    RCQR_TRY(launch_gauss_gemm(W1, n, sh.s1, sh.s2, p->seed, scale, sh.kc_len, sh.nkc, wpart, s));
  } else {
    const bool bf16 = (p->flags & RCQR_FLAG_GEMM_BF16) != 0;
    RCQR_TRY(launch_gauss_mfma(W1, n, sh.s1, sh.s2, p->seed, scale, sh.kc_len, sh.nkc, bf16, wpart, s));
  }
  RCQR_TRY(launch_reduce_parts(wpart, sh.nkc, sh.s2 * sh.n, sh.s2 * sh.n, p->at<T>(L.w), s));
  return RCQR_OK;
}

// G = (V Rp^{-1})^T (V Rp^{-1}) into the compact buffer.  Up to 64 columns Q0 is never stored
// (the final pass recomputes it); for 65..128 columns Q0 is written into Q and read back.
static rcqr_status_t run_gram(rcqr_plan_t p, const double* V, int64_t ldv, const double* rpk, double* Q, int64_t ldq,
                              bool store_q0 = false) {
  const Shape& sh = p->sh;
  const int len = gram_compact_len(sh.np);
  const int32_t* info = p->at<int32_t>(p->L.info);
  if (sh.np <= 64) {
    RCQR_TRY(launch_trsm_gram(sh.np, V, sh.m, (int)sh.n, ldv, rpk, info, p->at<double>(p->L.gpart), store_q0 ? Q : nullptr,
                              store_q0 ? ldq : 0, p->stream));
  } else {
    RCQR_TRY(launch_solve128_gram(V, sh.m, (int)sh.n, ldv, rpk, info, Q, ldq, p->at<double>(p->L.gplo), p->stream, p->grid_mult));
    RCQR_TRY(launch_syrk128(Q, sh.m, (int)sh.n, ldq, info, p->at<double>(p->L.gpart), p->at<double>(p->L.gplo), gram_blocks(sh.m),
                            p->stream));
  }
  const int nparts = sh.np <= 64 ? gram_blocks(sh.m) : kGramBlocks;  // the 65-128-column Gram keeps the full grid
  RCQR_TRY(launch_reduce_parts(p->at<double>(p->L.gpart), nparts, len, len, p->at<double>(p->L.gc), p->stream));
  return RCQR_OK;
}

// Q = (V R0^{-1}) R1^{-1}: recomputed from V up to 64 columns, from the stored Q0 (in Q) above.
static rcqr_status_t run_final(rcqr_plan_t p, const double* V, int64_t ldv, const double* r0pk, const double* r1pk, double* Q,
                               int64_t ldq) {
  const Shape& sh = p->sh;
  const int32_t* info = p->at<int32_t>(p->L.info);
  if (sh.np <= 64) {
    RCQR_TRY(launch_final(sh.np, true, V, sh.m, (int)sh.n, ldv, r0pk, r1pk, info, Q, ldq, p->stream, p->grid_mult));
  } else {
    RCQR_TRY(launch_rinv128(r1pk, info, p->at<double>(p->L.rinv), p->stream));
    RCQR_TRY(launch_apply_rinv128(Q, sh.m, (int)sh.n, ldq, p->at<double>(p->L.rinv), info, p->grid_mult, p->stream));
  }
  return RCQR_OK;
}

// X R^{-1} written to Q (one row-wise substitution; Q may alias X).
static rcqr_status_t run_solve(rcqr_plan_t p, const double* X, int64_t ldx, const double* rpk, double* Q, int64_t ldq) {
  const Shape& sh = p->sh;
  const int32_t* info = p->at<int32_t>(p->L.info);
  if (sh.np <= 64) {
    RCQR_TRY(launch_final(sh.np, false, X, sh.m, (int)sh.n, ldx, rpk, rpk, info, Q, ldq, p->stream));
  } else {
    RCQR_TRY(launch_solve128(X, sh.m, (int)sh.n, ldx, rpk, info, Q, ldq, p->stream));
  }
  return RCQR_OK;
}

extern "C" {

size_t rcqr_workspace_bytes(int64_t m, int64_t n, int64_t s1, int64_t s2, uint32_t flags) {
  if (check_shape(m, n, s1, s2) != RCQR_OK || !flags_valid(flags)) return 0;
  return make_layout(make_shape(m, n, s1, s2)).total;
}

rcqr_status_t rcqr_plan(rcqr_plan_t* plan, int64_t m, int64_t n, int64_t s1, int64_t s2, uint64_t seed, uint32_t flags,
                        void* d_workspace, size_t workspace_bytes, void* stream) {
  if (plan == nullptr) return RCQR_E_INVALID;
  *plan = nullptr;
  const rcqr_status_t st = check_shape(m, n, s1, s2);
  if (st != RCQR_OK) return st;
  if (!flags_valid(flags)) return RCQR_E_INVALID;
  const Shape sh = make_shape(m, n, s1, s2);
  const Layout L = make_layout(sh);
  if (d_workspace == nullptr || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
    return RCQR_E_INVALID;
  rcqr_plan_s* p = new (std::nothrow) rcqr_plan_s();
  if (p == nullptr) return RCQR_E_NOMEM;
  p->sh = sh;
  p->L = L;
  p->seed = seed;
  p->flags = flags;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->ws = reinterpret_cast<char*>(d_workspace);
  p->ws_bytes = workspace_bytes;
  p->final_mode = RCQR_FINAL_RECOMPUTE;
  p->grid_mult = 2;
  p->cap = 0;
  p->recorded = 0;
  p->ev = nullptr;
  p->staged = nullptr;
  p->staged_cap = 0;
  if ((flags & RCQR_FLAG_SKETCH_AT_PLAN) && !sh.lds_cs && build_bucket_index(p) != RCQR_OK) {
    delete p;
    return RCQR_E_HIP;
  }
  *plan = p;
  return RCQR_OK;
}

rcqr_status_t rcqr_destroy(rcqr_plan_t p) {
  if (p == nullptr) return RCQR_E_INVALID;
  free_events(p);
  delete[] p->staged;
  delete p;
  return RCQR_OK;
}

rcqr_status_t rcqr_set_timing(rcqr_plan_t p, int32_t steps) {
  if (p == nullptr || steps < 0 || steps > 4096) return RCQR_E_INVALID;
  free_events(p);
  if (steps == 0) return RCQR_OK;
  p->ev = new (std::nothrow) hipEvent_t[(size_t)steps * (kPhases + 1)]();
  if (p->ev == nullptr) return RCQR_E_NOMEM;
  p->cap = steps;
  for (int i = 0; i < steps * (kPhases + 1); ++i) {
    if (hipEventCreate(&p->ev[i]) != hipSuccess) {
      free_events(p);
      return RCQR_E_HIP;
    }
  }
  return RCQR_OK;
}

rcqr_status_t rcqr_phase_times(rcqr_plan_t p, float* ms, int32_t max, int32_t* count) {
  if (p == nullptr || count == nullptr || (ms == nullptr && max > 0)) return RCQR_E_INVALID;
  *count = 0;
  if (p->cap == 0 || p->recorded == 0) return RCQR_E_INVALID;
  RCQR_TRY(hipStreamSynchronize(p->stream));
  const int steps = p->recorded < p->cap ? p->recorded : p->cap;
  const int k = max < kPhases ? max : kPhases;
  for (int i = 0; i < k; ++i) {
    double sum = 0.0;
    for (int st = 0; st < steps; ++st) {
      float t = 0.f;
      RCQR_TRY(hipEventElapsedTime(&t, p->ev[st * (kPhases + 1) + i], p->ev[st * (kPhases + 1) + i + 1]));
      sum += t;
    }
    ms[i] = (float)(sum / steps);
  }
  *count = kPhases;
  p->recorded = 0;
  return RCQR_OK;
}

const char* rcqr_phase_name(int32_t phase) { return (phase >= 0 && phase < kPhases) ? kPhaseNames[phase] : "?"; }

const char* rcqr_status_string(int32_t status) {
  switch (status) {
    case RCQR_OK: return "ok";
    case RCQR_E_INVALID: return "invalid argument";
    case RCQR_E_UNSUPPORTED: return "unsupported shape";
    case RCQR_E_NOMEM: return "out of host memory";
    case RCQR_E_HIP: return "HIP runtime error";
    case RCQR_E_RANK: return "sketch R0 has a zero or non-finite diagonal entry";
    case RCQR_E_CHOL: return "Cholesky of the Gram matrix met a non-positive pivot";
    case RCQR_E_SCRATCH: return "workspace of the shape exceeds the static scratch of rcqr_factor_static";
    default: return "unknown status";
  }
}

static rcqr_status_t check_io(rcqr_plan_t p, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr) {
  if (p == nullptr || V == nullptr || Q == nullptr || R == nullptr) return RCQR_E_INVALID;
  if (ldv < p->sh.n || ldq < p->sh.n || ldr < p->sh.n) return RCQR_E_INVALID;
  if ((const void*)Q == (const void*)V && ldq != ldv) return RCQR_E_INVALID;
  return RCQR_OK;
}

rcqr_status_t rcqr_factor(rcqr_plan_t p, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr) {
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  // 65..128 columns store Q0 in Q; the second Cholesky QR reads V again, so V must survive
  if ((p->flags & RCQR_FLAG_REORTH) && p->sh.np > 64 && (const void*)Q == (const void*)V) return RCQR_E_INVALID;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  const int n = (int)sh.n;
  hipStream_t s = p->stream;
  int32_t* info = p->at<int32_t>(L.info);
  double* W1 = p->at<double>(L.w1);

  RCQR_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(info), 16, 0u, s));
  if (mark(p, 0) != RCQR_OK) return RCQR_E_HIP;
  const bool fp32 = (p->flags & RCQR_FLAG_SKETCH_FP32) != 0;
  const bool reorth = (p->flags & RCQR_FLAG_REORTH) != 0;
  // Algorithm 1, step 1: W1 = S1 V, W = S2 W1
  if ((fp32 ? run_sketch<float>(p, V, ldv) : run_sketch<double>(p, V, ldv)) != RCQR_OK) return RCQR_E_HIP;
  if (mark(p, 2) != RCQR_OK) return RCQR_E_HIP;
  // Algorithm 1, step 2: R0 = hhqr(W)
  if ((fp32 ? run_householder<float>(p) : run_householder<double>(p)) != RCQR_OK) return RCQR_E_HIP;
  if (mark(p, 3) != RCQR_OK) return RCQR_E_HIP;
  // Algorithm 1, step 3 + Algorithm 2, step 1: Q0 = V R0^{-1}, G = Q0^T Q0 (Q0 stored in Q when
  // materialising: the same rows the final pass would recompute)
  const bool mat = p->final_mode == RCQR_FINAL_MATERIALIZE && sh.np <= 64 && !reorth;
  if (run_gram(p, V, ldv, p->at<double>(L.r0pk), Q, ldq, mat) != RCQR_OK) return RCQR_E_HIP;
  if (mark(p, 4) != RCQR_OK) return RCQR_E_HIP;
  // Algorithm 2, step 2 and Algorithm 3, step 3: R1 = chol(G), R = R1 R0
  double* r_first = reorth ? p->at<double>(L.rtmp) : R;
  const int64_t ld_first = reorth ? n : ldr;
  RCQR_TRY(launch_cholesky(p->at<double>(L.gc), n, sh.np, p->at<double>(L.r0), 0.0, info, p->at<double>(L.g),
                           p->at<double>(L.r1), p->at<double>(L.r1pk), r_first, ld_first, s));
  if (mark(p, 5) != RCQR_OK) return RCQR_E_HIP;
  const double* first_pk = p->at<double>(L.r0pk);
  if (reorth) {
    // one more Cholesky QR: Q1 = V Rc^{-1} with Rc = R1 R0, R2 = chol(Q1^T Q1), R = R2 Rc
    RCQR_TRY(launch_finalize_r0(p->at<double>(L.rtmp), n, sh.np, info, p->at<double>(L.ra), p->at<double>(L.rapk), s));
    if (run_gram(p, V, ldv, p->at<double>(L.rapk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
    RCQR_TRY(launch_cholesky(p->at<double>(L.gc), n, sh.np, p->at<double>(L.ra), 0.0, info, p->at<double>(L.g),
                             p->at<double>(L.r1), p->at<double>(L.r1pk), R, ldr, s));
    first_pk = p->at<double>(L.rapk);
  }
  if (mark(p, 6) != RCQR_OK) return RCQR_E_HIP;
  // Algorithm 2, step 3 on Q0 (or Q1): Q = Q0 R1^{-1}
  if (mat) {
    RCQR_TRY(launch_apply_rinv(sh.np, Q, sh.m, n, ldq, p->at<double>(L.r1pk), info, p->grid_mult, s));
  } else if (run_final(p, V, ldv, first_pk, p->at<double>(L.r1pk), Q, ldq) != RCQR_OK) {
    return RCQR_E_HIP;
  }
  if (mark(p, 7) != RCQR_OK) return RCQR_E_HIP;
  if (p->cap > 0) ++p->recorded;
  return RCQR_OK;
}

// Algorithm 3 on a batch (every kernel launched once for all members; see MemberStride): the
// steps of rcqr_factor in FP64, members of the plan's n, s1 and s2.
static rcqr_status_t run_batch(rcqr_plan_t p, const MemberStride& ms, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R,
                               int64_t ldr) {
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  const int n = (int)sh.n;
  const int count = ms.count;
  hipStream_t s = p->stream;
  int32_t* info = p->at<int32_t>(L.info);
  RCQR_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(info), 16, 0u, s, count, ms.ws / 4));
  // Algorithm 1, step 1: W1 = S1 V, W = S2 W1
  if (sh.lds_cs) {
    RCQR_TRY(launch_countsketch_lds(V, ldv, sh.m, n, sh.s1, p->seed, p->at<double>(L.csparts), sh.cs_parts, s, ms));
    RCQR_TRY(launch_reduce_parts(p->at<double>(L.csparts), sh.cs_parts, sh.s1 * sh.n, sh.s1 * sh.n, p->at<double>(L.w1), s, ms,
                                 kPartsCountSketch));
  } else {
    uint32_t* counts = p->at<uint32_t>(L.counts);
    uint32_t* offsets = p->at<uint32_t>(L.offsets);
    uint32_t* hist = p->at<uint32_t>(L.hist);
    uint32_t* codes = p->at<uint32_t>(L.codes);
    uint32_t* entries = p->at<uint32_t>(L.entries);
    uint8_t* unsorted = p->at<uint8_t>(L.unsorted);
    RCQR_TRY(launch_hash_hist(sh.m, sh.s1, p->seed, sh.nchunk, codes, hist, s, ms));
    RCQR_TRY(launch_hist_colscan(sh.nchunk, sh.s1, hist, counts, unsorted, s, ms));
    RCQR_TRY(launch_bucket_scan(counts, sh.s1, offsets, nullptr, s, ms));
    RCQR_TRY(launch_bucket_scatter(sh.m, sh.s1, sh.nchunk, codes, offsets, hist, entries, unsorted, s, ms));
    RCQR_TRY(launch_bucket_gather(V, ldv, sh.m, n, sh.s1, offsets, entries, bucket_scatter_sorts(sh.s1) ? unsorted : nullptr,
                                  p->at<double>(L.w1), s, ms));
  }
  const double scale = 1.0 / std::sqrt((double)sh.s2);
  RCQR_TRY(launch_gauss_gemm(p->at<double>(L.w1), n, sh.s1, sh.s2, p->seed, scale, sh.kc_len, sh.nkc, p->at<double>(L.wpart), s, ms));
  RCQR_TRY(launch_reduce_parts(p->at<double>(L.wpart), sh.nkc, sh.s2 * sh.n, sh.s2 * sh.n, p->at<double>(L.w), s, ms));
  // Algorithm 1, step 2: R0 = hhqr(W), the TSQR levels of run_householder
  {
    const double* in = p->at<double>(L.w);
    int64_t rows = sh.s2, rpb = kQrRows;
    double* bufs[2] = {p->at<double>(L.qra), p->at<double>(L.qrb)};
    int which = 0;
    for (;;) {
      const int64_t nblocks = (rows + rpb - 1) / rpb;
      if (nblocks == 1) {  // the last level writes R0, its packed form and the rank status itself
        RCQR_TRY(launch_qr_blocks(in, n, rows, rpb, n, bufs[which], 1, s, ms, p->at<double>(L.r0), p->at<double>(L.r0pk), info,
                                  sh.np));
        break;
      }
      RCQR_TRY(launch_qr_blocks(in, n, rows, rpb, n, bufs[which], (int)nblocks, s, ms));
      in = bufs[which];
      which ^= 1;
      rows = nblocks * n;
      rpb = (kQrRows / n) * n;
    }
  }
  // Algorithm 1, step 3 + Algorithm 2, step 1: G = Q0^T Q0 (Q0 stored in Q above 64 columns)
  const int64_t len = gram_compact_len(sh.np);
  if (sh.np <= 64) {
    RCQR_TRY(launch_trsm_gram(sh.np, V, sh.m, n, ldv, p->at<double>(L.r0pk), info, p->at<double>(L.gpart), nullptr, ldq, s, ms));
    RCQR_TRY(launch_reduce_parts(p->at<double>(L.gpart), gram_blocks(sh.m), len, len, p->at<double>(L.gc), s, ms, kPartsGram));
  } else {
    RCQR_TRY(launch_solve128_gram(V, sh.m, n, ldv, p->at<double>(L.r0pk), info, Q, ldq, p->at<double>(L.gplo), s, p->grid_mult, ms));
    RCQR_TRY(launch_syrk128(Q, sh.m, n, ldq, info, p->at<double>(L.gpart), p->at<double>(L.gplo), gram_blocks(sh.m), s, ms));
    RCQR_TRY(launch_reduce_parts(p->at<double>(L.gpart), kGramBlocks, len, len, p->at<double>(L.gc), s, ms));
  }
  // Algorithm 2, step 2 and Algorithm 3, step 3: R1 = chol(G), R = R1 R0
  RCQR_TRY(launch_cholesky(p->at<double>(L.gc), n, sh.np, p->at<double>(L.r0), 0.0, info, p->at<double>(L.g), p->at<double>(L.r1),
                           p->at<double>(L.r1pk), R, ldr, s, ms));
  // Algorithm 2, step 3 on Q0: Q = Q0 R1^{-1}
  if (sh.np <= 64) {
    RCQR_TRY(launch_final(sh.np, true, V, sh.m, n, ldv, p->at<double>(L.r0pk), p->at<double>(L.r1pk), info, Q, ldq, s, p->grid_mult, ms));
  } else {
    RCQR_TRY(launch_rinv128(p->at<double>(L.r1pk), info, p->at<double>(L.rinv), s, ms));
    RCQR_TRY(launch_apply_rinv128(Q, sh.m, n, ldq, p->at<double>(L.rinv), info, p->grid_mult, s, ms));
  }
  return RCQR_OK;
}

rcqr_status_t rcqr_factor_batch(rcqr_plan_t p, int32_t count, const double* V, int64_t ldv, int64_t sv, double* Q, int64_t ldq,
                                int64_t sq, double* R, int64_t ldr, int64_t sr, const uint64_t* d_seeds) {
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  if (count < 1 || (size_t)count > p->ws_bytes / L.total) return RCQR_E_INVALID;
  // members must not overlap (Q may be V itself, member by member)
  if (sv < sh.m * ldv || sq < sh.m * ldq || sr < sh.n * ldr) return RCQR_E_INVALID;
  if ((const void*)Q == (const void*)V && sq != sv) return RCQR_E_INVALID;
  if (p->flags != 0 || count > kMaxBatch) return RCQR_E_UNSUPPORTED;
  MemberStride ms;
  ms.ws = (int64_t)L.total;
  ms.v = sv;
  ms.q = sq;
  ms.r = sr;
  ms.count = count;
  ms.seeds = d_seeds;
  return run_batch(p, ms, V, ldv, Q, ldq, R, ldr);
}

static bool rows_aligned(const void* a, int64_t ld) { return (reinterpret_cast<uintptr_t>(a) % 16 == 0) && (ld % 2 == 0); }

rcqr_status_t rcqr_factor_ragged(rcqr_plan_t p, int32_t count, const rcqr_member_t* members) {
  if (p == nullptr || members == nullptr || count < 1) return RCQR_E_INVALID;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  if ((size_t)count > p->ws_bytes / L.total) return RCQR_E_INVALID;
  if (p->flags != 0 || count > kMaxBatch) return RCQR_E_UNSUPPORTED;
  if (p->staged_cap < count) {
    MemberInfo* fresh = new (std::nothrow) MemberInfo[count];
    if (fresh == nullptr) return RCQR_E_NOMEM;
    delete[] p->staged;
    p->staged = fresh;
    p->staged_cap = count;
  }
  bool aligned = true;
  for (int32_t b = 0; b < count; ++b) {
    const rcqr_member_t& r = members[b];
    if (r.V == nullptr || r.Q == nullptr || r.R == nullptr || r.m < sh.n || r.m > sh.m) return RCQR_E_INVALID;
    if (r.ldv < sh.n || r.ldq < sh.n || r.ldr < sh.n) return RCQR_E_INVALID;
    if ((const void*)r.Q == (const void*)r.V && r.ldq != r.ldv) return RCQR_E_INVALID;
    MemberInfo& mi = p->staged[b];
    mi.V = r.V;
    mi.Q = r.Q;
    mi.R = r.R;
    mi.m = r.m;
    mi.ldv = r.ldv;
    mi.ldq = r.ldq;
    mi.ldr = r.ldr;
    mi.seed = r.seed;
    mi.nchunk = bucket_nchunk(r.m, sh.s1);
    mi.chunk_rows = bucket_chunk_rows(r.m, mi.nchunk);
    mi.cs_parts = sh.lds_cs ? countsketch_lds_parts(r.m, sh.s1, (int)sh.n) : 0;
    mi.gblocks = gram_blocks(r.m);
    mi.pad = 0;
    aligned = aligned && rows_aligned(r.V, r.ldv) && rows_aligned(r.Q, r.ldq);
  }
  // the member descriptions into their workspace slices (one strided copy), then the batch
  RCQR_TRY(hipMemcpy2DAsync(p->ws + L.minfo, L.total, p->staged, sizeof(MemberInfo), sizeof(MemberInfo), (size_t)count,
                            hipMemcpyHostToDevice, p->stream));
  MemberStride ms;
  ms.ws = (int64_t)L.total;
  ms.count = count;
  ms.info = p->at<MemberInfo>(L.minfo);
  ms.aligned = aligned;
  // V, Q, R below only size the launches (every kernel takes its member's from the table)
  return run_batch(p, ms, members[0].V, members[0].ldv, members[0].Q, members[0].ldq, members[0].R, members[0].ldr);
}

rcqr_status_t rcqr_info_member(rcqr_plan_t p, int32_t member, int32_t* status, int32_t* column) {
  if (p == nullptr || status == nullptr || column == nullptr || member < 0 || (size_t)member >= p->ws_bytes / p->L.total)
    return RCQR_E_INVALID;
  int32_t h[2] = {0, 0};
  RCQR_TRY(hipMemcpyAsync(h, p->ws + (size_t)member * p->L.total + p->L.info, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  RCQR_TRY(hipStreamSynchronize(p->stream));
  *status = h[0];
  *column = h[1];
  return RCQR_OK;
}

rcqr_status_t rcqr_info_batch(rcqr_plan_t p, int32_t count, int32_t* status, int32_t* column) {
  if (p == nullptr || status == nullptr || column == nullptr || count < 1 || (size_t)count > p->ws_bytes / p->L.total)
    return RCQR_E_INVALID;
  int32_t* h = new (std::nothrow) int32_t[2 * (size_t)count];
  if (h == nullptr) return RCQR_E_NOMEM;
  // one strided copy: the first two words of every member's status block
  const hipError_t e = hipMemcpy2DAsync(h, 2 * sizeof(int32_t), p->ws + p->L.info, p->L.total, 2 * sizeof(int32_t), (size_t)count,
                                        hipMemcpyDeviceToHost, p->stream);
  const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(p->stream) : e;
  if (e2 == hipSuccess) {
    for (int32_t b = 0; b < count; ++b) {
      status[b] = h[2 * b];
      column[b] = h[2 * b + 1];
    }
  }
  delete[] h;
  return e2 == hipSuccess ? RCQR_OK : RCQR_E_HIP;
}

rcqr_status_t rcqr_cholqr2(rcqr_plan_t p, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr) {
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  const int n = (int)sh.n;
  hipStream_t s = p->stream;
  int32_t* info = p->at<int32_t>(L.info);
  RCQR_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(info), 16, 0u, s));
  // first cholQR: G = V^T V (R0 := I), Ra = chol(G)
  RCQR_TRY(launch_identity_factor(n, sh.np, p->at<double>(L.r0), p->at<double>(L.r0pk), s));
  if (run_gram(p, V, ldv, p->at<double>(L.r0pk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  RCQR_TRY(launch_cholesky(p->at<double>(L.gc), n, sh.np, p->at<double>(L.r0), 0.0, info, p->at<double>(L.g),
                           p->at<double>(L.ra), p->at<double>(L.rapk), p->at<double>(L.rtmp), n, s));
  // second cholQR on Q0 = V Ra^{-1}: Rb = chol(Q0^T Q0), R = Rb Ra
  if (run_gram(p, V, ldv, p->at<double>(L.rapk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  RCQR_TRY(launch_cholesky(p->at<double>(L.gc), n, sh.np, p->at<double>(L.rtmp), 0.0, info, p->at<double>(L.g),
                           p->at<double>(L.r1), p->at<double>(L.r1pk), R, ldr, s));
  if (run_final(p, V, ldv, p->at<double>(L.rapk), p->at<double>(L.r1pk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  return RCQR_OK;
}

rcqr_status_t rcqr_scholqr3(rcqr_plan_t p, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr) {
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  const int n = (int)sh.n;
  hipStream_t s = p->stream;
  int32_t* info = p->at<int32_t>(L.info);
  double* gc = p->at<double>(L.gc);
  double* g = p->at<double>(L.g);
  const double u = std::ldexp(1.0, -52);
  const double coef = 11.0 * ((double)sh.m * (double)sh.n + (double)sh.n * (double)(sh.n + 1)) * u;
  RCQR_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(info), 16, 0u, s));
  RCQR_TRY(launch_identity_factor(n, sh.np, p->at<double>(L.r0), p->at<double>(L.r0pk), s));
  // shifted cholQR: Ra = chol(V^T V + s I), s = coef ||V||_F^2; Qa = V Ra^{-1} stored in Q
  if (run_gram(p, V, ldv, p->at<double>(L.r0pk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  RCQR_TRY(launch_cholesky(gc, n, sh.np, p->at<double>(L.r0), coef, info, g, p->at<double>(L.ra), p->at<double>(L.rapk),
                           p->at<double>(L.rtmp), n, s));
  if (run_solve(p, V, ldv, p->at<double>(L.rapk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  // cholQR2 of Qa in place: Rb = chol(Qa^T Qa), Rc = chol((Qa Rb^{-1})^T (Qa Rb^{-1})), R = Rc Rb Ra
  if (run_gram(p, Q, ldq, p->at<double>(L.r0pk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  RCQR_TRY(launch_cholesky(gc, n, sh.np, p->at<double>(L.rtmp), 0.0, info, g, p->at<double>(L.r1), p->at<double>(L.r1pk),
                           p->at<double>(L.rtmp2), n, s));
  if (run_gram(p, Q, ldq, p->at<double>(L.r1pk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  RCQR_TRY(launch_cholesky(gc, n, sh.np, p->at<double>(L.rtmp2), 0.0, info, g, p->at<double>(L.ra), p->at<double>(L.rapk), R,
                           ldr, s));
  if (run_final(p, Q, ldq, p->at<double>(L.r1pk), p->at<double>(L.rapk), Q, ldq) != RCQR_OK) return RCQR_E_HIP;
  return RCQR_OK;
}

rcqr_status_t rcqr_info(rcqr_plan_t p, int32_t* status, int32_t* column) {
  if (p == nullptr || status == nullptr || column == nullptr) return RCQR_E_INVALID;
  int32_t h[2] = {0, 0};
  RCQR_TRY(hipMemcpyAsync(h, p->at<int32_t>(p->L.info), sizeof(h), hipMemcpyDeviceToHost, p->stream));
  RCQR_TRY(hipStreamSynchronize(p->stream));
  *status = h[0];
  *column = h[1];
  return RCQR_OK;
}

rcqr_status_t rcqr_sketch_hash(rcqr_plan_t p, int64_t row0, int64_t count, int32_t* d_bucket, int8_t* d_sign) {
  if (p == nullptr || row0 < 0 || count < 0 || row0 + count > kMaxRows || (count > 0 && (!d_bucket || !d_sign)))
    return RCQR_E_INVALID;
  RCQR_TRY(launch_hash_debug(row0, count, p->sh.s1, p->seed, d_bucket, d_sign, p->stream));
  return RCQR_OK;
}

rcqr_status_t rcqr_gaussian_block(rcqr_plan_t p, int64_t j0, int64_t nj, int64_t k0, int64_t nk, double* d_out) {
  if (p == nullptr || j0 < 0 || nj < 0 || k0 < 0 || nk < 0 || (nj * nk > 0 && d_out == nullptr)) return RCQR_E_INVALID;
  const double scale = 1.0 / std::sqrt((double)p->sh.s2);
  RCQR_TRY(launch_gaussian_block(j0, nj, k0, nk, p->seed, scale, d_out, p->stream));
  return RCQR_OK;
}

rcqr_status_t rcqr_intermediates(rcqr_plan_t p, double* d_W1, double* d_W, double* d_R0, double* d_G, double* d_R1) {
  if (p == nullptr) return RCQR_E_INVALID;
  const Shape& sh = p->sh;
  const size_t nn = (size_t)sh.n * sh.n * 8;
  struct {
    double* dst;
    size_t off, bytes;
  } c[5] = {{d_W1, p->L.w1, (size_t)sh.s1 * sh.n * 8},
            {d_W, p->L.w, (size_t)sh.s2 * sh.n * 8},
            {d_R0, p->L.r0, nn},
            {d_G, p->L.g, nn},
            {d_R1, p->L.r1, nn}};
  const bool fp32 = (p->flags & RCQR_FLAG_SKETCH_FP32) != 0;
  for (int i = 0; i < 5; ++i) {
    auto& e = c[i];
    if (!e.dst) continue;
    if (fp32 && i < 2)  // W1 and W of the single-precision sketch are FP32 in the workspace
      RCQR_TRY(launch_widen(reinterpret_cast<const float*>(p->ws + e.off), (int64_t)(e.bytes / 8), e.dst, p->stream));
    else
      RCQR_TRY(hipMemcpyAsync(e.dst, p->ws + e.off, e.bytes, hipMemcpyDeviceToDevice, p->stream));
  }
  return RCQR_OK;
}

rcqr_status_t rcqr_set_tuning(rcqr_plan_t p, int32_t final_mode, int32_t grid_mult) {
  if (p == nullptr || (final_mode != RCQR_FINAL_RECOMPUTE && final_mode != RCQR_FINAL_MATERIALIZE) || grid_mult < 1 ||
      grid_mult > 8)
    return RCQR_E_INVALID;
  p->final_mode = final_mode;
  p->grid_mult = grid_mult;
  return RCQR_OK;
}

rcqr_status_t rcqr_get_tuning(rcqr_plan_t p, int32_t* final_mode, int32_t* grid_mult) {
  if (p == nullptr || final_mode == nullptr || grid_mult == nullptr) return RCQR_E_INVALID;
  *final_mode = p->final_mode;
  *grid_mult = p->grid_mult;
  return RCQR_OK;
}

rcqr_status_t rcqr_tune(rcqr_plan_t p, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr, int32_t reps,
                        float* best_ms) {
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  if ((const void*)Q == (const void*)V || reps < 1 || reps > 1000) return RCQR_E_INVALID;  // V must survive the trials
  const int modes = (p->sh.np <= 64 && !(p->flags & RCQR_FLAG_REORTH)) ? 2 : 1;
  const int mults[3] = {1, 2, 4};
  const int cap = p->cap;
  p->cap = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rcqr_status_t out = RCQR_OK;
  float best = 0.f;
  int best_mode = p->final_mode, best_mult = p->grid_mult;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) out = RCQR_E_HIP;
  for (int mo = 0; mo < modes && out == RCQR_OK; ++mo) {
    for (int k = 0; k < 3 && out == RCQR_OK; ++k) {
      p->final_mode = mo;
      p->grid_mult = mults[k];
      if (rcqr_factor(p, V, ldv, Q, ldq, R, ldr) != RCQR_OK) out = RCQR_E_HIP;  // warm-up
      if (out == RCQR_OK && hipEventRecord(e0, p->stream) != hipSuccess) out = RCQR_E_HIP;
      for (int r = 0; r < reps && out == RCQR_OK; ++r)
        if (rcqr_factor(p, V, ldv, Q, ldq, R, ldr) != RCQR_OK) out = RCQR_E_HIP;
      float ms = 0.f;
      if (out == RCQR_OK && (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        out = RCQR_E_HIP;
      ms /= reps;
      if (out == RCQR_OK && (best == 0.f || ms < best)) {
        best = ms;
        best_mode = mo;
        best_mult = mults[k];
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  p->cap = cap;
  p->final_mode = best_mode;
  p->grid_mult = best_mult;
  if (best_ms) *best_ms = best;
  return out;
}

struct rcqr_graph_s {
  rcqr_plan_t plan;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

rcqr_status_t rcqr_graph_create(rcqr_plan_t p, int32_t method, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R,
                                int64_t ldr, rcqr_graph_t* out) {
  if (out == nullptr) return RCQR_E_INVALID;
  *out = nullptr;
  if (p == nullptr || method < RCQR_METHOD_RAND_CHOLQR || method > RCQR_METHOD_SCHOLQR3) return RCQR_E_INVALID;
  if (p->stream == nullptr) return RCQR_E_INVALID;  // the legacy default stream cannot be captured
  const rcqr_status_t st = check_io(p, V, ldv, Q, ldq, R, ldr);
  if (st != RCQR_OK) return st;
  // host-side, one-time setup outside the capture
  RCQR_TRY(prepare_cholesky(p->sh.np));
  RCQR_TRY(prepare_stream_launches());
  const int cap = p->cap;
  p->cap = 0;  // no timing events inside the graph
  RCQR_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  rcqr_status_t sc = RCQR_OK;
  if (method == RCQR_METHOD_RAND_CHOLQR) sc = rcqr_factor(p, V, ldv, Q, ldq, R, ldr);
  else if (method == RCQR_METHOD_CHOLQR2) sc = rcqr_cholqr2(p, V, ldv, Q, ldq, R, ldr);
  else sc = rcqr_scholqr3(p, V, ldv, Q, ldq, R, ldr);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->stream, &graph);
  p->cap = cap;
  if (sc != RCQR_OK || ec != hipSuccess || graph == nullptr) {
    if (graph) (void)hipGraphDestroy(graph);
    return sc != RCQR_OK ? sc : RCQR_E_HIP;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return RCQR_E_HIP;
  }
  rcqr_graph_s* g = new (std::nothrow) rcqr_graph_s();
  if (g == nullptr) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return RCQR_E_NOMEM;
  }
  g->plan = p;
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return RCQR_OK;
}

rcqr_status_t rcqr_graph_launch(rcqr_graph_t g) {
  if (g == nullptr) return RCQR_E_INVALID;
  RCQR_TRY(hipGraphLaunch(g->exec, g->plan->stream));
  return RCQR_OK;
}

rcqr_status_t rcqr_graph_destroy(rcqr_graph_t g) {
  if (g == nullptr) return RCQR_E_INVALID;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return RCQR_OK;
}

struct rcqr_batch_s {
  int32_t count;
  hipStream_t s0;              // the first plan's stream: fork and join point
  hipStream_t* streams;        // each member's plan stream
  hipGraph_t* graphs;          // one captured factorization per member
  hipGraphExec_t* execs;
  hipEvent_t fork;
  hipEvent_t* join;            // per member (unused for members on s0)
};

static rcqr_status_t run_method(rcqr_plan_t p, int32_t method, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R,
                                int64_t ldr) {
  if (method == RCQR_METHOD_RAND_CHOLQR) return rcqr_factor(p, V, ldv, Q, ldq, R, ldr);
  if (method == RCQR_METHOD_CHOLQR2) return rcqr_cholqr2(p, V, ldv, Q, ldq, R, ldr);
  return rcqr_scholqr3(p, V, ldv, Q, ldq, R, ldr);
}

static void free_batch(rcqr_batch_s* b) {
  if (b == nullptr) return;
  for (int32_t i = 0; i < b->count; ++i) {
    if (b->execs && b->execs[i]) (void)hipGraphExecDestroy(b->execs[i]);
    if (b->graphs && b->graphs[i]) (void)hipGraphDestroy(b->graphs[i]);
    if (b->join && b->join[i]) (void)hipEventDestroy(b->join[i]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete[] b->streams;
  delete[] b->graphs;
  delete[] b->execs;
  delete[] b->join;
  delete b;
}

// One member captured on its own plan stream (as rcqr_graph_create does).
static rcqr_status_t capture_member(rcqr_plan_t p, int32_t method, const double* V, int64_t ldv, double* Q, int64_t ldq, double* R,
                                    int64_t ldr, hipGraph_t* graph, hipGraphExec_t* exec) {
  const int cap = p->cap;
  p->cap = 0;  // no timing events inside the graph
  if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    p->cap = cap;
    return RCQR_E_HIP;
  }
  const rcqr_status_t sc = run_method(p, method, V, ldv, Q, ldq, R, ldr);
  const hipError_t ec = hipStreamEndCapture(p->stream, graph);
  p->cap = cap;
  if (sc != RCQR_OK) return sc;
  if (ec != hipSuccess || *graph == nullptr) return RCQR_E_HIP;
  if (hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0) != hipSuccess) return RCQR_E_HIP;
  return RCQR_OK;
}

rcqr_status_t rcqr_batch_create(int32_t count, const rcqr_plan_t* plans, int32_t method, const double* const* V, const int64_t* ldv,
                                double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr, rcqr_batch_t* out) {
  if (out == nullptr) return RCQR_E_INVALID;
  *out = nullptr;
  if (count < 1 || plans == nullptr || V == nullptr || ldv == nullptr || Q == nullptr || ldq == nullptr || R == nullptr ||
      ldr == nullptr)
    return RCQR_E_INVALID;
  if (method < RCQR_METHOD_RAND_CHOLQR || method > RCQR_METHOD_SCHOLQR3) return RCQR_E_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    const rcqr_plan_t p = plans[i];
    if (p == nullptr || p->stream == nullptr) return RCQR_E_INVALID;
    for (int32_t k = 0; k < i; ++k)
      if (plans[k] == p) return RCQR_E_INVALID;
    const rcqr_status_t st = check_io(p, V[i], ldv[i], Q[i], ldq[i], R[i], ldr[i]);
    if (st != RCQR_OK) return st;
  }
  // host-side, one-time setup outside the captures
  for (int32_t i = 0; i < count; ++i) RCQR_TRY(prepare_cholesky(plans[i]->sh.np));
  RCQR_TRY(prepare_stream_launches());
  rcqr_batch_s* b = new (std::nothrow) rcqr_batch_s();
  if (b == nullptr) return RCQR_E_NOMEM;
  b->count = count;
  b->s0 = plans[0]->stream;
  b->streams = new (std::nothrow) hipStream_t[count]();
  b->graphs = new (std::nothrow) hipGraph_t[count]();
  b->execs = new (std::nothrow) hipGraphExec_t[count]();
  b->join = new (std::nothrow) hipEvent_t[count]();
  if (!b->streams || !b->graphs || !b->execs || !b->join) {
    free_batch(b);
    return RCQR_E_NOMEM;
  }
  rcqr_status_t sc = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess ? RCQR_OK : RCQR_E_HIP;
  for (int32_t i = 0; i < count && sc == RCQR_OK; ++i) {
    b->streams[i] = plans[i]->stream;
    if (hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess) sc = RCQR_E_HIP;
    if (sc == RCQR_OK) sc = capture_member(plans[i], method, V[i], ldv[i], Q[i], ldq[i], R[i], ldr[i], &b->graphs[i], &b->execs[i]);
  }
  if (sc != RCQR_OK) {
    free_batch(b);
    return sc;
  }
  *out = b;
  return RCQR_OK;
}

rcqr_status_t rcqr_batch_launch(rcqr_batch_t b) {
  if (b == nullptr) return RCQR_E_INVALID;
  RCQR_TRY(hipEventRecord(b->fork, b->s0));
  for (int32_t i = 0; i < b->count; ++i) {
    const bool side = b->streams[i] != b->s0;
    if (side) RCQR_TRY(hipStreamWaitEvent(b->streams[i], b->fork, 0));
    RCQR_TRY(hipGraphLaunch(b->execs[i], b->streams[i]));
    if (side) {
      RCQR_TRY(hipEventRecord(b->join[i], b->streams[i]));
      RCQR_TRY(hipStreamWaitEvent(b->s0, b->join[i], 0));
    }
  }
  return RCQR_OK;
}

rcqr_status_t rcqr_batch_destroy(rcqr_batch_t b) {
  if (b == nullptr) return RCQR_E_INVALID;
  free_batch(b);
  return RCQR_OK;
}

rcqr_status_t rcqr_factor_static(int64_t m, int64_t n, int64_t s1, int64_t s2, uint64_t seed, uint32_t flags, const double* V,
                                 int64_t ldv, double* Q, int64_t ldq, double* R, int64_t ldr, int32_t* d_info, void* stream) {
  const rcqr_status_t st = check_shape(m, n, s1, s2);
  if (st != RCQR_OK) return st;
  if (!flags_valid(flags)) return RCQR_E_INVALID;
  const Shape sh = make_shape(m, n, s1, s2);
  const Layout L = make_layout(sh);
  if (L.total > kScratchBytes) return RCQR_E_SCRATCH;
  char* ws = nullptr;
  const rcqr_status_t ss = scratch_address(reinterpret_cast<hipStream_t>(stream), &ws);
  if (ss != RCQR_OK) return ss;
  // a plan on the stack over the scratch array: rcqr_factor's launches, nothing allocated
  rcqr_plan_s p{};
  p.sh = sh;
  p.L = L;
  p.seed = seed;
  p.flags = flags & ~RCQR_FLAG_SKETCH_AT_PLAN;  // no plan outlives the call: the sketch is made in it
  p.stream = reinterpret_cast<hipStream_t>(stream);
  p.ws = ws;
  p.ws_bytes = kScratchBytes;
  p.final_mode = RCQR_FINAL_RECOMPUTE;
  p.grid_mult = 2;
  p.cap = 0;
  p.recorded = 0;
  p.ev = nullptr;
  const rcqr_status_t sf = rcqr_factor(&p, V, ldv, Q, ldq, R, ldr);
  if (sf != RCQR_OK) return sf;
  if (d_info != nullptr) RCQR_TRY(launch_copy_i32(p.at<int32_t>(L.info), d_info, 2, p.stream));
  return RCQR_OK;
}

rcqr_status_t rcqr_q0_twice(rcqr_plan_t p, const double* V, int64_t ldv, double* Q0a, double* Q0b, int64_t ldq) {
  if (p == nullptr || V == nullptr || Q0a == nullptr || Q0b == nullptr || ldv < p->sh.n || ldq < p->sh.n) return RCQR_E_INVALID;
  const Shape& sh = p->sh;
  const Layout& L = p->L;
  if (sh.np <= 64) {
    // the Gram pass as the materialising mode runs it (Q0 stored from its LDS staging), and the
    // final pass the factorization runs, given R1 = I: its product by the identity adds only
    // zeros to each x_k (one MFMA term is x_k * 1, the others 0 * R), so it returns the Q0 rows
    // it recomputed unchanged
    RCQR_TRY(launch_trsm_gram(sh.np, V, sh.m, (int)sh.n, ldv, p->at<double>(L.r0pk), p->at<int32_t>(L.info), p->at<double>(L.gpart),
                              Q0a, ldq, p->stream));
    RCQR_TRY(launch_identity_factor((int)sh.n, sh.np, p->at<double>(L.ra), p->at<double>(L.rapk), p->stream));
    RCQR_TRY(launch_final(sh.np, true, V, sh.m, (int)sh.n, ldv, p->at<double>(L.r0pk), p->at<double>(L.rapk),
                          p->at<int32_t>(L.info), Q0b, ldq, p->stream, p->grid_mult));
  } else {  // Q0 is stored, not recomputed: both outputs come from the Gram phase's solve
    RCQR_TRY(launch_solve128_gram(V, sh.m, (int)sh.n, ldv, p->at<double>(L.r0pk), p->at<int32_t>(L.info), Q0a, ldq,
                                  p->at<double>(L.gplo), p->stream));
    RCQR_TRY(launch_solve128_gram(V, sh.m, (int)sh.n, ldv, p->at<double>(L.r0pk), p->at<int32_t>(L.info), Q0b, ldq,
                                  p->at<double>(L.gplo), p->stream));
  }
  return RCQR_OK;
}

}  // extern "C"
