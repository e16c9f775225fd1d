// Host runtime and C ABI of the library (include/anyseq_mi.h).
//
// Per call: argument checks on the host, then on the caller's stream
//   1. classify: per pair, offsets are validated, empty pairs are scored by
//      their closed form (mode paragraphs of the paper's section 2.1), every
//      other pair gets an orientation (which sequence is streamed down the
//      rows) and is appended to the work list; the a priori score range is
//      checked against the 32-bit cell budget;
//   2. the counters are read back (one small device-to-host copy);
//   3. the persistent full-DP kernel drains the work list;
//   4. the status word is read back and turned into the return code.
#include <mutex>
#include <string.h>
#include <vector>

#include "internal.h"
#include "anyseq_mi.h"

namespace asmi {
namespace {

constexpr int64_t kMaxLen = (int64_t)1 << 30;
constexpr int64_t kCellBudget32 = (int64_t)1 << 28;  // |shifted cell| must stay below

__global__ void classify_kernel(const int64_t *__restrict__ offs_a,
                                const int64_t *__restrict__ offs_b, int64_t n_pairs, int32_t mode,
                                int32_t alpha, int32_t beta, int32_t smax_abs, int32_t stripe_w,
                                PairDesc *__restrict__ items, Counters *ctr,
                                int32_t *__restrict__ scores) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = offs_a[p], a1 = offs_a[p + 1];
    const int64_t b0 = offs_b[p], b1 = offs_b[p + 1];
    if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0) {
      atomicOr(&ctr->status, kStatusBadOffsets);
      continue;
    }
    const int64_t m = a1 - a0, n = b1 - b0;
    atomicAdd(&ctr->cells, (unsigned long long)(m * n));
    // Every cell value, in either frame the kernels use, is bounded in
    // magnitude by (|sigma|max + alpha + 2 beta) * (m + n + 2).
    if (m >= kMaxLen || n >= kMaxLen ||
        (int64_t)(smax_abs + alpha + 2 * beta) * (m + n + 2) >= kCellBudget32) {
      atomicOr(&ctr->status, kStatusRange);
      continue;
    }
    if (m == 0 || n == 0) {
      // one gap of length m + n (global) or the empty alignment (others)
      const int64_t len = m + n;
      scores[p] = (mode == kGlobal && len > 0) ? (int32_t)(-alpha - beta * (len - 1)) : 0;
      continue;
    }
    // Orientation: the cost of a stripe pass is (rows + 15) steps over 16*K
    // columns; pick the cheaper of A-as-rows and B-as-rows.
    const int64_t sa = (n + stripe_w - 1) / stripe_w, sb = (m + stripe_w - 1) / stripe_w;
    const int64_t cost_a = sa * (m + kGroup - 1), cost_b = sb * (n + kGroup - 1);
    const bool tr = cost_b < cost_a;
    PairDesc d;
    d.row_off = tr ? b0 : a0;
    d.col_off = tr ? a0 : b0;
    d.m = (int32_t)(tr ? n : m);
    d.n = (int32_t)(tr ? m : n);
    d.pair = (int32_t)p;
    d.flags = tr ? kTransposed : 0;
    const int slot = atomicAdd(&ctr->n_full32, 1);
    items[slot] = d;
    if (d.n > stripe_w) atomicMax(&ctr->max_rows_multi, d.m);
  }
}

struct Workspace {
  int device = -1;
  int num_cu = 0;
  PairDesc *items = nullptr;
  int64_t items_cap = 0;
  Counters *ctr = nullptr;
  Counters *host_ctr = nullptr;  // pinned
  int8_t *subst = nullptr;       // 32*32 bytes
  int2 *bnd = nullptr;
  int64_t bnd_cap = 0;           // int2 elements
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

bool g_timing = false;
as_timing g_last_timing;

std::mutex g_lock;
std::vector<Workspace> g_ws;

#define AS_HIP(call)                         \
  do {                                       \
    if ((call) != hipSuccess) return AS_ERR_HIP; \
  } while (0)

int get_workspace(Workspace **out) {
  int dev = 0;
  AS_HIP(hipGetDevice(&dev));
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  Workspace &w = g_ws[dev];
  if (w.device < 0) {
    hipDeviceProp_t prop;
    AS_HIP(hipGetDeviceProperties(&prop, dev));
    w.num_cu = prop.multiProcessorCount;
    AS_HIP(hipMalloc(&w.ctr, sizeof(Counters)));
    AS_HIP(hipHostMalloc(&w.host_ctr, sizeof(Counters), hipHostMallocDefault));
    AS_HIP(hipMalloc(&w.subst, 32 * 32));
    for (auto &e : w.ev) AS_HIP(hipEventCreate(&e));
    w.device = dev;
  }
  *out = &w;
  return AS_OK;
}

int grow(void **ptr, int64_t *cap, int64_t need, size_t elem) {
  if (*cap >= need) return AS_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  const int64_t n = need + need / 4;
  AS_HIP(hipMalloc(ptr, (size_t)n * elem));
  *cap = n;
  return AS_OK;
}

int status_to_code(int32_t st) {
  if (st & kStatusBadOffsets) return AS_ERR_OFFSETS;
  if (st & kStatusBadResidue) return AS_ERR_RESIDUE;
  if (st & kStatusRange) return AS_ERR_RANGE;
  return AS_OK;
}

}  // namespace
}  // namespace asmi

using namespace asmi;

extern "C" int as_align_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                              const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                              int32_t mode, int32_t *scores_out, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scores_out || !scoring->subst)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  const int asz = scoring->alphabet_size;
  const int alpha = scoring->gap_open, beta = scoring->gap_extend;
  if (asz < 2 || asz > 32 || beta < 0 || alpha < beta || alpha > 10000 || mode < 0 || mode > 2)
    return AS_ERR_SCORING;
  int smin = 127, smax = -128;
  for (int i = 0; i < asz * asz; ++i) {
    smin = scoring->subst[i] < smin ? scoring->subst[i] : smin;
    smax = scoring->subst[i] > smax ? scoring->subst[i] : smax;
  }
  // The 32-bit kernel stores sigma + bias as int8 (bias = alpha + beta, or
  // alpha for local; padding columns store the bias itself).
  const int bias = (mode == kLocal) ? alpha : alpha + beta;
  if (smax + bias > 127 || smin + bias < -128 || bias > 127) return AS_ERR_SCORING;
  if (n_pairs == 0) return AS_OK;
  const int smax_abs = (smax > -smin) ? smax : -smin;

  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  int rc = get_workspace(&w);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  rc = grow((void **)&w->items, &w->items_cap, n_pairs, sizeof(PairDesc));
  if (rc) return rc;

  AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)asz * asz, hipMemcpyHostToDevice, stream));
  AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
  const bool timing = g_timing;
  memset(&g_last_timing, 0, sizeof(g_last_timing));
  if (timing) AS_HIP(hipEventRecord(w->ev[0], stream));
  const int stripe_w = full_dp_i32_stripe_width();
  {
    const int threads = 256;
    int64_t blocks = (n_pairs + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, offs_a,
                       offs_b, n_pairs, mode, alpha, beta, smax_abs, stripe_w, w->items, w->ctr,
                       scores_out);
    AS_HIP(hipGetLastError());
  }
  if (timing) AS_HIP(hipEventRecord(w->ev[1], stream));
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  const Counters c = *w->host_ctr;
  g_last_timing.cells = (int64_t)c.cells;
  g_last_timing.pairs_full32 = c.n_full32;
  if (timing) AS_HIP(hipEventElapsedTime(&g_last_timing.classify_ms, w->ev[0], w->ev[1]));
  rc = status_to_code(c.status);
  if (rc) return rc;

  if (c.n_full32 > 0) {
    const int bpc = full_dp_i32_blocks_per_cu(mode, asz);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need_waves = ((int64_t)c.n_full32 + kGroupsPerWave - 1) / kGroupsPerWave;
    if (grid > need_waves) grid = need_waves;
    const int64_t bnd_rows = c.max_rows_multi > 0 ? (int64_t)c.max_rows_multi + 1 : 1;
    rc = grow((void **)&w->bnd, &w->bnd_cap, grid * kGroupsPerWave * 2 * bnd_rows, sizeof(int2));
    if (rc) return rc;
    FullDpArgs args;
    args.seqs_a = seqs_a;
    args.seqs_b = seqs_b;
    args.items = w->items;
    args.ctr = w->ctr;
    args.subst = w->subst;
    args.asz = asz;
    args.alpha = alpha;
    args.beta = beta;
    args.scores = scores_out;
    args.bnd = w->bnd;
    args.bnd_rows = bnd_rows;
    if (timing) AS_HIP(hipEventRecord(w->ev[2], stream));
    AS_HIP(launch_full_dp_i32(mode, args, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[3], stream));
  }
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  if (timing && c.n_full32 > 0)
    AS_HIP(hipEventElapsedTime(&g_last_timing.full32_ms, w->ev[2], w->ev[3]));
  return status_to_code(w->host_ctr->status);
}

extern "C" int as_enable_timing(int on) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int prev = g_timing ? 1 : 0;
  g_timing = on != 0;
  return prev;
}

extern "C" int as_last_timing(as_timing *out) {
  if (!out) return AS_ERR_NULL;
  std::lock_guard<std::mutex> guard(g_lock);
  *out = g_last_timing;
  return AS_OK;
}

extern "C" const char *as_strerror(int code) {
  switch (code) {
    case AS_OK: return "success";
    case AS_ERR_NULL: return "a required pointer is NULL";
    case AS_ERR_OFFSETS: return "offsets decrease or are negative";
    case AS_ERR_RESIDUE: return "a residue code is >= alphabet_size";
    case AS_ERR_SCORING: return "invalid scoring (alphabet size, alpha, beta, mode or sigma range)";
    case AS_ERR_RANGE: return "a score could leave the 32-bit range";
    case AS_ERR_HIP: return "a HIP runtime call failed";
    case AS_ERR_ARG: return "an argument is out of range";
    default: return "unknown error";
  }
}

extern "C" int as_release_workspace(void) {
  std::lock_guard<std::mutex> guard(g_lock);
  for (Workspace &w : g_ws) {
    if (w.device < 0) continue;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w.device);
    if (w.items) (void)hipFree(w.items);
    if (w.ctr) (void)hipFree(w.ctr);
    if (w.host_ctr) (void)hipHostFree(w.host_ctr);
    if (w.subst) (void)hipFree(w.subst);
    if (w.bnd) (void)hipFree(w.bnd);
    for (auto &e : w.ev) if (e) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    w = Workspace();
  }
  return AS_OK;
}

extern "C" const char *as_build_info(void) {
  return "anyseq_mi gfx950: full DP int32 (16-lane DPP groups, K=16, int8 LDS profile)";
}
