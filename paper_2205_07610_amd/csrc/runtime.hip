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

struct ClassifyParams {
  const int64_t *offs_a;
  const int64_t *offs_b;
  int64_t n_pairs;
  int32_t mode, alpha, beta, smax_abs, smax_pos;
  int32_t stripe_w, allow16, stripe_w16;
  int32_t long_w;         // stripe width of the wavefront kernel
  int32_t long_min_rows;  // pairs with at least this many rows and more than
                          // one wavefront stripe of columns go to the wavefront
};

// Route of one pair: 0 none (error or empty pair, scored here), 1 the 32-bit
// list, 2 the packed 16-bit list.  Fills d for routes 1 and 2.
__device__ int route_pair(const ClassifyParams &c, int64_t p, Counters *ctr,
                          int32_t *__restrict__ scores, bool first_pass, PairDesc &d,
                          unsigned long long &cells) {
  const int64_t a0 = c.offs_a[p], a1 = c.offs_a[p + 1];
  const int64_t b0 = c.offs_b[p], b1 = c.offs_b[p + 1];
  if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0) {
    if (first_pass) atomicOr(&ctr->status, kStatusBadOffsets);
    return 0;
  }
  const int64_t m = a1 - a0, n = b1 - b0;
  cells = (unsigned long long)(m * n);
  // Every cell value, in either frame the kernels use, is bounded in
  // magnitude by (|sigma|max + alpha + 2 beta) * (m + n + 2).
  if (m >= kMaxLen || n >= kMaxLen ||
      (int64_t)(c.smax_abs + c.alpha + 2 * c.beta) * (m + n + 2) >= kCellBudget32) {
    if (first_pass) atomicOr(&ctr->status, kStatusRange);
    return 0;
  }
  if (m == 0 || n == 0) {
    // one gap of length m + n (global) or the empty alignment (others)
    const int64_t len = m + n;
    if (first_pass)
      scores[p] = (c.mode == kGlobal && len > 0) ? (int32_t)(-c.alpha - c.beta * (len - 1)) : 0;
    return 0;
  }
  // Orientation: a stripe pass costs (rows + 15) steps over 16*K columns;
  // take the cheaper of A-as-rows and B-as-rows.
  const int64_t sa = (n + c.stripe_w - 1) / c.stripe_w, sb = (m + c.stripe_w - 1) / c.stripe_w;
  const int64_t cost_a = sa * (m + kGroup - 1), cost_b = sb * (n + kGroup - 1);
  const bool tr = cost_b < cost_a;
  d.row_off = tr ? b0 : a0;
  d.col_off = tr ? a0 : b0;
  d.m = (int32_t)(tr ? n : m);
  d.n = (int32_t)(tr ? m : n);
  d.pair = (int32_t)p;
  d.flags = tr ? kTransposed : 0;
  if (c.allow16 && d.n <= c.stripe_w16) {
    if (c.mode == kLocal) return 2;  // saturation is detected at run time
    // shifted-frame cells stay below sigma_max*min(m,n) + beta*(m+n), plus
    // the profile byte and the padding offset beta*W16
    const int64_t ub = (int64_t)c.smax_pos * (m < n ? m : n) + (int64_t)c.beta * (m + n) +
                       (int64_t)c.beta * c.stripe_w16 + c.alpha + 2 * c.beta + 256;
    if (ub < 32000) return 2;
  }
  if (d.n > c.long_w && d.m >= c.long_min_rows) return 3;
  if (first_pass && d.n > c.stripe_w) atomicMax(&ctr->max_rows_multi, d.m);
  return 1;
}

// Block-wide exclusive prefix of a per-thread 0/1 flag (256 threads).
// Returns the prefix; *total gets the block's count.
__device__ int block_prefix(bool flag, int *lds4, int *total) {
  const unsigned long long mask = __ballot(flag);
  const int lane = (int)__lane_id(), wave = threadIdx.x >> 6;
  const int in_wave = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) lds4[wave] = __popcll(mask);
  __syncthreads();
  int before = 0, sum = 0;
  for (int w = 0; w < 4; ++w) {
    const int v = lds4[w];
    before += (w < wave) ? v : 0;
    sum += v;
  }
  __syncthreads();
  *total = sum;
  return before + in_wave;
}

// Each block owns a contiguous range of pairs: it counts its routes, reserves
// its slice of each work list with one atomic per list, then scatters.  Items
// of a block stay in pair order inside the lists.
__global__ void __launch_bounds__(256) classify_kernel(ClassifyParams c, PairDesc *__restrict__ items32,
                                                       PairDesc *__restrict__ items16,
                                                       LongItem *__restrict__ items_long,
                                                       Counters *ctr, int32_t *__restrict__ scores) {
  __shared__ int lds4[4];
  __shared__ int base_sh[3];
  const int64_t chunk = (c.n_pairs + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < c.n_pairs ? lo + chunk : c.n_pairs;
  int cnt32 = 0, cnt16 = 0, cntl = 0;
  unsigned long long cells = 0;
  for (int64_t t0 = lo; t0 < hi; t0 += 256) {
    const int64_t p = t0 + threadIdx.x;
    int r = 0;
    if (p < hi) {
      PairDesc d;
      unsigned long long cl = 0;
      r = route_pair(c, p, ctr, scores, true, d, cl);
      cells += cl;
    }
    cnt32 += (r == 1);
    cnt16 += (r == 2);
    cntl += (r == 3);
  }
  // block totals: one atomic per list and one for the cell count
  for (int off = 32; off > 0; off >>= 1) {
    cnt32 += __shfl_xor(cnt32, off);
    cnt16 += __shfl_xor(cnt16, off);
    cntl += __shfl_xor(cntl, off);
    cells += __shfl_xor(cells, off);
  }
  __shared__ int s32[4], s16[4], sl[4];
  __shared__ unsigned long long sc[4];
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 0) { s32[wave] = cnt32; s16[wave] = cnt16; sl[wave] = cntl; sc[wave] = cells; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t32 = s32[0] + s32[1] + s32[2] + s32[3];
    const int t16 = s16[0] + s16[1] + s16[2] + s16[3];
    const unsigned long long tc = sc[0] + sc[1] + sc[2] + sc[3];
    base_sh[0] = t32 ? atomicAdd(&ctr->n_full32, t32) : 0;
    base_sh[1] = t16 ? atomicAdd(&ctr->n_full16, t16) : 0;
    const int tl = sl[0] + sl[1] + sl[2] + sl[3];
    base_sh[2] = tl ? atomicAdd(&ctr->n_long, tl) : 0;
    if (tc) atomicAdd(&ctr->cells, tc);
  }
  __syncthreads();
  int cur32 = base_sh[0], cur16 = base_sh[1], curl = base_sh[2];
  for (int64_t t0 = lo; t0 < hi; t0 += 256) {
    const int64_t p = t0 + threadIdx.x;
    int r = 0;
    PairDesc d;
    if (p < hi) {
      unsigned long long cl = 0;
      r = route_pair(c, p, ctr, scores, false, d, cl);
    }
    int n32, n16, nl;
    const int i32 = block_prefix(r == 1, lds4, &n32);
    const int i16 = block_prefix(r == 2, lds4, &n16);
    const int il = block_prefix(r == 3, lds4, &nl);
    if (r == 1) items32[cur32 + i32] = d;
    if (r == 2) items16[cur16 + i16] = d;
    if (r == 3) items_long[curl + il].d = d;
    cur32 += n32;
    cur16 += n16;
    curl += nl;
  }
}

// One block: prefix sums over the wavefront list (first ticket and boundary
// offset of every long pair), and the score seed that the stripes' atomic
// maxima start from (0 = the empty alignment / boundary cells).
__global__ void __launch_bounds__(256) long_prep_kernel(LongItem *items, Counters *ctr, int32_t long_w,
                                                        int32_t mode, int32_t *scores) {
  __shared__ int lds4[4];
  const int n = ctr->n_long;
  int task = 0;
  long long bnd = 0;
  for (int b = 0; b < n; b += 256) {
    const int i = b + threadIdx.x;
    int st = 0;
    long long be = 0;
    if (i < n) {
      const PairDesc d = items[i].d;
      st = (d.n + long_w - 1) / long_w;
      be = (long long)(st - 1) * (d.m + 1);
      if (mode != kGlobal) scores[d.pair] = 0;
    }
    // block-wide inclusive scans of st and be (256 threads, simple two-level)
    __shared__ int sst[256];
    __shared__ long long sbe[256];
    sst[threadIdx.x] = st;
    sbe[threadIdx.x] = be;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int vs = threadIdx.x >= off ? sst[threadIdx.x - off] : 0;
      const long long vb = threadIdx.x >= off ? sbe[threadIdx.x - off] : 0;
      __syncthreads();
      sst[threadIdx.x] += vs;
      sbe[threadIdx.x] += vb;
      __syncthreads();
    }
    if (i < n) {
      items[i].task0 = task + sst[threadIdx.x] - st;
      items[i].stripes = st;
      items[i].bnd_off = bnd + sbe[threadIdx.x] - be;
    }
    task += sst[255];
    bnd += sbe[255];
    __syncthreads();
  }
  (void)lds4;
  if (threadIdx.x == 0) {
    ctr->n_long_tasks = task;
    ctr->long_bnd_total = bnd;
  }
}

struct Workspace {
  int device = -1;
  int num_cu = 0;
  PairDesc *items = nullptr;    // 32-bit work list
  int64_t items_cap = 0;
  PairDesc *items16 = nullptr;  // 16-bit work list
  int64_t items16_cap = 0;
  PairDesc *rerun = nullptr;    // saturated 16-bit pairs
  int64_t rerun_cap = 0;
  LongItem *items_long = nullptr;  // wavefront list
  int64_t items_long_cap = 0;
  int2 *bnd_long = nullptr;        // wavefront boundary columns
  int64_t bnd_long_cap = 0;
  int32_t *flags = nullptr;        // wavefront progress counters
  int64_t flags_cap = 0;
  Counters *ctr = nullptr;
  Counters *host_ctr = nullptr;  // pinned
  int8_t *subst = nullptr;       // 32*32 bytes
  int2 *bnd = nullptr;
  int64_t bnd_cap = 0;           // int2 elements
  hipEvent_t ev[10] = {};
};

bool g_timing = false;
int32_t g_i16_limit = 32767;
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
  if (st & kStatusStall) return AS_ERR_HIP;
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
  // The packed kernel keeps sigma + bias as unsigned bytes in registers, one
  // byte per letter of an alphabet of at most four.
  const int allow16 = (asz <= 4 && smin + bias >= 0 && smax + bias <= 255) ? 1 : 0;

  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  int rc = get_workspace(&w);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  if ((rc = grow((void **)&w->items, &w->items_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->items16, &w->items16_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->rerun, &w->rerun_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->items_long, &w->items_long_cap, n_pairs, sizeof(LongItem)))) return rc;

  AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)asz * asz, hipMemcpyHostToDevice, stream));
  AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
  const bool timing = g_timing;
  memset(&g_last_timing, 0, sizeof(g_last_timing));
  if (timing) AS_HIP(hipEventRecord(w->ev[0], stream));
  const int stripe_w = full_dp_i32_stripe_width();
  const int stripe_w16 = full_dp_i16_stripe_width();
  {
    ClassifyParams cp;
    cp.offs_a = offs_a;
    cp.offs_b = offs_b;
    cp.n_pairs = n_pairs;
    cp.mode = mode;
    cp.alpha = alpha;
    cp.beta = beta;
    cp.smax_abs = smax_abs;
    cp.smax_pos = smax > 0 ? smax : 0;
    cp.stripe_w = stripe_w;
    cp.allow16 = allow16;
    cp.stripe_w16 = stripe_w16;
    cp.long_w = long_dp_i32_stripe_width();
    cp.long_min_rows = 2048;
    int64_t blocks = (n_pairs + 1023) / 1024;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, cp, w->items,
                       w->items16, w->items_long, w->ctr, scores_out);
    AS_HIP(hipGetLastError());
    hipLaunchKernelGGL(long_prep_kernel, dim3(1), dim3(256), 0, stream, w->items_long, w->ctr,
                       cp.long_w, mode, scores_out);
    AS_HIP(hipGetLastError());
  }
  if (timing) AS_HIP(hipEventRecord(w->ev[1], stream));
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  const Counters c = *w->host_ctr;
  g_last_timing.cells = (int64_t)c.cells;
  g_last_timing.pairs_full32 = c.n_full32;
  g_last_timing.pairs_full16 = c.n_full16;
  if (timing) AS_HIP(hipEventElapsedTime(&g_last_timing.classify_ms, w->ev[0], w->ev[1]));
  rc = status_to_code(c.status);
  if (rc) return rc;

  if (c.n_full16 > 0) {
    const int bpc = full_dp_i16_blocks_per_cu(mode);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need = ((int64_t)c.n_full16 + 2 * kGroupsPerWave - 1) / (2 * kGroupsPerWave);
    if (grid > need) grid = need;
    FullDp16Args a16;
    a16.seqs_a = seqs_a;
    a16.seqs_b = seqs_b;
    a16.items = w->items16;
    a16.ctr = w->ctr;
    a16.rerun = w->rerun;
    a16.subst = w->subst;
    a16.asz = asz;
    a16.alpha = alpha;
    a16.beta = beta;
    a16.sat_limit = g_i16_limit;
    a16.scores = scores_out;
    if (timing) AS_HIP(hipEventRecord(w->ev[2], stream));
    AS_HIP(launch_full_dp_i16(mode, a16, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[3], stream));
  }

  FullDpArgs args;
  args.seqs_a = seqs_a;
  args.seqs_b = seqs_b;
  args.ctr = w->ctr;
  args.subst = w->subst;
  args.asz = asz;
  args.alpha = alpha;
  args.beta = beta;
  args.scores = scores_out;
  if (c.n_full32 > 0) {
    const int bpc = full_dp_i32_blocks_per_cu(mode, asz);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need_waves = ((int64_t)c.n_full32 + kGroupsPerWave - 1) / kGroupsPerWave;
    if (grid > need_waves) grid = need_waves;
    const int64_t bnd_rows = c.max_rows_multi > 0 ? (int64_t)c.max_rows_multi + 1 : 1;
    rc = grow((void **)&w->bnd, &w->bnd_cap, grid * kGroupsPerWave * 2 * bnd_rows, sizeof(int2));
    if (rc) return rc;
    args.items = w->items;
    args.n_items = &w->ctr->n_full32;
    args.next = &w->ctr->next_full32;
    args.bnd = w->bnd;
    args.bnd_rows = bnd_rows;
    if (timing) AS_HIP(hipEventRecord(w->ev[4], stream));
    AS_HIP(launch_full_dp_i32(mode, args, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[5], stream));
  }
  if (c.n_long > 0) {
    if ((rc = grow((void **)&w->bnd_long, &w->bnd_long_cap, c.long_bnd_total > 0 ? c.long_bnd_total : 1,
                   sizeof(int2))))
      return rc;
    if ((rc = grow((void **)&w->flags, &w->flags_cap, c.n_long_tasks, sizeof(int32_t)))) return rc;
    AS_HIP(hipMemsetAsync(w->flags, 0, sizeof(int32_t) * (size_t)c.n_long_tasks, stream));
    const int bpc = long_dp_i32_blocks_per_cu(mode, asz);
    int64_t grid = (int64_t)bpc * w->num_cu;
    if (grid > c.n_long_tasks) grid = c.n_long_tasks;
    LongDpArgs la;
    la.seqs_a = seqs_a;
    la.seqs_b = seqs_b;
    la.items = w->items_long;
    la.ctr = w->ctr;
    la.subst = w->subst;
    la.asz = asz;
    la.alpha = alpha;
    la.beta = beta;
    la.scores = scores_out;
    la.bnd = w->bnd_long;
    la.flags = w->flags;
    if (timing) AS_HIP(hipEventRecord(w->ev[8], stream));
    AS_HIP(launch_long_dp_i32(mode, la, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[9], stream));
  }
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  const Counters c2 = *w->host_ctr;
  g_last_timing.pairs_long = c.n_long;
  if (timing && c.n_long > 0)
    AS_HIP(hipEventElapsedTime(&g_last_timing.long_ms, w->ev[8], w->ev[9]));
  if (timing && c.n_full16 > 0)
    AS_HIP(hipEventElapsedTime(&g_last_timing.full16_ms, w->ev[2], w->ev[3]));
  if (timing && c.n_full32 > 0)
    AS_HIP(hipEventElapsedTime(&g_last_timing.full32_ms, w->ev[4], w->ev[5]));
  rc = status_to_code(c2.status);
  if (rc) return rc;

  // 32-bit re-run of the 16-bit pairs whose maximum saturated
  g_last_timing.pairs_rerun32 = c2.n_rerun32;
  if (c2.n_rerun32 > 0) {
    const int bpc = full_dp_i32_blocks_per_cu(mode, asz);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need_waves = ((int64_t)c2.n_rerun32 + kGroupsPerWave - 1) / kGroupsPerWave;
    if (grid > need_waves) grid = need_waves;
    // re-run pairs fit one 16-bit stripe, hence one 32-bit stripe: no boundary buffer
    if ((rc = grow((void **)&w->bnd, &w->bnd_cap, grid * kGroupsPerWave * 2, sizeof(int2)))) return rc;
    args.items = w->rerun;
    args.n_items = &w->ctr->n_rerun32;
    args.next = &w->ctr->next_rerun32;
    args.bnd = w->bnd;
    args.bnd_rows = 1;
    if (timing) AS_HIP(hipEventRecord(w->ev[6], stream));
    AS_HIP(launch_full_dp_i32(mode, args, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[7], stream));
    AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
    AS_HIP(hipStreamSynchronize(stream));
    if (timing) AS_HIP(hipEventElapsedTime(&g_last_timing.rerun32_ms, w->ev[6], w->ev[7]));
    rc = status_to_code(w->host_ctr->status);
    if (rc) return rc;
  }
  return AS_OK;
}

extern "C" int as_set_i16_limit(int32_t limit) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int32_t prev = g_i16_limit;
  g_i16_limit = (limit <= 0 || limit > 32767) ? 32767 : limit;
  return prev;
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
    if (w.items16) (void)hipFree(w.items16);
    if (w.rerun) (void)hipFree(w.rerun);
    if (w.items_long) (void)hipFree(w.items_long);
    if (w.bnd_long) (void)hipFree(w.bnd_long);
    if (w.flags) (void)hipFree(w.flags);
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
  return "anyseq_mi gfx950: full DP int32 (16-lane DPP groups, K=16, int8 LDS profile); "
         "full DP packed int16x2 (2 pairs per group, K=16, v_perm register profile, alphabet <= 4)";
}
