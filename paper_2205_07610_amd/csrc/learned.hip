// C ABI of the learned band (include/anyseq_mi.h): per-pair features,
// network inference and training, band labels from the full DP, and the
// learned-band alignment (features -> network -> certified banded rounds ->
// full-DP fallback).
//
// Labels.  For a pair with full-DP score S, no band whose leave bound
// exceeds S can be accepted (its banded score is at most S), so the search
// starts at w_cert, the smallest w whose bound is <= S (bisection on the
// closed form).  Exact bands are then tried on the GPU: while nothing has
// been accepted w goes to 2w + 1, afterwards the interval (largest rejected,
// smallest accepted) is bisected.  Acceptance is monotone in w (the banded
// score grows and the bound shrinks as the band widens), so this finds the
// smallest accepted w.  Every round is one exact-band launch over the pairs
// still searching.
#include <math.h>
#include <mutex>
#include <string.h>
#include <vector>

#include "internal.h"

namespace asmi {
namespace {

static_assert(AS_MLP_PARAMS == kMlpParams, "parameter count");
static_assert(AS_FEATURES == kMlpInputs, "feature count");
constexpr int kWideLabel = AS_BAND_WIDE;
constexpr int kMaxLabelRounds = 64;

struct LabelState {
  int32_t rej;  // largest half-width known to be rejected (-1: none)
  int32_t acc;  // smallest known to be accepted (cap + 1: none yet)
  int32_t cap;  // largest half-width whose band fits the widest class
  int32_t pad;
};

struct LearnedWs {
  int device = -1;
  int num_cu = 0;
  float *features = nullptr;
  int64_t features_cap = 0;
  int32_t *w = nullptr;        // predicted / tried half-widths
  int64_t w_cap = 0;
  int32_t *full = nullptr;     // full-DP scores (labels)
  int64_t full_cap = 0;
  int32_t *band = nullptr;     // banded scores (labels)
  int64_t band_cap = 0;
  int32_t *accept = nullptr;
  int64_t accept_cap = 0;
  LabelState *state = nullptr;
  int64_t state_cap = 0;
  int32_t *labels = nullptr;   // labels of as_train_band_model
  int64_t labels_cap = 0;
  float *partials = nullptr;   // [kMlpMaxParts][kMlpPartialStride]
  float *adam = nullptr;       // [2][kMlpParams], as_train_band_model
  int32_t *dstat = nullptr;    // device: [0] status bits, [1] counter
  int32_t *hstat = nullptr;    // pinned copy
  hipEvent_t ev[4] = {};
};

std::mutex g_llock;
std::vector<LearnedWs> g_lws;

#define LS_HIP(call)                             \
  do {                                           \
    if ((call) != hipSuccess) return AS_ERR_HIP; \
  } while (0)

int get_lws(LearnedWs **out) {
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));
  if ((int)g_lws.size() <= dev) g_lws.resize(dev + 1);
  LearnedWs &w = g_lws[dev];
  if (w.device < 0) {
    hipDeviceProp_t prop;
    LS_HIP(hipGetDeviceProperties(&prop, dev));
    w.num_cu = prop.multiProcessorCount;
    LS_HIP(hipMalloc(&w.dstat, 2 * sizeof(int32_t)));
    LS_HIP(hipHostMalloc(&w.hstat, 2 * sizeof(int32_t), hipHostMallocDefault));
    LS_HIP(hipMalloc(&w.partials, sizeof(float) * kMlpMaxParts * kMlpPartialStride));
    LS_HIP(hipMalloc(&w.adam, sizeof(float) * 2 * kMlpParams));
    for (auto &e : w.ev) LS_HIP(hipEventCreate(&e));
    w.device = dev;
  }
  *out = &w;
  return AS_OK;
}

template <typename T>
int grow(T **ptr, int64_t *cap, int64_t need) {
  if (*cap >= need) return AS_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  const int64_t n = need + need / 4;
  LS_HIP(hipMalloc((void **)ptr, (size_t)n * sizeof(T)));
  *cap = n;
  return AS_OK;
}

int read_stat(LearnedWs *w, hipStream_t stream) {
  LS_HIP(hipMemcpyAsync(w->hstat, w->dstat, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  LS_HIP(hipStreamSynchronize(stream));
  return AS_OK;
}

int stat_code(int32_t st) {
  if (st & kStatusBadOffsets) return AS_ERR_OFFSETS;
  if (st & kStatusBadResidue) return AS_ERR_RESIDUE;
  if (st) return AS_ERR_ARG;
  return AS_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------- labels

__global__ void __launch_bounds__(256) label_init_kernel(const int64_t *offs_a, const int64_t *offs_b,
                                                         int64_t n_pairs, const int32_t *full, int32_t smax,
                                                         int32_t alpha, int32_t beta, int32_t mode,
                                                         LabelState *state, int32_t *w_try, int32_t *labels,
                                                         int32_t *active) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int64_t m0 = offs_a[p + 1] - offs_a[p], n0 = offs_b[p + 1] - offs_b[p];
  w_try[p] = -1;
  if (m0 == 0 || n0 == 0) {
    labels[p] = 0;
    return;
  }
  // orientation of the banded kernel: rows = the shorter sequence
  const int m = (int)(m0 < n0 ? m0 : n0), n = (int)(m0 < n0 ? n0 : m0);
  const int dn = n - m;
  const int cap = (kExactBandMax - 1 - dn) / 2;
  if (dn > kExactBandMax - 1) {
    labels[p] = kWideLabel;
    return;
  }
  const int64_t S = full[p];
  auto bound_ok = [&](int w) -> bool {
    int64_t ub = 0;
    const bool leave = band_leave_bound(m, n, -w, dn + w, smax, alpha, beta, mode, &ub);
    return !leave || S >= ub;
  };
  if (!bound_ok(cap)) {
    labels[p] = kWideLabel;
    return;
  }
  int wc = 0;
  if (!bound_ok(0)) {
    int lo = 0, hi = cap;  // lo fails, hi passes
    while (hi - lo > 1) {
      const int mid = lo + (hi - lo) / 2;
      if (bound_ok(mid)) hi = mid;
      else lo = mid;
    }
    wc = hi;
  }
  LabelState st;
  st.rej = wc - 1;
  st.acc = cap + 1;
  st.cap = cap;
  st.pad = 0;
  state[p] = st;
  w_try[p] = wc;
  atomicAdd(active, 1);
}

__global__ void __launch_bounds__(256) label_step_kernel(int64_t n_pairs, const int32_t *accept,
                                                         LabelState *state, int32_t *w_try, int32_t *labels,
                                                         int32_t *active) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int w = w_try[p];
  if (w < 0) return;
  LabelState st = state[p];
  if (accept[p]) st.acc = w;
  else st.rej = w;
  int next;
  if (st.acc == st.rej + 1) {
    labels[p] = st.acc <= st.cap ? st.acc : kWideLabel;
    next = -1;
  } else if (st.acc > st.cap) {
    next = 2 * w + 1 < st.cap ? 2 * w + 1 : st.cap;  // nothing accepted yet: widen
  } else {
    next = st.rej + (st.acc - st.rej) / 2;             // bisect (rej, acc)
  }
  state[p] = st;
  w_try[p] = next;
  if (next >= 0) atomicAdd(active, 1);
}

// ---------------------------------------------------------------- training

__global__ void __launch_bounds__(256) train_check_kernel(const int32_t *order, int64_t n_order, int64_t n,
                                                          const int32_t *labels, int32_t *status) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_order;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= order[i] < 0 || order[i] >= n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= labels[i] < 0;
  if (bad) atomicOr(status, 1);
}

int blocks_for(int64_t n, int per = 256) {
  const int64_t b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : b);  // n < 2^31, so at most 2^23 blocks
}

// ---------------------------------------------------------------- implementations

int features_impl(LearnedWs *w, const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                  const int64_t *offs_b, int64_t n_pairs, float *out, hipStream_t stream) {
  LS_HIP(hipMemsetAsync(w->dstat, 0, 2 * sizeof(int32_t), stream));
  LS_HIP(launch_features(seqs_a, offs_a, seqs_b, offs_b, n_pairs, out, w->dstat, w->num_cu, stream));
  int rc = read_stat(w, stream);
  if (rc) return rc;
  return stat_code(w->hstat[0]);
}

int labels_impl(LearnedWs *w, const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                int32_t *labels, hipStream_t stream) {
  // scoring and mode checks of the banded path (no pair is touched)
  int rc = band_call(seqs_a, offs_a, seqs_b, offs_b, 0, scoring, mode, labels, 1, 1, 1, labels, nullptr,
                     nullptr, labels, nullptr, stream);
  if (rc) return rc;
  if ((rc = grow(&w->full, &w->full_cap, n_pairs))) return rc;
  if ((rc = grow(&w->band, &w->band_cap, n_pairs))) return rc;
  if ((rc = grow(&w->accept, &w->accept_cap, n_pairs))) return rc;
  if ((rc = grow(&w->state, &w->state_cap, n_pairs))) return rc;
  if ((rc = grow(&w->w, &w->w_cap, n_pairs))) return rc;
  if ((rc = as_align_batch(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, w->full, stream)))
    return rc;
  int smax = -128;
  const int asz = scoring->alphabet_size;
  for (int i = 0; i < asz * asz; ++i) smax = scoring->subst[i] > smax ? scoring->subst[i] : smax;
  LS_HIP(hipMemsetAsync(w->dstat, 0, 2 * sizeof(int32_t), stream));
  hipLaunchKernelGGL(label_init_kernel, dim3(blocks_for(n_pairs)), dim3(256), 0, stream, offs_a, offs_b,
                     n_pairs, w->full, smax, scoring->gap_open, scoring->gap_extend, mode, w->state, w->w,
                     labels, w->dstat + 1);
  LS_HIP(hipGetLastError());
  if ((rc = read_stat(w, stream))) return rc;
  for (int r = 0; w->hstat[1] > 0; ++r) {
    if (r >= kMaxLabelRounds) return AS_ERR_HIP;  // the search is bounded far below this
    rc = band_call(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, w->w, 1, 1, 1, w->band, nullptr,
                   nullptr, w->accept, nullptr, stream);
    if (rc) return rc;
    LS_HIP(hipMemsetAsync(w->dstat, 0, 2 * sizeof(int32_t), stream));
    hipLaunchKernelGGL(label_step_kernel, dim3(blocks_for(n_pairs)), dim3(256), 0, stream, n_pairs, w->accept,
                       w->state, w->w, labels, w->dstat + 1);
    LS_HIP(hipGetLastError());
    if ((rc = read_stat(w, stream))) return rc;
  }
  return AS_OK;
}

int train_impl(LearnedWs *w, float *params, float *m1, float *m2, const float *features, const int32_t *labels,
               int64_t n, const int32_t *order, int32_t n_steps, int32_t batch, int32_t t0, float lr, float tau,
               float *grads_out, hipStream_t stream) {
  const int64_t n_order = (int64_t)n_steps * batch;
  LS_HIP(hipMemsetAsync(w->dstat, 0, 2 * sizeof(int32_t), stream));
  hipLaunchKernelGGL(train_check_kernel, dim3(blocks_for(n_order > n ? n_order : n)), dim3(256), 0, stream,
                     order, n_order, n, labels, w->dstat);
  LS_HIP(hipGetLastError());
  int rc = read_stat(w, stream);
  if (rc) return rc;
  if (w->hstat[0]) return AS_ERR_ARG;
  for (int s = 0; s < n_steps; ++s) {
    const double t = (double)t0 + s;
    const float c1 = (float)(1.0 / (1.0 - pow(0.9, t)));
    const float c2 = (float)(1.0 / (1.0 - pow(0.999, t)));
    LS_HIP(launch_mlp_train_step(features, labels, order + (int64_t)s * batch, batch, tau, params, m1, m2,
                                 w->partials, s == 0 ? grads_out : nullptr, lr, c1, c2, stream));
  }
  return AS_OK;
}

bool bad_pairs_args(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b, const int64_t *offs_b) {
  return !seqs_a || !offs_a || !seqs_b || !offs_b;
}

bool bad_train_args(int64_t n, int32_t n_steps, int32_t batch, int32_t t0, float lr, float tau) {
  return n < 1 || n >= ((int64_t)1 << 31) - 1 || n_steps < 0 || batch < 1 || batch > (1 << 24) || t0 < 1 ||
         !(lr > 0.f) || !(lr < 1e3f) || !(tau > 0.f) || !(tau < 1.f);
}

}  // namespace

void release_learned_workspace() {
  std::lock_guard<std::mutex> guard(g_llock);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (LearnedWs &w : g_lws) {
    if (w.device < 0) continue;
    (void)hipSetDevice(w.device);
    void *bufs[] = {w.features, w.w, w.full, w.band, w.accept, w.state, w.labels, w.partials, w.adam, w.dstat};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
    if (w.hstat) (void)hipHostFree(w.hstat);
    for (auto &e : w.ev)
      if (e) (void)hipEventDestroy(e);
    w = LearnedWs();
  }
  (void)hipSetDevice(cur);
}

}  // namespace asmi

using namespace asmi;

extern "C" int as_pair_features(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                const int64_t *offs_b, int64_t n_pairs, float *features_out, void *stream) {
  if (bad_pairs_args(seqs_a, offs_a, seqs_b, offs_b) || !features_out) return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1 || !aligned16(features_out)) return AS_ERR_ARG;
  if (n_pairs == 0) return AS_OK;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  return features_impl(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, features_out, (hipStream_t)stream);
}

extern "C" int as_band_predict(const float *params, const float *features, int64_t n, int32_t *band_w_out,
                               float *y_out, void *stream) {
  if (!params || !features || !band_w_out) return AS_ERR_NULL;
  if (n < 0 || n >= ((int64_t)1 << 31) - 1 || !aligned16(features)) return AS_ERR_ARG;
  if (n == 0) return AS_OK;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  LS_HIP(launch_mlp_predict(params, features, n, band_w_out, y_out, w->num_cu, (hipStream_t)stream));
  return AS_OK;
}

extern "C" int as_band_labels(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                              const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                              int32_t *labels_out, void *stream) {
  if (bad_pairs_args(seqs_a, offs_a, seqs_b, offs_b) || !labels_out || !scoring || !scoring->subst)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  return labels_impl(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, labels_out, (hipStream_t)stream);
}

extern "C" int as_band_train(float *params, float *adam_m, float *adam_v, const float *features,
                             const int32_t *labels, int64_t n, const int32_t *order, int32_t n_steps,
                             int32_t batch, int32_t t0, float lr, float tau, float *grads_out, void *stream) {
  if (!params || !adam_m || !adam_v || !features || !labels || !order) return AS_ERR_NULL;
  if (bad_train_args(n, n_steps, batch, t0, lr, tau) || !aligned16(features)) return AS_ERR_ARG;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  return train_impl(w, params, adam_m, adam_v, features, labels, n, order, n_steps, batch, t0, lr, tau,
                    grads_out, (hipStream_t)stream);
}

extern "C" int as_train_band_model(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                                   int32_t mode, float *params, const int32_t *order, int32_t n_steps,
                                   int32_t batch, float lr, float tau, void *stream_ptr) {
  if (bad_pairs_args(seqs_a, offs_a, seqs_b, offs_b) || !scoring || !scoring->subst || !params || !order)
    return AS_ERR_NULL;
  if (bad_train_args(n_pairs, n_steps, batch, 1, lr, tau)) return AS_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_ptr;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  if ((rc = grow(&w->features, &w->features_cap, n_pairs * kMlpInputs))) return rc;
  if ((rc = grow(&w->labels, &w->labels_cap, n_pairs))) return rc;
  if ((rc = features_impl(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, w->features, stream))) return rc;
  if ((rc = labels_impl(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, w->labels, stream))) return rc;
  LS_HIP(hipMemsetAsync(w->adam, 0, sizeof(float) * 2 * kMlpParams, stream));
  return train_impl(w, params, w->adam, w->adam + kMlpParams, w->features, w->labels, n_pairs, order, n_steps,
                    batch, 1, lr, tau, nullptr, stream);
}

extern "C" int as_align_batch_learned(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                      const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                                      int32_t mode, const float *params, int32_t max_rounds, int32_t *scores_out,
                                      as_band_stats *stats, void *stream_ptr) {
  if (bad_pairs_args(seqs_a, offs_a, seqs_b, offs_b) || !scoring || !scoring->subst || !params || !scores_out)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_ptr;
  std::lock_guard<std::mutex> guard(g_llock);
  LearnedWs *w = nullptr;
  int rc = get_lws(&w);
  if (rc) return rc;
  // scoring, mode and round checks before any work
  if ((rc = band_call(seqs_a, offs_a, seqs_b, offs_b, 0, scoring, mode, scores_out, max_rounds, 0, 0,
                      scores_out, nullptr, nullptr, nullptr, stats, stream)))
    return rc;
  if (n_pairs == 0) return AS_OK;
  if ((rc = grow(&w->features, &w->features_cap, n_pairs * kMlpInputs))) return rc;
  if ((rc = grow(&w->w, &w->w_cap, n_pairs))) return rc;
  const bool timing = timing_enabled();
  if (timing) LS_HIP(hipEventRecord(w->ev[0], stream));
  if ((rc = features_impl(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, w->features, stream))) return rc;
  if (timing) LS_HIP(hipEventRecord(w->ev[1], stream));
  LS_HIP(launch_mlp_predict(params, w->features, n_pairs, w->w, nullptr, w->num_cu, stream));
  if (timing) LS_HIP(hipEventRecord(w->ev[2], stream));
  rc = band_call(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, w->w, max_rounds, 0, 0, scores_out,
                 nullptr, nullptr, nullptr, stats, stream);
  if (rc) return rc;
  if (timing) {
    float f = 0.f, m = 0.f;
    LS_HIP(hipEventSynchronize(w->ev[2]));
    (void)hipEventElapsedTime(&f, w->ev[0], w->ev[1]);
    (void)hipEventElapsedTime(&m, w->ev[1], w->ev[2]);
    record_learned_timing(f, m);
  }
  return AS_OK;
}

// ---- band model blobs ----
// Layout (little-endian): a 64-byte header
//   char magic[8] = "ASBANDMD"; uint32 version = 1; uint32 n_params = 6337;
//   uint32 inputs = 32; uint32 hidden = 64; uint32 has_adam (0/1);
//   uint32 reserved = 0; int64 adam_t; uint32 checksum; uint32 reserved[5]
// followed by the float32 parameters in the library's layout (w1 [32][64],
// b1 [64], w2 [64][64], b2 [64], w3 [64], b3) and, with has_adam, the Adam
// first and second moments in the same layout.  The checksum is FNV-1a
// (32-bit) over every payload byte.
namespace asmi {
namespace {

constexpr char kBlobMagic[8] = {'A', 'S', 'B', 'A', 'N', 'D', 'M', 'D'};
constexpr uint32_t kBlobVersion = 1;
constexpr int64_t kBlobHeader = 64;

uint32_t fnv1a(const uint8_t *p, int64_t n) {
  uint32_t h = 2166136261u;
  for (int64_t i = 0; i < n; ++i) h = (h ^ p[i]) * 16777619u;
  return h;
}

}  // namespace
}  // namespace asmi

extern "C" int64_t as_band_model_blob_size(int32_t with_adam) {
  return kBlobHeader + (int64_t)sizeof(float) * kMlpParams * (with_adam ? 3 : 1);
}

extern "C" int as_band_model_save(const float *params, const float *adam_m, const float *adam_v, int64_t adam_t,
                                  void *blob_out, int64_t blob_cap, int64_t *blob_size, void *stream_ptr) {
  if (!params || !blob_out) return AS_ERR_NULL;
  if ((adam_m == nullptr) != (adam_v == nullptr) || adam_t < 0) return AS_ERR_ARG;
  const int with_adam = adam_m ? 1 : 0;
  const int64_t need = as_band_model_blob_size(with_adam);
  if (blob_size) *blob_size = need;
  if (blob_cap < need) return AS_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_ptr;
  uint8_t *b = (uint8_t *)blob_out;
  float *payload = (float *)(b + kBlobHeader);
  const size_t bytes = sizeof(float) * kMlpParams;
  if (hipMemcpyAsync(payload, params, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess) return AS_ERR_HIP;
  if (with_adam) {
    if (hipMemcpyAsync(payload + kMlpParams, adam_m, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(payload + 2 * kMlpParams, adam_v, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess)
      return AS_ERR_HIP;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return AS_ERR_HIP;
  memset(b, 0, kBlobHeader);
  memcpy(b, kBlobMagic, 8);
  const uint32_t hdr[6] = {kBlobVersion, (uint32_t)kMlpParams, (uint32_t)kMlpInputs, (uint32_t)kMlpHidden,
                           (uint32_t)with_adam, 0u};
  memcpy(b + 8, hdr, sizeof(hdr));
  memcpy(b + 32, &adam_t, sizeof(adam_t));
  const uint32_t sum = fnv1a((const uint8_t *)payload, need - kBlobHeader);
  memcpy(b + 40, &sum, sizeof(sum));
  return AS_OK;
}

extern "C" int as_band_model_load(const void *blob, int64_t blob_size, float *params_out, float *adam_m_out,
                                  float *adam_v_out, int64_t *adam_t_out, void *stream_ptr) {
  if (!blob || !params_out) return AS_ERR_NULL;
  if (blob_size < kBlobHeader) return AS_ERR_ARG;
  const uint8_t *b = (const uint8_t *)blob;
  if (memcmp(b, kBlobMagic, 8) != 0) return AS_ERR_ARG;
  uint32_t hdr[6];
  memcpy(hdr, b + 8, sizeof(hdr));
  if (hdr[0] != kBlobVersion || hdr[1] != (uint32_t)kMlpParams || hdr[2] != (uint32_t)kMlpInputs ||
      hdr[3] != (uint32_t)kMlpHidden || hdr[4] > 1)
    return AS_ERR_ARG;
  const int with_adam = (int)hdr[4];
  if (blob_size != as_band_model_blob_size(with_adam)) return AS_ERR_ARG;
  uint32_t sum = 0;
  memcpy(&sum, b + 40, sizeof(sum));
  if (fnv1a(b + kBlobHeader, blob_size - kBlobHeader) != sum) return AS_ERR_ARG;
  if ((adam_m_out || adam_v_out) && !with_adam) return AS_ERR_ARG;
  if ((adam_m_out == nullptr) != (adam_v_out == nullptr)) return AS_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_ptr;
  const float *payload = (const float *)(b + kBlobHeader);
  const size_t bytes = sizeof(float) * kMlpParams;
  if (hipMemcpyAsync(params_out, payload, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return AS_ERR_HIP;
  if (adam_m_out) {
    if (hipMemcpyAsync(adam_m_out, payload + kMlpParams, bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(adam_v_out, payload + 2 * kMlpParams, bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
      return AS_ERR_HIP;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return AS_ERR_HIP;  // the blob is the caller's
  if (adam_t_out) memcpy(adam_t_out, b + 32, sizeof(int64_t));
  return AS_OK;
}

