// Band network: 32 -> 64 -> 64 -> 1 multilayer perceptron with ReLU that
// predicts y = log2(w + 1) for a pair's band half-width w.  Every matrix
// product runs on the matrix cores as v_mfma_f32_16x16x16_bf16 with operands
// rounded to bfloat16 (nearest even) and float32 accumulation; biases, ReLU,
// the loss and the optimiser are float32.
//
// Transposed formulation.  A wave handles 16 samples at a time and computes
// Z^T = W^T X^T, so hidden units run along the MFMA's M dimension and the 16
// samples along N.  The 16x16x16 instruction's operand layouts are (lane l,
// q = l / 16, r = l % 16, c = 0..3):
//   A (M x K): lane holds A[r][4q + c]
//   B (K x N): lane holds B[4q + c][r]
//   D (M x N): lane holds D[4q + c][r]
// so the D block of one layer, rounded, is already the B operand of the next
// layer's K block: activations never leave registers in the forward pass.
// Weights are held in registers as A operands for the whole kernel.
//
// Backward (one Adam step per minibatch):
//   dy    = d(pinball)/dy / S
//   dz2   = dy * w3 * [z2 > 0]                (D layout, float32)
//   dh1^T = W2 dz2b^T                         (MFMA, dz2b in registers)
//   dz1   = dh1 * [z1 > 0]
//   dW2   = h1b^T dz2b,  dW1 = xb^T dz1b      (MFMA over the sample axis)
// The last two contract over samples, so their operands are the transposes
// of the D layout: they go through a small LDS buffer per wave
// (write [unit][sample] as 16-bit, read four consecutive samples of one unit).
// Gradients of a wave accumulate in MFMA accumulators across its tiles and
// are written as one partial per wave; a second kernel sums the partials in a
// fixed order (deterministic) and applies Adam.
//
// Parameter layout (float32): w1[32][64] (input-major), b1[64], w2[64][64],
// b2[64], w3[64], b3[1].
#include "internal.h"

namespace asmi {
namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kIn = kMlpInputs, kHid = kMlpHidden;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid;
static_assert(kOffB3 + 1 == kMlpParams, "parameter layout");

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16r(float x) { return __uint_as_float(bf16_bits(x) << 16); }
__device__ __forceinline__ bf4 pack(float a, float b, float c, float d) {
  bf4 v;
  v[0] = (short)bf16_bits(a);
  v[1] = (short)bf16_bits(b);
  v[2] = (short)bf16_bits(c);
  v[3] = (short)bf16_bits(d);
  return v;
}
__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 zero4() {
  f4 z;
  z[0] = z[1] = z[2] = z[3] = 0.f;
  return z;
}

// Weights of one wave, as MFMA A operands plus the per-lane vectors.
struct Net {
  bf4 w1t[4][2];   // A = W1^T, block (mb, kk): lane holds w1[16kk + 4q + c][16mb + r]
  bf4 w2t[4][4];   // A = W2^T, block (mb, kk): w2[16kk + 4q + c][16mb + r]
  float b1[4][4], b2[4][4], w3[4][4];  // unit 16mb + 4q + c (w3 rounded to bfloat16)
  float b3;
};

__device__ void load_net(const float *P, Net &nt) {
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const float *w = P + kOffW1 + (16 * kk + 4 * q) * kHid + 16 * mb + r;
      nt.w1t[mb][kk] = pack(w[0], w[kHid], w[2 * kHid], w[3 * kHid]);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float *w = P + kOffW2 + (16 * kk + 4 * q) * kHid + 16 * mb + r;
      nt.w2t[mb][kk] = pack(w[0], w[kHid], w[2 * kHid], w[3 * kHid]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int u = 16 * mb + 4 * q + c;
      nt.b1[mb][c] = P[kOffB1 + u];
      nt.b2[mb][c] = P[kOffB2 + u];
      nt.w3[mb][c] = bf16r(P[kOffW3 + u]);
    }
  }
  nt.b3 = P[kOffB3];
}

// Forward state of one 16-sample tile (sample r of the tile in lane r, 16+r, ...).
struct Tile {
  float xb[2][4];                 // B layout of X^T: feature 16kk + 4q + c (bfloat16 values)
  float z1[4][4], h1[4][4];       // D layout: unit 16mb + 4q + c; h1 rounded
  float z2[4][4], h2[4][4];
  float y;                        // network output of sample r (every lane)
};

__device__ void forward(const Net &nt, const float *x /* this lane's sample, 32 floats */, bool valid,
                        Tile &T) {
  const int l = threadIdx.x & 63, q = l >> 4;
  bf4 X[2];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
      const float4 f = *reinterpret_cast<const float4 *>(x + 16 * kk + 4 * q);
      v[0] = f.x;
      v[1] = f.y;
      v[2] = f.z;
      v[3] = f.w;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) T.xb[kk][c] = bf16r(v[c]);
    X[kk] = pack(v[0], v[1], v[2], v[3]);
  }
  bf4 H1[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f4 acc = zero4();
    acc = mfma(nt.w1t[mb][0], X[0], acc);
    acc = mfma(nt.w1t[mb][1], X[1], acc);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T.z1[mb][c] = acc[c] + nt.b1[mb][c];
      T.h1[mb][c] = bf16r(fmaxf(T.z1[mb][c], 0.f));
    }
    H1[mb] = pack(T.h1[mb][0], T.h1[mb][1], T.h1[mb][2], T.h1[mb][3]);
  }
  float part = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f4 acc = zero4();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = mfma(nt.w2t[mb][kk], H1[kk], acc);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T.z2[mb][c] = acc[c] + nt.b2[mb][c];
      T.h2[mb][c] = bf16r(fmaxf(T.z2[mb][c], 0.f));
      part += nt.w3[mb][c] * T.h2[mb][c];  // bfloat16 x bfloat16 is exact in float32
    }
  }
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  T.y = part + nt.b3;
}

// ---------------------------------------------------------------- inference

__global__ void __launch_bounds__(256) mlp_predict_kernel(const float *params, const float *features,
                                                          int64_t n, int32_t *w_out, float *y_out) {
  Net nt;
  load_net(params, nt);
  const int l = threadIdx.x & 63, r = l & 15;
  const int64_t n_tiles = (n + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
    const int64_t s = tile * 16 + r;
    const bool valid = s < n;
    Tile T;
    forward(nt, features + (valid ? s : 0) * kIn, valid, T);
    if (l < 16 && valid) {
      if (y_out) y_out[s] = T.y;
      // w = ceil(2^y - 1), clamped to [0, 2^20]
      float y = T.y;
      if (!(y < 20.f)) y = 20.f;
      float w = ceilf(exp2f(y) - 1.f);
      w = w > 0.f ? w : 0.f;
      w_out[s] = (int32_t)w;
    }
  }
}

// ---------------------------------------------------------------- training

struct GradArgs {
  const float *params;
  const float *features;   // [n][32]
  const int32_t *labels;   // [n] band labels; target = log2(label + 1)
  const int32_t *order;    // minibatch: indices of its `batch` samples
  int32_t batch;
  float tau;               // pinball quantile
  float *partials;         // [gridDim.x][kMlpPartialStride]
};

// Transpose buffer of one wave: [unit][sample] as 16-bit values.
struct TBuf {
  uint16_t x[kIn][16];
  uint16_t h1[kHid][16];
  uint16_t dz2[kHid][16];
  uint16_t dz1[kHid][16];
};

__device__ __forceinline__ bf4 read_t(const uint16_t (*buf)[16], int unit) {
  const int q = (threadIdx.x & 63) >> 4;
  const uint2 v = *reinterpret_cast<const uint2 *>(&buf[unit][4 * q]);
  bf4 o;
  o[0] = (short)(v.x & 0xFFFFu);
  o[1] = (short)(v.x >> 16);
  o[2] = (short)(v.y & 0xFFFFu);
  o[3] = (short)(v.y >> 16);
  return o;
}

__device__ __forceinline__ float reduce16(float v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  return v;
}

__global__ void __launch_bounds__(64) mlp_grad_kernel(GradArgs a) {
  __shared__ TBuf tb;
  Net nt;
  load_net(a.params, nt);
  const int l = threadIdx.x, q = l >> 4, r = l & 15;
  // A = W2 (not transposed) for dh1^T = W2 dz2b^T, block (ma, kb): w2[16ma + r][16kb + 4q + c]
  bf4 w2n[4][4];
#pragma unroll
  for (int ma = 0; ma < 4; ++ma)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const float *w = a.params + kOffW2 + (16 * ma + r) * kHid + 16 * kb + 4 * q;
      w2n[ma][kb] = pack(w[0], w[1], w[2], w[3]);
    }
  f4 gw2[4][4], gw1[2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gw2[i][j] = zero4();
      if (i < 2) gw1[i][j] = zero4();
    }
  float gb1[4][4] = {}, gb2[4][4] = {}, gw3[4][4] = {};
  float gb3 = 0.f;
  const float inv_s = 1.f / (float)a.batch;
  const int n_tiles = (a.batch + 15) / 16;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int j = tile * 16 + r;
    const bool valid = j < a.batch;
    const int s = valid ? a.order[j] : 0;
    Tile T;
    forward(nt, a.features + (int64_t)s * kIn, valid, T);
    float gy = 0.f;
    if (valid) {
      const float target = (float)log2((double)a.labels[s] + 1.0);
      gy = T.y < target ? -a.tau : (T.y > target ? 1.f - a.tau : 0.f);
      gy *= inv_s;
    }
    if (l < 16) gb3 += gy;
    bf4 DZ2[4];
    float dz2b[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        gw3[mb][c] += T.h2[mb][c] * gy;
        const float d = T.z2[mb][c] > 0.f ? gy * nt.w3[mb][c] : 0.f;
        gb2[mb][c] += d;
        dz2b[mb][c] = bf16r(d);
      }
      DZ2[mb] = pack(dz2b[mb][0], dz2b[mb][1], dz2b[mb][2], dz2b[mb][3]);
    }
    float dz1b[4][4];
#pragma unroll
    for (int ma = 0; ma < 4; ++ma) {
      f4 acc = zero4();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma(w2n[ma][kb], DZ2[kb], acc);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float d = T.z1[ma][c] > 0.f ? acc[c] : 0.f;
        gb1[ma][c] += d;
        dz1b[ma][c] = bf16r(d);
      }
    }
    // [unit][sample] tiles for the sample-axis contractions
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int u = 16 * mb + 4 * q + c;
        tb.h1[u][r] = (uint16_t)bf16_bits(T.h1[mb][c]);
        tb.dz2[u][r] = (uint16_t)bf16_bits(dz2b[mb][c]);
        tb.dz1[u][r] = (uint16_t)bf16_bits(dz1b[mb][c]);
        if (mb < 2) tb.x[u][r] = (uint16_t)bf16_bits(T.xb[mb][c]);
      }
    __syncthreads();
    // dW2[a][b] += sum_j h1b[a][j] dz2b[b][j]: A = h1b (M = a), B = dz2b^T (N = b)
    bf4 Hs[4], Ds[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Hs[i] = read_t(tb.h1, 16 * i + r);
      Ds[i] = read_t(tb.dz2, 16 * i + r);
    }
#pragma unroll
    for (int ma = 0; ma < 4; ++ma)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) gw2[ma][nb] = mfma(Hs[ma], Ds[nb], gw2[ma][nb]);
    // dW1[f][a] += sum_j xb[j][f] dz1b[j][a]
    bf4 Xs[2], D1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      D1[i] = read_t(tb.dz1, 16 * i + r);
      if (i < 2) Xs[i] = read_t(tb.x, 16 * i + r);
    }
#pragma unroll
    for (int mf = 0; mf < 2; ++mf)
#pragma unroll
      for (int na = 0; na < 4; ++na) gw1[mf][na] = mfma(Xs[mf], D1[na], gw1[mf][na]);
    __syncthreads();  // the buffer is rewritten by the next tile
  }

  float *out = a.partials + (int64_t)blockIdx.x * kMlpPartialStride;
#pragma unroll
  for (int mf = 0; mf < 2; ++mf)
#pragma unroll
    for (int na = 0; na < 4; ++na)
#pragma unroll
      for (int c = 0; c < 4; ++c) out[kOffW1 + (16 * mf + 4 * q + c) * kHid + 16 * na + r] = gw1[mf][na][c];
#pragma unroll
  for (int ma = 0; ma < 4; ++ma)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int c = 0; c < 4; ++c) out[kOffW2 + (16 * ma + 4 * q + c) * kHid + 16 * nb + r] = gw2[ma][nb][c];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float v1 = reduce16(gb1[mb][c]);
      const float v2 = reduce16(gb2[mb][c]);
      const float v3 = reduce16(gw3[mb][c]);
      if (r == 0) {
        const int u = 16 * mb + 4 * q + c;
        out[kOffB1 + u] = v1;
        out[kOffB2 + u] = v2;
        out[kOffW3 + u] = v3;
      }
    }
  const float v = reduce16(gb3);
  if (l == 0) out[kOffB3] = v;
}

// Sum of the partials in wave order, then one Adam step (bias corrections
// c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t) come from the host).
__global__ void __launch_bounds__(256) mlp_adam_kernel(const float *partials, int n_parts, float *params,
                                                       float *m1, float *m2, float *grads_out, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float g = 0.f;
  for (int w = 0; w < n_parts; ++w) g += partials[(int64_t)w * kMlpPartialStride + p];
  if (grads_out) grads_out[p] = g;
  const float m = b1 * m1[p] + (1.f - b1) * g;
  const float v = b2 * m2[p] + (1.f - b2) * g * g;
  m1[p] = m;
  m2[p] = v;
  params[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

}  // namespace

hipError_t launch_mlp_predict(const float *params, const float *features, int64_t n, int32_t *w_out,
                              float *y_out, int num_cu, hipStream_t stream) {
  const int64_t tiles = (n + 15) / 16;
  int64_t grid = (tiles + 3) / 4;
  const int64_t cap = (int64_t)num_cu * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)grid), dim3(256), 0, stream, params, features, n,
                     w_out, y_out);
  return hipGetLastError();
}

int mlp_grad_parts(int batch) {
  const int tiles = (batch + 15) / 16;
  return tiles < kMlpMaxParts ? tiles : kMlpMaxParts;
}

hipError_t launch_mlp_train_step(const float *features, const int32_t *labels, const int32_t *order,
                                 int32_t batch, float tau, float *params, float *m1, float *m2,
                                 float *partials, float *grads_out, float lr, float c1, float c2,
                                 hipStream_t stream) {
  GradArgs ga;
  ga.params = params;
  ga.features = features;
  ga.labels = labels;
  ga.order = order;
  ga.batch = batch;
  ga.tau = tau;
  ga.partials = partials;
  const int parts = mlp_grad_parts(batch);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(parts), dim3(64), 0, stream, ga);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, partials, parts,
                     params, m1, m2, grads_out, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
  return hipGetLastError();
}

}  // namespace asmi
