// Sub-step surrogate network on the gfx950 matrix cores: a per-particle
// multilayer perceptron in_dim -> 128 -> 128 -> 128 -> out_dim (SiLU hidden
// activations), bfloat16 operands with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, gfx950's 32-deep BF16 matrix-core form), FP32
// master weights trained with Adam.  The operand layouts are described with
// the shared building blocks (mlp_device.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp_device.h"
#include "mlp_internal.h"
#include "mrsph.h"
#include "mrsph_mlp.h"

namespace mrsph {

// Forward pass over tiles of kMlpTile rows: all weights in LDS, each wave owns
// 16 rows through all four layers.
template <bool TRAIN>
__global__ void __launch_bounds__(256) k_mlp_forward(MlpDev M, const float *x, float *yout, int rows) {
  extern __shared__ __align__(16) unsigned short lds[];
  const FwdLds L = fwd_lds_layout(lds);
  const int t = threadIdx.x, l = t & 63;
  const int row0 = blockIdx.x * kMlpTile;
  stage_weights(M, L);
  for (int i = t; i < kMlpTile * kMlpIn; i += blockDim.x) {
    int r = i / kMlpIn, c = i % kMlpIn;
    float v = (row0 + r < rows && c < M.in_dim) ? x[(size_t)(row0 + r) * M.in_dim + c] : 0.0f;
    unsigned short h = f2bf(v);
    L.HA[r * pitch(kMlpIn) + c] = h;
    if (TRAIN && row0 + r < rows) M.hin[0][(size_t)(row0 + r) * kMlpIn + c] = h;
  }
  __syncthreads();
  const f4 out = forward_tile<TRAIN>(L, M, row0, rows);
  const int r0 = (t >> 6) * 16;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int r = r0 + (l >> 4) * 4 + j, c = l & 15;
    if (row0 + r >= rows) continue;
    float y = out[j] + L.bias[3 * kMlpHid + c];
    if (TRAIN) M.y[(size_t)(row0 + r) * kMlpOut + c] = y;
    if (c < M.out_dim && yout) yout[(size_t)(row0 + r) * M.out_dim + c] = y;
  }
}

// Output error of 0.5 mean_rows sum_cols (y - t)^2: d = (y - t) / rows (zero in
// the padding columns), and per-block partial sums of (y - t)^2.
__global__ void __launch_bounds__(256) k_mlp_out_err(MlpDev M, const float *tgt, int rows) {
  __shared__ double red[256];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < rows * kMlpOut) {
    int r = i / kMlpOut, c = i % kMlpOut;
    float d = 0.0f;
    if (c < M.out_dim) {
      float e = M.y[i] - tgt[(size_t)r * M.out_dim + c];
      sq = (double)e * (double)e;
      d = e / (float)rows;
    }
    M.d0[i] = d;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) M.loss_part[blockIdx.x] = red[0];
}

__global__ void k_mlp_loss_final(MlpDev M, int nparts, int rows) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += M.loss_part[i];
  M.loss[0] = 0.5 * s / rows;
}

// Error of a layer input: din (rows x K) = (bf16(dout) (rows x N) x W^T) * SiLU'(zin).
template <int K, int N>
__global__ void __launch_bounds__(256) k_mlp_back_err(const unsigned short *Wbf, const float *dout, const float *zin,
                                                      float *din, int rows) {
  extern __shared__ __align__(16) unsigned short lds[];
  unsigned short *Ws = lds;                 // K x pitch(N)
  unsigned short *Dt = Ws + K * pitch(N);   // 64 x pitch(N)
  const int t = threadIdx.x, w = t >> 6, l = t & 63, kq = (l >> 4) * 8;
  const int row0 = blockIdx.x * kMlpTile;
  stage_rows(Wbf, Ws, K, N);
  for (int i = t; i < kMlpTile * N; i += blockDim.x) {
    int r = i / N, c = i % N;
    Dt[r * pitch(N) + c] = f2bf(row0 + r < rows ? dout[(size_t)(row0 + r) * N + c] : 0.0f);
  }
  __syncthreads();
  constexpr int KT = K / 16;
  f4 acc[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) acc[kt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int r0 = w * 16;
  if constexpr (N % 32 == 0) {
#pragma unroll
    for (int n0 = 0; n0 < N; n0 += 32) {
      s8 a = lds8(Dt + (r0 + (l & 15)) * pitch(N) + n0 + kq);
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        s8 b = lds8(Ws + (kt * 16 + (l & 15)) * pitch(N) + n0 + kq);
        acc[kt] = mfma_bf16(a, b, acc[kt]);
      }
    }
  } else {
    // the output layer's 16 columns: one 16-deep product (lanes hold 4 of k)
    static_assert(N == 16, "error pass over 16 output columns");
    const int kq4 = (l >> 4) * 4;
    s4 a = *reinterpret_cast<const s4 *>(Dt + (r0 + (l & 15)) * pitch(N) + kq4);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      s4 b = *reinterpret_cast<const s4 *>(Ws + (kt * 16 + (l & 15)) * pitch(N) + kq4);
      acc[kt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[kt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int kt = 0; kt < KT; ++kt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = r0 + (l >> 4) * 4 + j, c = kt * 16 + (l & 15);
      if (row0 + r < rows) {
        size_t o = (size_t)(row0 + r) * K + c;
        din[o] = acc[kt][j] * silu_grad(zin[o]);
      }
    }
}

// Partial weight and bias gradients of one chunk of kMlpChunk rows:
// G (K x N) = hin^T (K x rows) x bf16(dout) (rows x N); gb = sum_rows dout.
template <int K, int N>
__global__ void __launch_bounds__(256) k_mlp_back_weight(const unsigned short *hin, const float *dout, float *partW,
                                                         float *partb, int rows) {
  extern __shared__ __align__(16) unsigned short lds[];
  unsigned short *Ht = lds;                         // K x pitch(kMlpChunk)
  unsigned short *Dt = Ht + K * pitch(kMlpChunk);   // N x pitch(kMlpChunk)
  const int t = threadIdx.x, w = t >> 6, l = t & 63, kq = (l >> 4) * 8;
  const int row0 = blockIdx.x * kMlpChunk;
  for (int i = t; i < kMlpChunk * K; i += blockDim.x) {
    int m = i / K, k = i % K;
    Ht[k * pitch(kMlpChunk) + m] = row0 + m < rows ? hin[(size_t)(row0 + m) * K + k] : (unsigned short)0;
  }
  for (int i = t; i < kMlpChunk * N; i += blockDim.x) {
    int m = i / N, n = i % N;
    Dt[n * pitch(kMlpChunk) + m] = f2bf(row0 + m < rows ? dout[(size_t)(row0 + m) * N + n] : 0.0f);
  }
  __syncthreads();
  if (t < N) {
    float s = 0.0f;
    for (int m = 0; m < kMlpChunk && row0 + m < rows; ++m) s += dout[(size_t)(row0 + m) * N + t];
    partb[(size_t)blockIdx.x * N + t] = s;
  }
  constexpr int NT = N / 16, TILES = (K / 16) * NT, TPW = TILES / 4;
  f4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m0 = 0; m0 < kMlpChunk; m0 += 32) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      int tile = w + 4 * i, kt = tile / NT, nt = tile % NT;
      s8 a = lds8(Ht + (kt * 16 + (l & 15)) * pitch(kMlpChunk) + m0 + kq);
      s8 b = lds8(Dt + (nt * 16 + (l & 15)) * pitch(kMlpChunk) + m0 + kq);
      acc[i] = mfma_bf16(a, b, acc[i]);
    }
  }
  float *P = partW + (size_t)blockIdx.x * K * N;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    int tile = w + 4 * i, kt = tile / NT, nt = tile % NT;
#pragma unroll
    for (int j = 0; j < 4; ++j) P[(size_t)(kt * 16 + (l >> 4) * 4 + j) * N + nt * 16 + (l & 15)] = acc[i][j];
  }
}

// Sum of the chunk partials in chunk order (deterministic).
__global__ void k_mlp_sum_parts(const float *partW, const float *partb, float *gW, float *gb, int KN, int N,
                                int chunks) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < KN) {
    float s = 0.0f;
    for (int c = 0; c < chunks; ++c) s += partW[(size_t)c * KN + i];
    gW[i] = s;
  } else if (i < KN + N) {
    int n = i - KN;
    float s = 0.0f;
    for (int c = 0; c < chunks; ++c) s += partb[(size_t)c * N + n];
    gb[n] = s;
  }
}

// Adam over the contiguous padded parameter block (FP32 master copy).
__global__ void k_mlp_adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bfloat16 copies W (K x N) and W^T (N x K) of one layer.
__global__ void k_mlp_to_bf16(const float *W, unsigned short *Wbf, unsigned short *WTbf, int K, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * N) return;
  int k = i / N, n = i % N;
  unsigned short h = f2bf(W[i]);
  Wbf[i] = h;
  WTbf[(size_t)n * K + k] = h;
}

template <int K, int N>
constexpr size_t err_lds_bytes() {
  return sizeof(unsigned short) * (size_t)(K * pitch(N) + kMlpTile * pitch(N));
}
template <int K, int N>
constexpr size_t wgt_lds_bytes() {
  return sizeof(unsigned short) * (size_t)((K + N) * pitch(kMlpChunk));
}

void mlp_launch_forward(const MlpDev &M, const float *x, float *y, int rows, bool train, hipStream_t st) {
  dim3 grid((rows + kMlpTile - 1) / kMlpTile);
  if (train) hipLaunchKernelGGL(k_mlp_forward<true>, grid, dim3(256), fwd_lds_bytes(), st, M, x, y, rows);
  else hipLaunchKernelGGL(k_mlp_forward<false>, grid, dim3(256), fwd_lds_bytes(), st, M, x, y, rows);
}

static hipError_t allow_lds() {
  hipError_t e = hipSuccess;
  auto set = [&](const void *f, size_t b) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
  };
  set((const void *)k_mlp_forward<true>, fwd_lds_bytes());
  set((const void *)k_mlp_forward<false>, fwd_lds_bytes());
  set((const void *)k_mlp_back_err<kMlpHid, kMlpOut>, err_lds_bytes<kMlpHid, kMlpOut>());
  set((const void *)k_mlp_back_err<kMlpHid, kMlpHid>, err_lds_bytes<kMlpHid, kMlpHid>());
  set((const void *)k_mlp_back_weight<kMlpHid, kMlpOut>, wgt_lds_bytes<kMlpHid, kMlpOut>());
  set((const void *)k_mlp_back_weight<kMlpHid, kMlpHid>, wgt_lds_bytes<kMlpHid, kMlpHid>());
  set((const void *)k_mlp_back_weight<kMlpIn, kMlpHid>, wgt_lds_bytes<kMlpIn, kMlpHid>());
  return e;
}

}  // namespace mrsph

using namespace mrsph;

namespace {

constexpr size_t kAlignM = 256;

struct MlpPlan {
  int in_dim, out_dim, max_rows;
};

size_t mlp_carve(char *base, const MlpPlan &p, MlpDev &D) {
  size_t off = 0;
  auto take = [&](auto *&ptr, size_t count) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + kAlignM - 1) / kAlignM * kAlignM;
    ptr = reinterpret_cast<T *>(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
  };
  float *blocks[4];
  for (float *&b : blocks) take(b, kParamsPadded);
  auto split = [&](float *blk, float **W, float **b) {
    size_t o = 0;
    for (int l = 0; l < kMlpLayers; ++l) {
      W[l] = blk + o;
      o += (size_t)mlp_K(l) * mlp_N(l);
      b[l] = blk + o;
      o += mlp_N(l);
    }
  };
  split(blocks[0], D.W, D.b);
  float *mb_dummy[4], *vb_dummy[4];
  split(blocks[1], D.mW, mb_dummy);
  split(blocks[2], D.vW, vb_dummy);
  for (int l = 0; l < kMlpLayers; ++l) {
    D.mb[l] = mb_dummy[l];
    D.vb[l] = vb_dummy[l];
  }
  split(blocks[3], D.gW, D.gb);
  for (int l = 0; l < kMlpLayers; ++l) {
    take(D.Wbf[l], (size_t)mlp_K(l) * mlp_N(l));
    take(D.WTbf[l], (size_t)mlp_K(l) * mlp_N(l));
  }
  size_t R = (size_t)p.max_rows;
  for (int l = 0; l < kMlpLayers; ++l) take(D.hin[l], R * mlp_K(l));
  for (int l = 0; l < kMlpLayers - 1; ++l) take(D.z[l], R * kMlpHid);
  take(D.y, R * kMlpOut);
  take(D.d0, R * kMlpHid);
  take(D.d1, R * kMlpHid);
  size_t chunks = (R + kMlpChunk - 1) / kMlpChunk;
  take(D.partW, chunks * kMlpHid * kMlpHid);
  take(D.partb, chunks * kMlpHid);
  take(D.loss_part, (R * kMlpOut + 255) / 256 + 1);
  take(D.loss, 1);
  return off + kAlignM;
}

bool mlp_plan(int in_dim, int out_dim, int max_rows, MlpPlan &p) {
  if (in_dim < 1 || in_dim > kMlpIn || out_dim < 1 || out_dim > kMlpOut || max_rows < 1 || max_rows > (1 << 24))
    return false;
  p = {in_dim, out_dim, max_rows};
  return true;
}

// host parameter order W1 b1 ... W4 b4 (unpadded) <-> padded device block
size_t unpadded_count(int in_dim, int out_dim) {
  return (size_t)in_dim * kMlpHid + kMlpHid + 2 * ((size_t)kMlpHid * kMlpHid + kMlpHid) + (size_t)kMlpHid * out_dim +
         out_dim;
}

void pad_params(const float *host, int in_dim, int out_dim, std::vector<float> &blk) {
  blk.assign(kParamsPadded, 0.0f);
  size_t hi = 0, o = 0;
  for (int l = 0; l < kMlpLayers; ++l) {
    int K = mlp_K(l), N = mlp_N(l);
    int kr = l == 0 ? in_dim : K, nr = l == kMlpLayers - 1 ? out_dim : N;
    for (int k = 0; k < kr; ++k)
      for (int n = 0; n < nr; ++n) blk[o + (size_t)k * N + n] = host[hi++];
    o += (size_t)K * N;
    for (int n = 0; n < nr; ++n) blk[o + n] = host[hi++];
    o += N;
  }
}

void unpad_params(const std::vector<float> &blk, int in_dim, int out_dim, float *host) {
  size_t hi = 0, o = 0;
  for (int l = 0; l < kMlpLayers; ++l) {
    int K = mlp_K(l), N = mlp_N(l);
    int kr = l == 0 ? in_dim : K, nr = l == kMlpLayers - 1 ? out_dim : N;
    for (int k = 0; k < kr; ++k)
      for (int n = 0; n < nr; ++n) host[hi++] = blk[o + (size_t)k * N + n];
    o += (size_t)K * N;
    for (int n = 0; n < nr; ++n) host[hi++] = blk[o + n];
    o += N;
  }
}

int refresh_bf16(mlp_ctx *m) {
  for (int l = 0; l < kMlpLayers; ++l) {
    int KN = mlp_K(l) * mlp_N(l);
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((KN + 255) / 256), dim3(256), 0, m->stream, m->D.W[l], m->D.Wbf[l],
                       m->D.WTbf[l], mlp_K(l), mlp_N(l));
  }
  return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
}

}  // namespace

extern "C" {

size_t mlp_arena_bytes(int in_dim, int out_dim, int max_rows) {
  MlpPlan p;
  if (!mlp_plan(in_dim, out_dim, max_rows, p)) return 0;
  MlpDev D;
  std::memset(&D, 0, sizeof D);
  return mlp_carve(nullptr, p, D);
}

int mlp_init(int in_dim, int out_dim, int max_rows, void *dev_arena, size_t arena_bytes, void *stream,
             mlp_ctx **out) {
  if (!out) return SPH_E_ARG;
  *out = nullptr;
  MlpPlan p;
  if (!mlp_plan(in_dim, out_dim, max_rows, p) || !dev_arena) return SPH_E_ARG;
  MlpDev D;
  std::memset(&D, 0, sizeof D);
  size_t need = mlp_carve(nullptr, p, D);
  if (arena_bytes < need) return SPH_E_ARG;
  char *base = (char *)(((uintptr_t)dev_arena + kAlignM - 1) / kAlignM * kAlignM);
  mlp_carve(base, p, D);
  D.in_dim = in_dim;
  D.out_dim = out_dim;
  D.max_rows = max_rows;
  if (allow_lds() != hipSuccess) return SPH_E_HIP;
  mlp_ctx *m = new mlp_ctx();
  m->D = D;
  m->stream = (hipStream_t)stream;
  m->step = 0;
  m->nparam = unpadded_count(in_dim, out_dim);
  // parameters, moments and gradients start at zero
  if (hipMemsetAsync(D.W[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess ||
      hipMemsetAsync(D.mW[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess ||
      hipMemsetAsync(D.vW[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess ||
      hipMemsetAsync(D.gW[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess ||
      refresh_bf16(m) != SPH_OK || hipStreamSynchronize(m->stream) != hipSuccess) {
    delete m;
    return SPH_E_HIP;
  }
  *out = m;
  return SPH_OK;
}

size_t mlp_param_count(const mlp_ctx *m) { return m ? m->nparam : 0; }

int mlp_set_params(mlp_ctx *m, const float *host, size_t n) {
  if (!m) return SPH_E_ORDER;
  if (!host || n != m->nparam) return SPH_E_ARG;
  std::vector<float> blk;
  pad_params(host, m->D.in_dim, m->D.out_dim, blk);
  if (hipMemcpyAsync(m->D.W[0], blk.data(), sizeof(float) * kParamsPadded, hipMemcpyHostToDevice, m->stream) !=
          hipSuccess ||
      hipMemsetAsync(m->D.mW[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess ||
      hipMemsetAsync(m->D.vW[0], 0, sizeof(float) * kParamsPadded, m->stream) != hipSuccess)
    return SPH_E_HIP;
  m->step = 0;
  if (refresh_bf16(m) != SPH_OK) return SPH_E_HIP;
  return hipStreamSynchronize(m->stream) == hipSuccess ? SPH_OK : SPH_E_HIP;
}

static int copy_block(mlp_ctx *m, const float *dev, float *host, size_t n) {
  if (!m) return SPH_E_ORDER;
  if (!host || n != m->nparam) return SPH_E_ARG;
  std::vector<float> blk(kParamsPadded);
  if (hipMemcpyAsync(blk.data(), dev, sizeof(float) * kParamsPadded, hipMemcpyDeviceToHost, m->stream) !=
          hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return SPH_E_HIP;
  unpad_params(blk, m->D.in_dim, m->D.out_dim, host);
  return SPH_OK;
}

int mlp_get_params(mlp_ctx *m, float *host, size_t n) { return copy_block(m, m ? m->D.W[0] : nullptr, host, n); }
int mlp_get_grads(mlp_ctx *m, float *host, size_t n) { return copy_block(m, m ? m->D.gW[0] : nullptr, host, n); }

int mlp_forward(mlp_ctx *m, const float *x_dev, float *y_dev, int rows) {
  if (!m) return SPH_E_ORDER;
  if (!x_dev || !y_dev || rows < 1 || rows > m->D.max_rows) return SPH_E_ARG;
  mlp_launch_forward(m->D, x_dev, y_dev, rows, false, m->stream);
  return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
}

int mlp_backward(mlp_ctx *m, const float *x_dev, const float *t_dev, int rows, double *loss_host) {
  if (!m) return SPH_E_ORDER;
  if (!x_dev || !t_dev || rows < 1 || rows > m->D.max_rows) return SPH_E_ARG;
  const MlpDev &D = m->D;
  hipStream_t st = m->stream;
  mlp_launch_forward(D, x_dev, nullptr, rows, true, st);
  int nparts = (rows * kMlpOut + 255) / 256;
  hipLaunchKernelGGL(k_mlp_out_err, dim3(nparts), dim3(256), 0, st, D, t_dev, rows);
  hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, st, D, nparts, rows);
  const int tiles = (rows + kMlpTile - 1) / kMlpTile, chunks = (rows + kMlpChunk - 1) / kMlpChunk;
  auto sum_parts = [&](int l) {
    int KN = mlp_K(l) * mlp_N(l), N = mlp_N(l);
    hipLaunchKernelGGL(k_mlp_sum_parts, dim3((KN + N + 255) / 256), dim3(256), 0, st, D.partW, D.partb, D.gW[l],
                       D.gb[l], KN, N, chunks);
  };
  // layer 4 (output): error d0 (rows x 16)
  hipLaunchKernelGGL((k_mlp_back_weight<kMlpHid, kMlpOut>), dim3(chunks), dim3(256), (wgt_lds_bytes<kMlpHid, kMlpOut>()),
                     st, D.hin[3], D.d0, D.partW, D.partb, rows);
  sum_parts(3);
  hipLaunchKernelGGL((k_mlp_back_err<kMlpHid, kMlpOut>), dim3(tiles), dim3(256), (err_lds_bytes<kMlpHid, kMlpOut>()),
                     st, D.Wbf[3], D.d0, D.z[2], D.d1, rows);
  // layer 3: error d1 (rows x 128)
  hipLaunchKernelGGL((k_mlp_back_weight<kMlpHid, kMlpHid>), dim3(chunks), dim3(256), (wgt_lds_bytes<kMlpHid, kMlpHid>()),
                     st, D.hin[2], D.d1, D.partW, D.partb, rows);
  sum_parts(2);
  hipLaunchKernelGGL((k_mlp_back_err<kMlpHid, kMlpHid>), dim3(tiles), dim3(256), (err_lds_bytes<kMlpHid, kMlpHid>()),
                     st, D.Wbf[2], D.d1, D.z[1], D.d0, rows);
  // layer 2: error d0 (rows x 128)
  hipLaunchKernelGGL((k_mlp_back_weight<kMlpHid, kMlpHid>), dim3(chunks), dim3(256), (wgt_lds_bytes<kMlpHid, kMlpHid>()),
                     st, D.hin[1], D.d0, D.partW, D.partb, rows);
  sum_parts(1);
  hipLaunchKernelGGL((k_mlp_back_err<kMlpHid, kMlpHid>), dim3(tiles), dim3(256), (err_lds_bytes<kMlpHid, kMlpHid>()),
                     st, D.Wbf[1], D.d0, D.z[0], D.d1, rows);
  // layer 1: error d1 (rows x 128); the input error is not needed
  hipLaunchKernelGGL((k_mlp_back_weight<kMlpIn, kMlpHid>), dim3(chunks), dim3(256), (wgt_lds_bytes<kMlpIn, kMlpHid>()),
                     st, D.hin[0], D.d1, D.partW, D.partb, rows);
  sum_parts(0);
  if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
  if (loss_host) {
    if (hipMemcpyAsync(loss_host, D.loss, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SPH_E_HIP;
  }
  return SPH_OK;
}

int mlp_adam(mlp_ctx *m, float lr, float beta1, float beta2, float eps) {
  if (!m) return SPH_E_ORDER;
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return SPH_E_ARG;
  m->step += 1;
  float c1 = 1.0f - (float)std::pow((double)beta1, m->step), c2 = 1.0f - (float)std::pow((double)beta2, m->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kParamsPadded + 255) / 256), dim3(256), 0, m->stream, m->D.W[0], m->D.mW[0],
                     m->D.vW[0], m->D.gW[0], kParamsPadded, lr, beta1, beta2, eps, c1, c2);
  return refresh_bf16(m);
}

int mlp_train_step(mlp_ctx *m, const float *x_dev, const float *t_dev, int rows, float lr, float beta1, float beta2,
                   float eps, double *loss_host) {
  int rc = mlp_backward(m, x_dev, t_dev, rows, nullptr);
  if (rc != SPH_OK) return rc;
  rc = mlp_adam(m, lr, beta1, beta2, eps);
  if (rc != SPH_OK || !loss_host) return rc;
  if (hipMemcpyAsync(loss_host, m->D.loss, sizeof(double), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return SPH_E_HIP;
  return SPH_OK;
}

int mlp_sync(mlp_ctx *m) {
  if (!m) return SPH_E_ORDER;
  return hipStreamSynchronize(m->stream) == hipSuccess ? SPH_OK : SPH_E_HIP;
}

void mlp_destroy(mlp_ctx *m) { delete m; }

}  // extern "C"
