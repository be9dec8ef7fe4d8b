// Device building blocks of the surrogate network's passes on the gfx950
// matrix cores, shared by the network's own kernels and the solver's fused
// surrogate pass: bfloat16 conversion, SiLU, the LDS operand layout and the
// per-wave 16-row product of a layer.
//
// Matrix-core operand layout (16x16x32, wave64):
//   A (16 x 32, rows x k):  lane l holds A[l % 16][8 (l / 16) + j], j = 0..7
//   B (32 x 16, k x cols):  lane l holds B[8 (l / 16) + j][l % 16]
//   D (16 x 16):            lane l holds D[4 (l / 16) + j][l % 16]
// (the error pass through the 16-wide output layer uses the 16-deep form,
// v_mfma_f32_16x16x16_bf16, with 4 of k per lane: A[l % 16][4 (l / 16) + j]).
// Every operand fragment is 8 consecutive bfloat16 in an LDS row (one 16-byte
// read): the forward pass keeps W transposed (N x K), the error pass keeps W
// (K x N), the weight-gradient pass transposes its tiles while staging them.
#pragma once
#include <hip/hip_runtime.h>

#include "mlp_internal.h"

namespace mrsph {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// D += A B over one 16 x 16 x 32 tile (operands as 8 raw bfloat16 per lane)
__device__ __forceinline__ f4 mfma_bf16(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}

// bfloat16 of an FP32 value, nearest with ties to even (NaN stays NaN)
__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoidf(z); }
__device__ __forceinline__ float silu_grad(float z) {
  float s = sigmoidf(z);
  return s * (1.0f + z * (1.0f - s));
}

// LDS row pitch in bfloat16 elements: 8 extra elements shift consecutive rows
// by four banks and keep the 16-byte alignment of the operand reads.
constexpr int pitch(int k) { return k + 8; }

constexpr int kParamsPadded = kMlpIn * kMlpHid + kMlpHid + 2 * (kMlpHid * kMlpHid + kMlpHid) + kMlpHid * kMlpOut +
                              kMlpOut;

__device__ __forceinline__ s8 lds8(const unsigned short *p) { return *reinterpret_cast<const s8 *>(p); }

// Copy a K-wide row-major bfloat16 matrix of `rows` rows into LDS rows of pitch(K).
__device__ __forceinline__ void stage_rows(const unsigned short *src, unsigned short *dst, int rows, int K) {
  const int per = K / 4;
  for (int idx = threadIdx.x; idx < rows * per; idx += blockDim.x) {
    int r = idx / per, c = (idx - r * per) * 4;
    *reinterpret_cast<s4 *>(dst + r * pitch(K) + c) = *reinterpret_cast<const s4 *>(src + (size_t)r * K + c);
  }
}

// One wave: D (16 rows starting at r0, N cols) = Hin (pitch(K)) x W, with W^T
// (N rows of pitch(K)) in LDS.
template <int K, int N>
__device__ __forceinline__ void wave_gemm_fwd(const unsigned short *Hin, const unsigned short *WT, int r0, f4 *acc) {
  constexpr int NT = N / 16;
  const int l = threadIdx.x & 63, kq = (l >> 4) * 8;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    s8 a = lds8(Hin + (r0 + (l & 15)) * pitch(K) + k0 + kq);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      s8 b = lds8(WT + (nt * 16 + (l & 15)) * pitch(K) + k0 + kq);
      acc[nt] = mfma_bf16(a, b, acc[nt]);
    }
  }
}

// Hidden-layer epilogue: bias, SiLU, bfloat16 into the next LDS buffer; with
// train, the pre-activation and the next layer's input go to global memory.
template <bool TRAIN>
__device__ __forceinline__ void hidden_epilogue(const f4 *acc, const float *bias, unsigned short *Hout, int r0,
                                                int row0, int rows, float *zg, unsigned short *hg) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int nt = 0; nt < kMlpHid / 16; ++nt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = r0 + (l >> 4) * 4 + j, c = nt * 16 + (l & 15);
      float z = acc[nt][j] + bias[c];
      unsigned short h = f2bf(silu(z));
      Hout[r * pitch(kMlpHid) + c] = h;
      if (TRAIN && row0 + r < rows) {
        zg[(size_t)(row0 + r) * kMlpHid + c] = z;
        hg[(size_t)(row0 + r) * kMlpHid + c] = h;
      }
    }
}

// LDS of a forward pass over one tile: the four transposed weight matrices,
// two activation tiles and the biases.
constexpr size_t fwd_lds_bytes() {
  return sizeof(unsigned short) * (size_t)(kMlpHid * pitch(kMlpIn) + 2 * kMlpHid * pitch(kMlpHid) +
                                           kMlpOut * pitch(kMlpHid) + 2 * kMlpTile * pitch(kMlpHid)) +
         sizeof(float) * (3 * kMlpHid + kMlpOut);
}

// Stage the network's weights (bfloat16, transposed) and biases into the
// forward pass's LDS layout; returns the two activation tiles and the biases.
struct FwdLds {
  unsigned short *WT0, *WT1, *WT2, *WT3, *HA, *HB;
  float *bias;
};
__device__ __forceinline__ FwdLds fwd_lds_layout(unsigned short *lds) {
  FwdLds L;
  L.WT0 = lds;                                 // 128 x pitch(32)
  L.WT1 = L.WT0 + kMlpHid * pitch(kMlpIn);     // 128 x pitch(128)
  L.WT2 = L.WT1 + kMlpHid * pitch(kMlpHid);    // 128 x pitch(128)
  L.WT3 = L.WT2 + kMlpHid * pitch(kMlpHid);    // 16 x pitch(128)
  L.HA = L.WT3 + kMlpOut * pitch(kMlpHid);     // 64 x pitch(128)
  L.HB = L.HA + kMlpTile * pitch(kMlpHid);     // 64 x pitch(128)
  L.bias = reinterpret_cast<float *>(L.HB + kMlpTile * pitch(kMlpHid));  // 3 x 128 + 16
  return L;
}
__device__ __forceinline__ void stage_weights(const MlpDev &M, const FwdLds &L) {
  stage_rows(M.WTbf[0], L.WT0, kMlpHid, kMlpIn);
  stage_rows(M.WTbf[1], L.WT1, kMlpHid, kMlpHid);
  stage_rows(M.WTbf[2], L.WT2, kMlpHid, kMlpHid);
  stage_rows(M.WTbf[3], L.WT3, kMlpOut, kMlpHid);
  for (int i = threadIdx.x; i < 3 * kMlpHid + kMlpOut; i += blockDim.x)
    L.bias[i] = i < 3 * kMlpHid ? M.b[i / kMlpHid][i % kMlpHid] : M.b[3][i - 3 * kMlpHid];
}

// The four layers over the tile whose input (bfloat16, pitch(kMlpIn)) is in
// L.HA, after a barrier; each wave owns 16 rows.  Returns the wave's output
// fragment (pre-bias): lane l holds rows r0 + 4 (l / 16) + j, column l % 16.
template <bool TRAIN>
__device__ __forceinline__ f4 forward_tile(const FwdLds &L, const MlpDev &M, int row0, int rows) {
  const int r0 = (threadIdx.x >> 6) * 16;
  f4 acc[kMlpHid / 16];
  wave_gemm_fwd<kMlpIn, kMlpHid>(L.HA, L.WT0, r0, acc);
  hidden_epilogue<TRAIN>(acc, L.bias, L.HB, r0, row0, rows, M.z[0], M.hin[1]);
  __syncthreads();
  wave_gemm_fwd<kMlpHid, kMlpHid>(L.HB, L.WT1, r0, acc);
  __syncthreads();  // HA is overwritten below while other waves may still read HB only
  hidden_epilogue<TRAIN>(acc, L.bias + kMlpHid, L.HA, r0, row0, rows, M.z[1], M.hin[2]);
  __syncthreads();
  wave_gemm_fwd<kMlpHid, kMlpHid>(L.HA, L.WT2, r0, acc);
  __syncthreads();
  hidden_epilogue<TRAIN>(acc, L.bias + 2 * kMlpHid, L.HB, r0, row0, rows, M.z[2], M.hin[3]);
  __syncthreads();
  f4 out[1];
  wave_gemm_fwd<kMlpHid, kMlpOut>(L.HB, L.WT3, r0, out);
  return out[0];
}

}  // namespace mrsph
