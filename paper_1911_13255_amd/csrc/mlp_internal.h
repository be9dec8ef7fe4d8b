// Device layout of the surrogate network shared by the network kernels and
// the solver (which runs inference inside the solid step).
#pragma once
#include <hip/hip_runtime.h>

namespace mrsph {

constexpr int kMlpIn = 32;      // padded input width (in_dim <= 32)
constexpr int kMlpHid = 128;    // hidden width
constexpr int kMlpOut = 16;     // padded output width (out_dim <= 16)
constexpr int kMlpLayers = 4;
constexpr int kMlpTile = 64;    // rows per workgroup in the forward and error passes
constexpr int kMlpChunk = 128;  // rows per partial weight gradient

constexpr int mlp_K(int l) { return l == 0 ? kMlpIn : kMlpHid; }
constexpr int mlp_N(int l) { return l == kMlpLayers - 1 ? kMlpOut : kMlpHid; }

struct MlpDev {
  int in_dim, out_dim, max_rows;
  // FP32 master parameters, padded: W[l] is K_l x N_l row-major, b[l] has N_l
  float *W[kMlpLayers], *b[kMlpLayers];
  float *mW[kMlpLayers], *vW[kMlpLayers], *mb[kMlpLayers], *vb[kMlpLayers];  // Adam moments
  float *gW[kMlpLayers], *gb[kMlpLayers];                                     // gradients
  unsigned short *Wbf[kMlpLayers];   // bfloat16 W (K x N), error pass operand
  unsigned short *WTbf[kMlpLayers];  // bfloat16 W^T (N x K), forward operand
  // training activations (rows x width)
  unsigned short *hin[kMlpLayers];   // bfloat16 input of each layer
  float *z[kMlpLayers - 1];          // hidden pre-activations
  float *y;                          // output, rows x kMlpOut
  float *d0, *d1;                    // back-propagated errors, rows x kMlpHid
  float *partW, *partb;              // per-chunk partial gradients
  double *loss_part, *loss;
};

// y (rows x out_dim) = network(x (rows x in_dim)); with train the layer inputs,
// pre-activations and padded output are stored for the error pass.
void mlp_launch_forward(const MlpDev &M, const float *x, float *y, int rows, bool train, hipStream_t st);

}  // namespace mrsph

struct mlp_ctx {
  mrsph::MlpDev D;
  hipStream_t stream;
  int step;
  size_t nparam;
};
