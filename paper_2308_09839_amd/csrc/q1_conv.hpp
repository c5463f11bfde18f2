// Internal interface of the network kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace q1 {

using bf16 = uint16_t;  // bfloat16 bit pattern

// 3x3x3 convolution with zero padding over [B][D][H][W][C] tensors.  The input
// is the channel concatenation of a (ca channels; read at the parent voxel of
// the half-resolution grid when up_a is set) and b (cb channels, may be 0).
// Output channel count cout is 16, 32, 48, 64 or 96.
struct ConvArgs {
  const bf16 *a = nullptr, *b = nullptr;
  int ca = 0, cb = 0, up_a = 0;
  int B = 0, D = 0, H = 0, W = 0;
  const bf16 *wp = nullptr;  // packed weights [nchunks*4][cout][8]
  int ngroups = 0, nchunks = 0, cout = 0;
  const float *bias = nullptr;  // [cout] or null
  int relu = 0;
  const bf16 *mask = nullptr;  // [V][cout]: outputs where mask <= 0 are set to 0
  bf16 *out_bf = nullptr;      // [V][cout]
  float *out_f32 = nullptr;    // [V][cout], or [V][split] when split > 0
  int split = 0;
  float *out2_f32 = nullptr;   // [V][cout - split]
};

// Gradient of the weights: dW[t][ci][co] = sum_v X[v + d_t][ci] G[v][co] and
// db[co] = sum_v G[v][co], X read as in ConvArgs.
struct ConvWArgs {
  const bf16 *a = nullptr, *b = nullptr;
  int ca = 0, cb = 0, up_a = 0;
  int B = 0, D = 0, H = 0, W = 0;
  const bf16 *g = nullptr;  // [V][cout]
  int cout = 0;
  int cin_real = 0;  // input channels that have weights (<= ca + cb)
  int nchunks = 0;   // voxel chunks, one partial sum each
  float *part = nullptr;   // [nchunks][27][cin_real][cout]
  float *bpart = nullptr;  // [nchunks][cout]
};

int conv_forward(const ConvArgs &a, hipStream_t s);
int wgrad_chunks(const ConvWArgs &a);
int conv_wgrad(ConvWArgs a, float *gw, float *gb, hipStream_t s);
int pack_forward(const float *W, int cin_real, int cin_pad, int cout, int ngroups_pad, bf16 *wp,
                 hipStream_t s);
int pack_backward(const float *W, int cin, int cout, int ngroups_pad, bf16 *wq, hipStream_t s);
int pool2(const bf16 *in, int B, int D, int H, int W, int C, bf16 *out, hipStream_t s);
int up_adjoint_mask(const float *gup, const bf16 *mask, int B, int Dc, int Hc, int Wc, int C,
                    bf16 *out, hipStream_t s);
int pool_adjoint_add_mask(const float *gskip, const float *gp, const bf16 *mask, int B, int D,
                          int H, int W, int C, bf16 *out, hipStream_t s);
int head_forward(const bf16 *t, int64_t nv, const float *wh, float *out, hipStream_t s);
int head_backward(const float *dout, const bf16 *t, int64_t nv, const float *wh, bf16 *gpre,
                  float *part, int nblk, float *gwh, hipStream_t s);
int mse(const float *out, const float *tgt, const float *wgt, int64_t n, double *part, int nblk,
        float *dout, float *loss, hipStream_t s);
int adam(float *th, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
         float eps, int step, hipStream_t s);

}  // namespace q1
