// Internal interface of the network kernels (not part of the C ABI).
//
// Every tensor the convolutions read is stored channel-last with a zero halo:
// the logical grid D x H x W sits at offset 1 inside Dp x Hp x Wp with
// Dp = round_up(D, 4) + 2 (same for H, W), so the 27 taps of every voxel of
// a 4 x 4 x 4 output tile read memory without bounds tests.  Kernels only ever
// write logical voxels; the rest stays zero from allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace q1 {

using bf16 = uint16_t;  // bfloat16 bit pattern

struct PGrid {
  int B = 0, D = 0, H = 0, W = 0, Dp = 0, Hp = 0, Wp = 0;
  __host__ __device__ PGrid() {}
  __host__ __device__ PGrid(int b, int d, int h, int w)
      : B(b), D(d), H(h), W(w), Dp(((d + 3) & ~3) + 2), Hp(((h + 3) & ~3) + 2),
        Wp(((w + 3) & ~3) + 2) {}
  // voxel index of logical (b, z, y, x); -1 and the round-up region address the halo
  __host__ __device__ int64_t at(int b, int z, int y, int x) const {
    return ((int64_t(b) * Dp + z + 1) * Hp + y + 1) * Wp + x + 1;
  }
  __host__ __device__ int64_t voxels() const { return int64_t(B) * Dp * Hp * Wp; }
  __host__ __device__ PGrid half() const { return PGrid(B, D / 2, H / 2, W / 2); }
  __host__ __device__ PGrid twice() const { return PGrid(B, 2 * D, 2 * H, 2 * W); }
};

// Channel window of a padded tensor: channels [co, co + n) of a tensor whose
// voxels hold cs channels.
struct Slice {
  bf16 *p = nullptr;
  int cs = 0, co = 0;
};

// 3x3x3 convolution with zero padding on a padded input of cin channels.
struct ConvArgs {
  const bf16 *x = nullptr;
  int cin = 0;
  PGrid g;                    // input and output grid
  const bf16 *wp = nullptr;   // packed weights [nchunks*4][cout][8], chunk-major K order
  int ngroups = 0, nchunks = 0, cout = 0;  // nchunks: K-steps (conv_ksteps(cin))
  const float *bias = nullptr;  // [cout] or null
  int relu = 0;
  Slice mask;                   // outputs where mask <= 0 become 0 (same grid), or p == null
  Slice out;                    // BF16 output channels [co, co + cout), or p == null
  int out_up = 0;               // write each value to the 8 children on the doubled grid
  float *o32 = nullptr;         // FP32 output [padded V][split or cout]
  int split = 0;
  float *o32b = nullptr;        // FP32 channels [split, cout) when split > 0
};

// Gradient of the weights: dW[t][ci][co] = sum_v X[v + d_t][ci] G[v][co] and
// db[co] = sum_v G[v][co] over the logical voxels.
struct ConvWArgs {
  const bf16 *x = nullptr;
  int cin = 0;
  PGrid g;
  const bf16 *gy = nullptr;  // padded [V][cout]
  int cout = 0;
  int cin_real = 0;  // input channels that have weights (<= cin)
  int nchunks = 0;   // brick chunks, one partial sum each
  float *part = nullptr;   // [nchunks][27][cin_real][cout]
  float *bpart = nullptr;  // [nchunks][cout]
};

int conv_forward(const ConvArgs &a, hipStream_t s);
// K-steps (4 groups of 8 channels each) of a convolution over cin input
// channels in the chunk-major order of the packed weights
int conv_ksteps(int cin);
int wgrad_chunks(const ConvWArgs &a);
int conv_wgrad(ConvWArgs a, float *gw, float *gb, hipStream_t s);
int pack_forward(const float *W, int cin_real, int cin_pad, int cout, int ngroups_pad, bf16 *wp,
                 hipStream_t s);
int pack_backward(const float *W, int cin, int cout, int ngroups_pad, bf16 *wq, hipStream_t s);
// unpadded [B][D][H][W][ca] (or its half grid when up_a) and [..][cb] -> padded concatenation
int gather_padded(const bf16 *a, int ca, int up_a, const bf16 *b, int cb, const PGrid &g, bf16 *out,
                  hipStream_t s);
// padded FP32 [V][C] -> unpadded [B][D][H][W][C]
int unpad_f32(const float *in, const PGrid &g, int C, float *out, hipStream_t s);
int pool2(Slice in, const PGrid &fine, int C, bf16 *out, hipStream_t s);
int up_adjoint_mask(const float *gup, Slice mask_fine, const PGrid &coarse, int C, bf16 *out,
                    hipStream_t s);
int pool_adjoint_add_mask(const float *gskip, const float *gp, Slice mask, const PGrid &fine,
                          int C, bf16 *out, hipStream_t s);
int head_forward(const bf16 *t, const PGrid &g, const float *wh, float *out, hipStream_t s);
int head_backward(const float *dout, const bf16 *t, const PGrid &g, const float *wh, bf16 *gpre,
                  float *part, int nblk, float *gwh, hipStream_t s);
int mse(const float *out, const float *tgt, const float *wgt, int64_t n, double *part, int nblk,
        float *dout, float *loss, hipStream_t s);
int adam(float *th, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
         float eps, int step, hipStream_t s);

}  // namespace q1
