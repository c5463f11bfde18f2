// BF16 matrix-core kernels of the learned preconditioner's network: 3x3x3
// convolution forward, its adjoint in the data (backward-data) and its
// gradient in the weights (backward-weight), all with FP32 accumulation on
// v_mfma_f32_16x16x32_bf16, plus the elementwise kernels around them
// (pooling, upsampling adjoints, ReLU masks, the 1x1 head, the loss, Adam,
// weight packing).
//
// Tensors are channel-last [B][D][H][W][C] (z, y, x, channel) with C a
// multiple of 8, so 8 channels of one voxel are one 16-byte load.  A
// convolution is the implicit GEMM  Y^T (Cout x V) = Wp (Cout x K) * X^T (K x V)
// with K = 27 taps x Cin in groups of 8 channels: group g = tap * Cin/8 + cg.
// The 16x16x32 instruction takes, per lane l, 8 consecutive K of row l%16 of
// the first operand and 8 consecutive K of column l%16 of the second, K-block
// l/16; so each lane loads one group (16 bytes) of the packed weights for its
// output channel and one group of the shifted input voxel for its voxel.  The
// result holds 4 consecutive output channels of one voxel per lane.
//
// Backward-data is the same kernel: the adjoint of a 3x3x3 correlation is
// the correlation with the tap-reversed kernel and transposed channel blocks,
// so only the weight packing differs.  Backward-weight contracts over voxels
// (K = 32 voxels per instruction), with the gradient block as the first
// operand (rows = output channels) and the shifted input as the second
// (columns = input channels); one wavefront keeps all 27 taps' accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "q1_conv.hpp"
#include "q1_internal.hpp"

namespace q1 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(unsigned short u) { return __uint_as_float(unsigned(u) << 16); }
__device__ __forceinline__ unsigned short f2bf(float f) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}
__device__ __forceinline__ bf16x8 ld8(const bf16 *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}

// ---- convolution forward / backward-data ---------------------------------------

constexpr int kZB = 4;  // z-slices per wavefront tile (tile: 4 x 4 x kZB voxels)

template <int NB>  // NB = Cout / 16
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int TX = (a.W + 3) >> 2, TY = (a.H + 3) >> 2, TZ = (a.D + kZB - 1) / kZB;
  const int64_t ntiles = int64_t(a.B) * TZ * TY * TX;
  if (wave >= ntiles) return;
  int64_t t = wave;
  const int tx = int(t % TX);
  t /= TX;
  const int ty = int(t % TY);
  t /= TY;
  const int tz = int(t % TZ);
  const int b = int(t / TZ);
  const int kg = lane >> 4, j = lane & 15;
  const int vx = tx * 4 + (j & 3), vy = ty * 4 + (j >> 2), z0 = tz * kZB;
  const int CG = (a.ca + a.cb) >> 3, CGA = a.ca >> 3;
  const int Dc = a.D >> 1, Hc = a.H >> 1, Wc = a.W >> 1;
  f32x4 acc[NB][kZB];
#pragma unroll
  for (int r = 0; r < NB; ++r)
#pragma unroll
    for (int z = 0; z < kZB; ++z) acc[r][z] = f32x4{0.f, 0.f, 0.f, 0.f};
  int tap = 0, cg = kg;
  while (cg >= CG) {
    cg -= CG;
    ++tap;
  }
  const bf16 *wrow = a.wp + size_t(j) * 8;
  for (int c = 0; c < a.nchunks; ++c) {
    const int g = 4 * c + kg;
    bf16x8 wv[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) wv[r] = ld8(wrow + (size_t(g) * a.cout + r * 16) * 8);
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int x = vx + dx, y = vy + dy;
    const bool inxy = g < a.ngroups && x >= 0 && x < a.W && y >= 0 && y < a.H;
    bf16x8 xv[kZB];
#pragma unroll
    for (int zb = 0; zb < kZB; ++zb) {
      const int z = z0 + zb + dz;
      if (inxy && z >= 0 && z < a.D) {
        const bf16 *src;
        if (cg < CGA) {
          src = a.up_a ? a.a + ((((size_t)b * Dc + (z >> 1)) * Hc + (y >> 1)) * Wc + (x >> 1)) * a.ca
                       : a.a + ((((size_t)b * a.D + z) * a.H + y) * a.W + x) * a.ca;
          src += cg * 8;
        } else {
          src = a.b + ((((size_t)b * a.D + z) * a.H + y) * a.W + x) * a.cb + (cg - CGA) * 8;
        }
        xv[zb] = ld8(src);
      } else {
        xv[zb] = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
      for (int zb = 0; zb < kZB; ++zb)
        acc[r][zb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[r], xv[zb], acc[r][zb], 0, 0, 0);
    cg += 4;
    while (cg >= CG) {
      cg -= CG;
      ++tap;
    }
  }
  // epilogue: lane holds output channels r*16 + 4*kg + i of voxel (vx, vy, z0 + zb)
  if (vx >= a.W || vy >= a.H) return;
#pragma unroll
  for (int zb = 0; zb < kZB; ++zb) {
    const int z = z0 + zb;
    if (z >= a.D) break;
    const size_t vox = (((size_t)b * a.D + z) * a.H + vy) * a.W + vx;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int c0 = r * 16 + kg * 4;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = acc[r][zb][i] + (a.bias ? a.bias[c0 + i] : 0.f);
        if (a.relu) v[i] = fmaxf(v[i], 0.f);
      }
      if (a.mask) {
        const bf16 *m = a.mask + vox * a.cout + c0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (!(bf2f(m[i]) > 0.f)) v[i] = 0.f;
      }
      if (a.out_bf) {
        ushort4 o{f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
        *reinterpret_cast<ushort4 *>(a.out_bf + vox * a.cout + c0) = o;
      }
      if (a.out_f32) {
        float4 o{v[0], v[1], v[2], v[3]};
        if (a.split == 0)
          *reinterpret_cast<float4 *>(a.out_f32 + vox * a.cout + c0) = o;
        else if (c0 < a.split)
          *reinterpret_cast<float4 *>(a.out_f32 + vox * a.split + c0) = o;
        else
          *reinterpret_cast<float4 *>(a.out2_f32 + vox * (a.cout - a.split) + (c0 - a.split)) = o;
      }
    }
  }
}

// ---- convolution backward-weight ---------------------------------------------------
// Bricks of 4 (x) x 4 (y) x 2 (z) voxels: K-block kg of a lane covers the 8
// voxels x = 0..3, y = 2 (kg & 1) + {0, 1}, z = kg >> 1 of the brick.

__device__ __forceinline__ unsigned short wg_load_x(const ConvWArgs &a, int b, int x, int y, int z,
                                                    int ci) {
  if (ci >= a.ca + a.cb || x < 0 || x >= a.W || y < 0 || y >= a.H || z < 0 || z >= a.D) return 0;
  if (ci < a.ca) {
    if (a.up_a)
      return a.a[((((size_t)b * (a.D >> 1) + (z >> 1)) * (a.H >> 1) + (y >> 1)) * (a.W >> 1) +
                   (x >> 1)) *
                      a.ca +
                  ci];
    return a.a[((((size_t)b * a.D + z) * a.H + y) * a.W + x) * a.ca + ci];
  }
  return a.b[((((size_t)b * a.D + z) * a.H + y) * a.W + x) * a.cb + (ci - a.ca)];
}

__global__ __launch_bounds__(256) void k_conv_wgrad(ConvWArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int nrb = a.cout >> 4, ncb = (a.ca + a.cb + 15) >> 4;
  if (wave >= int64_t(a.nchunks) * nrb * ncb) return;
  const int rbo = int(wave % nrb);
  const int cbi = int((wave / nrb) % ncb);
  const int ch = int(wave / (int64_t(nrb) * ncb));
  const int kg = lane >> 4, j = lane & 15;
  const int BX = (a.W + 3) >> 2, BY = (a.H + 3) >> 2, BZ = (a.D + 1) >> 1;
  const int64_t nbr = int64_t(a.B) * BZ * BY * BX;
  const int64_t br0 = nbr * ch / a.nchunks, br1 = nbr * (ch + 1) / a.nchunks;
  const int co = rbo * 16 + j, ci = cbi * 16 + j;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int64_t br = br0; br < br1; ++br) {
    int64_t q = br;
    const int bx = int(q % BX) * 4;
    q /= BX;
    const int by = int(q % BY) * 4 + 2 * (kg & 1);
    q /= BY;
    const int bz = int(q % BZ) * 2 + (kg >> 1);
    const int b = int(q / BZ);
    u16x8 gu;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int x = bx + (i & 3), y = by + (i >> 2);
      gu[i] = (x < a.W && y < a.H && bz < a.D)
                  ? a.g[((((size_t)b * a.D + bz) * a.H + y) * a.W + x) * a.cout + co]
                  : (unsigned short)0;
      bsum += bf2f(gu[i]);
    }
    const bf16x8 gv = __builtin_bit_cast(bf16x8, gu);
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      u16x8 xu;
#pragma unroll
      for (int i = 0; i < 8; ++i) xu[i] = wg_load_x(a, b, bx + (i & 3) + dx, by + (i >> 2) + dy, bz + dz, ci);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gv, __builtin_bit_cast(bf16x8, xu), acc[t],
                                                       0, 0, 0);
    }
  }
  // rows = output channels rbo*16 + 4*kg + i, column = input channel ci
  if (ci < a.cin_real) {
    const size_t nk = size_t(27) * a.cin_real * a.cout;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      float *p = a.part + ch * nk + (size_t(t) * a.cin_real + ci) * a.cout + rbo * 16 + kg * 4;
      *reinterpret_cast<float4 *>(p) = float4{acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
    }
  }
  if (cbi == 0) {
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (kg == 0) a.bpart[size_t(ch) * a.cout + co] = bsum;
  }
}

// out[k] = sum over c < nparts of part[c * n + k] (fixed order)
__global__ void k_sum_parts(const float *__restrict__ part, int nparts, int64_t n,
                            float *__restrict__ out) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float s = 0.f;
  for (int c = 0; c < nparts; ++c) s += part[c * n + k];
  out[k] = s;
}

// ---- weight packing ----------------------------------------------------------------------

// forward: wp[g][co][jj] = W[tap][cg*8 + jj][co] with g = tap*CG + cg; zero past the
// real groups and channels.  W is [27][cin_real][cout] FP32.
__global__ void k_pack_fwd(const float *__restrict__ W, int cin_real, int cin_pad, int cout,
                           int ngroups_pad, bf16 *__restrict__ wp) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(ngroups_pad) * cout * 8;
  if (i >= n) return;
  const int jj = int(i & 7);
  const int co = int((i >> 3) % cout);
  const int g = int((i >> 3) / cout);
  const int CG = cin_pad >> 3;
  const int tap = g / CG, c = (g % CG) * 8 + jj;
  const float v = (tap < 27 && c < cin_real) ? W[(size_t(tap) * cin_real + c) * cout + co] : 0.f;
  wp[i] = f2bf(v);
}

// backward-data: the correlation with reversed taps and swapped channels,
// wq[g][ci][jj] = W[26 - tap][ci][cg*8 + jj] with g = tap*(cout/8) + cg.
__global__ void k_pack_bwd(const float *__restrict__ W, int cin, int cout, int ngroups_pad,
                           bf16 *__restrict__ wq) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(ngroups_pad) * cin * 8;
  if (i >= n) return;
  const int jj = int(i & 7);
  const int ci = int((i >> 3) % cin);
  const int g = int((i >> 3) / cin);
  const int CG = cout >> 3;
  const int tap = g / CG, co = (g % CG) * 8 + jj;
  const float v = tap < 27 ? W[(size_t(26 - tap) * cin + ci) * cout + co] : 0.f;
  wq[i] = f2bf(v);
}

// ---- pooling, upsampling adjoints, masks -----------------------------------------------

// 2x2x2 average pooling, [B][D][H][W][C] -> [B][D/2][H/2][W/2][C]
__global__ void k_pool2(const bf16 *__restrict__ in, int B, int D, int H, int W, int C,
                        bf16 *__restrict__ out) {
  const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(B) * Dc * Hc * Wc * C;
  if (i >= n) return;
  const int c = int(i % C);
  int64_t v = i / C;
  const int x = int(v % Wc) * 2;
  v /= Wc;
  const int y = int(v % Hc) * 2;
  v /= Hc;
  const int z = int(v % Dc) * 2;
  const int b = int(v / Dc);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    s += bf2f(in[((((size_t)b * D + z + (k >> 2)) * H + y + ((k >> 1) & 1)) * W + x + (k & 1)) * C + c]);
  out[i] = f2bf(s * 0.125f);
}

// coarse gpre = (sum of the 8 children of gup) * (mask > 0), gup FP32 fine, mask/out coarse
__global__ void k_up_adjoint_mask(const float *__restrict__ gup, const bf16 *__restrict__ mask,
                                  int B, int Dc, int Hc, int Wc, int C, bf16 *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(B) * Dc * Hc * Wc * C;
  if (i >= n) return;
  const int c = int(i % C);
  int64_t v = i / C;
  const int x = int(v % Wc) * 2;
  v /= Wc;
  const int y = int(v % Hc) * 2;
  v /= Hc;
  const int z = int(v % Dc) * 2;
  const int b = int(v / Dc);
  const int D = 2 * Dc, H = 2 * Hc, W = 2 * Wc;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    s += gup[((((size_t)b * D + z + (k >> 2)) * H + y + ((k >> 1) & 1)) * W + x + (k & 1)) * C + c];
  out[i] = f2bf(bf2f(mask[i]) > 0.f ? s : 0.f);
}

// fine gpre = (gskip + gp[parent] / 8) * (mask > 0)
__global__ void k_pool_adjoint_add_mask(const float *__restrict__ gskip,
                                        const float *__restrict__ gp,
                                        const bf16 *__restrict__ mask, int B, int D, int H, int W,
                                        int C, bf16 *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(B) * D * H * W * C;
  if (i >= n) return;
  const int c = int(i % C);
  int64_t v = i / C;
  const int x = int(v % W);
  v /= W;
  const int y = int(v % H);
  v /= H;
  const int z = int(v % D);
  const int b = int(v / D);
  const float p = gp[((((size_t)b * (D >> 1) + (z >> 1)) * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1)) * C + c];
  const float s = gskip[i] + 0.125f * p;
  out[i] = f2bf(bf2f(mask[i]) > 0.f ? s : 0.f);
}

// ---- head, loss -------------------------------------------------------------------------

// out[v] = sum_c t[v][c] wh[c] + bh
__global__ void k_head_fwd(const bf16 *__restrict__ t, int C, int64_t nv,
                           const float *__restrict__ wh, float *__restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  float s = wh[C];
  for (int c = 0; c < C; ++c) s += bf2f(t[v * C + c]) * wh[c];
  out[v] = s;
}

constexpr int kHB = 256;  // threads per block of the head / loss reductions

// gpre[v][c] = dout[v] wh[c] (t[v][c] > 0); per-block partials of
// dL/dwh[c] = sum_v dout[v] t[v][c] and dL/dbh = sum_v dout[v]
__global__ __launch_bounds__(kHB) void k_head_bwd(const float *__restrict__ dout,
                                                 const bf16 *__restrict__ t, int64_t nv,
                                                 const float *__restrict__ wh,
                                                 bf16 *__restrict__ gpre,
                                                 float *__restrict__ part /*[nblk][17]*/) {
  constexpr int C = 16;
  __shared__ float sh[C + 1][kHB / 64];
  float acc[C + 1];
#pragma unroll
  for (int c = 0; c <= C; ++c) acc[c] = 0.f;
  for (int64_t v = int64_t(blockIdx.x) * kHB + threadIdx.x; v < nv; v += int64_t(gridDim.x) * kHB) {
    const float d = dout[v];
    acc[C] += d;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float tv = bf2f(t[v * C + c]);
      acc[c] += d * tv;
      gpre[v * C + c] = f2bf(tv > 0.f ? d * wh[c] : 0.f);
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c <= C; ++c) {
    float s = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) sh[c][w] = s;
  }
  __syncthreads();
  if (threadIdx.x <= C) {
    float s = 0.f;
    for (int k = 0; k < kHB / 64; ++k) s += sh[threadIdx.x][k];
    part[blockIdx.x * (C + 1) + threadIdx.x] = s;
  }
}

// per-block partials of sum(weight) and sum(weight (out - target)^2)
__global__ __launch_bounds__(kHB) void k_mse_partials(const float *__restrict__ out,
                                                     const float *__restrict__ tgt,
                                                     const float *__restrict__ wgt, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double sh[2][kHB / 64];
  double a = 0.0, s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kHB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kHB) {
    const double d = double(out[i]) - double(tgt[i]);
    a += wgt[i];
    s += double(wgt[i]) * d * d;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    s += __shfl_xor(s, o);
  }
  if (lane == 0) {
    sh[0][w] = a;
    sh[1][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double r = 0.0;
    for (int k = 0; k < kHB / 64; ++k) r += sh[threadIdx.x][k];
    part[blockIdx.x * 2 + threadIdx.x] = r;
  }
}

// dout = 2 weight (out - target) / sum(weight); loss = sum(w d^2) / sum(w)
__global__ __launch_bounds__(kHB) void k_mse_grad(const float *__restrict__ out,
                                                 const float *__restrict__ tgt,
                                                 const float *__restrict__ wgt, int64_t n,
                                                 const double *__restrict__ part, int nparts,
                                                 float *__restrict__ dout,
                                                 float *__restrict__ loss) {
  double den = 0.0, num = 0.0;
  for (int k = 0; k < nparts; ++k) {
    den += part[2 * k];
    num += part[2 * k + 1];
  }
  const float scale = den > 0.0 ? float(2.0 / den) : 0.f;
  for (int64_t i = int64_t(blockIdx.x) * kHB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kHB)
    dout[i] = scale * wgt[i] * (out[i] - tgt[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) *loss = den > 0.0 ? float(num / den) : 0.f;
}

// ---- Adam --------------------------------------------------------------------------------

__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- host launchers ---------------------------------------------------------------------

static inline dim3 g1(int64_t n, int bs = 256) { return dim3(unsigned((n + bs - 1) / bs)); }

int conv_forward(const ConvArgs &a, hipStream_t s) {
  const int64_t ntiles = int64_t(a.B) * ((a.D + kZB - 1) / kZB) * ((a.H + 3) / 4) * ((a.W + 3) / 4);
  const dim3 grid(unsigned((ntiles + 3) / 4)), block(256);
  switch (a.cout) {
    case 16: hipLaunchKernelGGL(k_conv_fwd<1>, grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_conv_fwd<2>, grid, block, 0, s, a); break;
    case 48: hipLaunchKernelGGL(k_conv_fwd<3>, grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL(k_conv_fwd<4>, grid, block, 0, s, a); break;
    case 96: hipLaunchKernelGGL(k_conv_fwd<6>, grid, block, 0, s, a); break;
    default: return fail(Q1_EUNSUPPORTED, "conv: %d output channels (16, 32, 48, 64, 96)", a.cout);
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int wgrad_chunks(const ConvWArgs &a) {
  const int64_t nbr = int64_t(a.B) * ((a.D + 1) / 2) * ((a.H + 3) / 4) * ((a.W + 3) / 4);
  const int units = (a.cout / 16) * ((a.ca + a.cb + 15) / 16);
  return int(std::max<int64_t>(1, std::min<int64_t>(nbr, std::max(1, 4096 / units))));
}

int conv_wgrad(ConvWArgs a, float *gw, float *gb, hipStream_t s) {
  const int64_t waves = int64_t(a.nchunks) * (a.cout / 16) * ((a.ca + a.cb + 15) / 16);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, s, a);
  const int64_t nk = int64_t(27) * a.cin_real * a.cout;
  hipLaunchKernelGGL(k_sum_parts, g1(nk), dim3(256), 0, s, a.part, a.nchunks, nk, gw);
  hipLaunchKernelGGL(k_sum_parts, g1(a.cout), dim3(256), 0, s, a.bpart, a.nchunks,
                     int64_t(a.cout), gb);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pack_forward(const float *W, int cin_real, int cin_pad, int cout, int ngroups_pad, bf16 *wp,
                 hipStream_t s) {
  const int64_t n = int64_t(ngroups_pad) * cout * 8;
  hipLaunchKernelGGL(k_pack_fwd, g1(n), dim3(256), 0, s, W, cin_real, cin_pad, cout, ngroups_pad, wp);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pack_backward(const float *W, int cin, int cout, int ngroups_pad, bf16 *wq, hipStream_t s) {
  const int64_t n = int64_t(ngroups_pad) * cin * 8;
  hipLaunchKernelGGL(k_pack_bwd, g1(n), dim3(256), 0, s, W, cin, cout, ngroups_pad, wq);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pool2(const bf16 *in, int B, int D, int H, int W, int C, bf16 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2, g1(int64_t(B) * (D / 2) * (H / 2) * (W / 2) * C), dim3(256), 0, s,
                     in, B, D, H, W, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int up_adjoint_mask(const float *gup, const bf16 *mask, int B, int Dc, int Hc, int Wc, int C,
                    bf16 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_up_adjoint_mask, g1(int64_t(B) * Dc * Hc * Wc * C), dim3(256), 0, s, gup,
                     mask, B, Dc, Hc, Wc, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pool_adjoint_add_mask(const float *gskip, const float *gp, const bf16 *mask, int B, int D,
                          int H, int W, int C, bf16 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_adjoint_add_mask, g1(int64_t(B) * D * H * W * C), dim3(256), 0, s,
                     gskip, gp, mask, B, D, H, W, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int head_forward(const bf16 *t, int64_t nv, const float *wh, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_head_fwd, g1(nv), dim3(256), 0, s, t, 16, nv, wh, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int head_backward(const float *dout, const bf16 *t, int64_t nv, const float *wh, bf16 *gpre,
                  float *part, int nblk, float *gwh, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nblk), dim3(kHB), 0, s, dout, t, nv, wh, gpre, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, nblk, int64_t(17), gwh);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int mse(const float *out, const float *tgt, const float *wgt, int64_t n, double *part, int nblk,
        float *dout, float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse_partials, dim3(nblk), dim3(kHB), 0, s, out, tgt, wgt, n, part);
  hipLaunchKernelGGL(k_mse_grad, dim3(nblk), dim3(kHB), 0, s, out, tgt, wgt, n, part, nblk, dout,
                     loss);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int adam(float *th, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
         float eps, int step, hipStream_t s) {
  const float c1 = 1.f - std::pow(b1, float(step)), c2 = 1.f - std::pow(b2, float(step));
  hipLaunchKernelGGL(k_adam, g1(n), dim3(256), 0, s, th, g, m, v, n, lr, b1, b2, eps, c1, c2);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace q1
