// BF16 matrix-core kernels of the learned preconditioner's network: 3x3x3
// convolution forward, its adjoint in the data (backward-data) and its
// gradient in the weights (backward-weight), all with FP32 accumulation on
// v_mfma_f32_16x16x32_bf16, plus the elementwise kernels around them
// (pooling, upsampling adjoints, ReLU masks, the 1x1 head, the loss, Adam,
// weight packing).
//
// Tensors are channel-last with a zero halo (PGrid): 8 channels of one voxel
// are one 16-byte load and every tap of an output tile is in memory, so the
// inner loops have no bounds tests.  A convolution is the implicit GEMM
// Y^T (Cout x V) = Wp (Cout x K) * X^T (K x V) with K = 27 taps x Cin in
// groups of 8 channels: group g = tap * Cin/8 + cg.  The 16x16x32 instruction
// takes, per lane l, 8 consecutive K of row l%16 of the first operand and 8
// consecutive K of column l%16 of the second, K-block l/16; so each lane
// loads one group (16 bytes) of the packed weights for its output channel and
// one group of the shifted input voxel for its voxel, the shift of group g
// coming from a per-block table in LDS.  The result holds 4 consecutive
// output channels of one voxel per lane.  A wavefront owns a 4 x 4 x 4 voxel
// tile: 16 voxels per instruction column block, 4 z-slices.
//
// Backward-data is the same kernel: the adjoint of a 3x3x3 correlation is
// the correlation with the tap-reversed kernel and transposed channel blocks,
// so only the weight packing differs.  Backward-weight contracts over voxels
// (K = 32 voxels per instruction, bricks of 4 x 4 x 2), with the gradient
// block as the first operand (rows = output channels) and the shifted input
// as the second (columns = input channels); one wavefront keeps all 27 taps'
// accumulators and writes one partial sum per brick chunk, which a second
// kernel adds in a fixed order.
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
//
// A workgroup of four wavefronts computes an 8 x 8 x 4 voxel tile for 16 NB
// output channels; wavefront w owns the 4 x 4 x 4 sub-tile at
// (4 (w & 1), 4 (w >> 1)).  The input channels are taken in chunks of CC (16,
// or 8 for an 8-channel input): the chunk's 10 x 10 x 6 halo tile (600 voxels
// x CC channels, zero outside the padded grid) is staged in LDS once, and all
// 27 taps of the chunk read their shifted voxels from there, so each input
// voxel is loaded from memory once per chunk instead of once per tap; the
// chunk's weights of the block's row group are staged beside it, so the K
// loop issues no global loads.  K is
// ordered chunk-major: chunk cc, then tap, then the 8-channel half h of the
// chunk; each chunk's 27 (CC/8) groups are padded to whole K-steps of 4
// groups with zero weights (conv_pack_* writes the matching layout).

constexpr int kTX = 8, kTY = 8, kTZ = 4;                 // output tile of a workgroup
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;  // its halo tile
constexpr int kHV = kHX * kHY * kHZ;                     // 600 voxels

template <int NB, int CC>  // NB = 16-channel row blocks per wavefront, CC = staged channels
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a) {
  constexpr int HG = CC / 8;                  // 8-channel groups per voxel and chunk
  constexpr int KSC = (27 * HG + 3) / 4;      // K-steps per chunk
  constexpr int ITEMS = (kHV * HG + 255) / 256;  // 16-byte input staging items per thread
  constexpr int WROWS = 16 * NB;              // weight rows (output channels) of the block
  constexpr int WITEMS = (KSC * 4 * WROWS + 255) / 256;  // 16-byte weight items per thread
  __shared__ __align__(16) bf16 sx[kHV * CC];
  __shared__ __align__(16) bf16 sw[KSC * 4 * WROWS * 8];  // the chunk's weights [ks][kg][row][8]
  const PGrid g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int TX = (g.W + kTX - 1) / kTX, TY = (g.H + kTY - 1) / kTY, TZ = (g.D + kTZ - 1) / kTZ;
  const int nrg = a.cout / (16 * NB);
  int64_t t = blockIdx.x;
  const int rg = int(t % nrg);
  t /= nrg;
  const int tx = int(t % TX);
  t /= TX;
  const int ty = int(t % TY);
  t /= TY;
  const int tz = int(t % TZ);
  const int b = int(t / TZ);
  if (b >= g.B) return;
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;  // logical origin; halo (0,0,0) is
                                                          // padded voxel (z0, y0, x0)
  const int kg = lane >> 4, j = lane & 15;
  const int vx = (w & 1) * 4 + (j & 3), vy = (w >> 1) * 4 + (j >> 2);  // in the tile

  f32x4 acc[NB][kTZ];
#pragma unroll
  for (int r = 0; r < NB; ++r)
#pragma unroll
    for (int z = 0; z < kTZ; ++z) acc[r][z] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nchunk = a.cin / CC;
  for (int cc = 0; cc < nchunk; ++cc) {
    if (cc) __syncthreads();  // the previous chunk's reads are done
    u16x8 stage[ITEMS], wst[WITEMS];
#pragma unroll
    for (int k = 0; k < WITEMS; ++k) {  // the chunk's weights of this row group
      const int it = k * 256 + tid;
      wst[k] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (it < KSC * 4 * WROWS) {
        const int row = it % WROWS, q = it / WROWS;  // q = ks * 4 + kg
        wst[k] = *reinterpret_cast<const u16x8 *>(
            a.wp + ((size_t(cc) * KSC * 4 + q) * a.cout + rg * WROWS + row) * 8);
      }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {  // all loads issued before any LDS write
      const int it = k * 256 + tid;
      stage[k] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (it < kHV * HG) {
        const int v = it / HG, h = it - v * HG;
        const int hx = v % kHX, hy = (v / kHX) % kHY, hz = v / (kHX * kHY);
        const int px = x0 + hx, py = y0 + hy, pz = z0 + hz;
        if (px < g.Wp && py < g.Hp && pz < g.Dp)
          stage[k] = *reinterpret_cast<const u16x8 *>(
              a.x + (((int64_t(b) * g.Dp + pz) * g.Hp + py) * g.Wp + px) * a.cin + cc * CC + h * 8);
      }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int it = k * 256 + tid;
      if (it < kHV * HG) *reinterpret_cast<u16x8 *>(sx + it * 8) = stage[k];
    }
#pragma unroll
    for (int k = 0; k < WITEMS; ++k) {
      const int it = k * 256 + tid;
      if (it < KSC * 4 * WROWS) *reinterpret_cast<u16x8 *>(sw + it * 8) = wst[k];
    }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < KSC; ++ks) {
      const int G = 4 * ks + kg;
      const bool real = G < 27 * HG;  // padding groups have zero weights
      const int tap = real ? G / HG : 13, h = real ? G - (G / HG) * HG : 0;
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
      bf16x8 wv[NB], xv[kTZ];
#pragma unroll
      for (int r = 0; r < NB; ++r)
        wv[r] = *reinterpret_cast<const bf16x8 *>(sw + ((ks * 4 + kg) * WROWS + r * 16 + j) * 8);
#pragma unroll
      for (int zb = 0; zb < kTZ; ++zb)
        xv[zb] = *reinterpret_cast<const bf16x8 *>(
            sx + (((zb + dz) * kHY + (vy + dy)) * kHX + (vx + dx)) * CC + h * 8);
#pragma unroll
      for (int r = 0; r < NB; ++r)
#pragma unroll
        for (int zb = 0; zb < kTZ; ++zb)
          acc[r][zb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[r], xv[zb], acc[r][zb], 0, 0, 0);
    }
  }
  // epilogue: lane holds output channels r*16 + 4*kg + i of voxel (x, y, z0 + zb)
  const int ox = x0 + vx, oy = y0 + vy;
  if (ox >= g.W || oy >= g.H) return;
  const PGrid f = g.twice();
#pragma unroll
  for (int zb = 0; zb < kTZ; ++zb) {
    const int z = z0 + zb;
    if (z >= g.D) break;
    const int64_t vox = g.at(b, z, oy, ox);
    for (int r = 0; r < NB; ++r) {
      const int c0 = (rg * NB + r) * 16 + kg * 4;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = acc[r][zb][i] + (a.bias ? a.bias[c0 + i] : 0.f);
        if (a.relu) v[i] = fmaxf(v[i], 0.f);
      }
      if (a.mask.p) {
        const bf16 *m = a.mask.p + vox * a.mask.cs + a.mask.co + c0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (!(bf2f(m[i]) > 0.f)) v[i] = 0.f;
      }
      if (a.out.p) {
        const ushort4 o{f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
        if (!a.out_up) {
          *reinterpret_cast<ushort4 *>(a.out.p + vox * a.out.cs + a.out.co + c0) = o;
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int64_t fv = f.at(b, 2 * z + (k >> 2), 2 * oy + ((k >> 1) & 1), 2 * ox + (k & 1));
            *reinterpret_cast<ushort4 *>(a.out.p + fv * a.out.cs + a.out.co + c0) = o;
          }
        }
      }
      if (a.o32) {
        const float4 o{v[0], v[1], v[2], v[3]};
        if (a.split == 0)
          *reinterpret_cast<float4 *>(a.o32 + vox * a.cout + c0) = o;
        else if (c0 < a.split)
          *reinterpret_cast<float4 *>(a.o32 + vox * a.split + c0) = o;
        else
          *reinterpret_cast<float4 *>(a.o32b + vox * (a.cout - a.split) + (c0 - a.split)) = o;
      }
    }
  }
}

// ---- convolution backward-weight ---------------------------------------------------
// Bricks of 4 (x) x 4 (y) x 2 (z) voxels over the grid rounded up (the
// round-up region reads zeros): K-block kg of a lane covers the 8 voxels
// x = 0..3, y = 2 (kg & 1) + {0, 1}, z = kg >> 1 of the brick.

__global__ __launch_bounds__(256) void k_conv_wgrad(ConvWArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int nrb = a.cout >> 4, ncb = (a.cin + 15) >> 4;
  if (wave >= int64_t(a.nchunks) * nrb * ncb) return;
  const PGrid g = a.g;
  const int rbo = int(wave % nrb);
  const int cbi = int((wave / nrb) % ncb);
  const int ch = int(wave / (int64_t(nrb) * ncb));
  const int kg = lane >> 4, j = lane & 15;
  const int BX = (g.W + 3) >> 2, BY = (g.H + 3) >> 2, BZ = (g.D + 1) >> 1;
  const int64_t nbr = int64_t(g.B) * BZ * BY * BX;
  const int64_t br0 = nbr * ch / a.nchunks, br1 = nbr * (ch + 1) / a.nchunks;
  const int co = rbo * 16 + j, ci = cbi * 16 + j;
  const int ci_ld = ci < a.cin ? ci : 0;  // columns past cin are computed but not stored
  int vo[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) vo[i] = ((i >> 2) * g.Wp + (i & 3));
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
    const int64_t vb = g.at(b, bz, by, bx);
    const bf16 *gp = a.gy + vb * a.cout + co;
    u16x8 gu;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      gu[i] = gp[vo[i] * a.cout];
      bsum += bf2f(gu[i]);
    }
    const bf16x8 gv = __builtin_bit_cast(bf16x8, gu);
    const bf16 *xp = a.x + vb * a.cin + ci_ld;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      const int toff = ((dz * g.Hp + dy) * g.Wp + dx) * a.cin;
      u16x8 xu;
#pragma unroll
      for (int i = 0; i < 8; ++i) xu[i] = xp[toff + vo[i] * a.cin];
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

// Fixed-order sums over parts: out[k] = sum_c part[c * n + k], in two stages.
// Stage 1: block (kb, grp) adds the parts of group grp (kGrp consecutive parts)
// for 64 consecutive k, its four wavefronts taking every fourth part, and
// writes the group sum over the group's first part (read by no other block).
// Stage 2 adds the group sums the same way.
constexpr int kGrp = 64;

__device__ __forceinline__ float sum4_fixed(float (&sh)[4][64], int lane, float v, int w) {
  sh[w][lane] = v;
  __syncthreads();
  return (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ __launch_bounds__(256) void k_sum_parts_grp(float *__restrict__ part, int nparts,
                                                       int64_t n) {
  __shared__ float sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t k = int64_t(blockIdx.x) * 64 + lane;
  const int c0 = blockIdx.y * kGrp, c1 = min(nparts, c0 + kGrp);
  float s = 0.f;
  if (k < n)
    for (int c = c0 + w; c < c1; c += 4) s += part[c * n + k];
  const float t = sum4_fixed(sh, lane, s, w);
  if (w == 0 && k < n) part[c0 * n + k] = t;
}

__global__ __launch_bounds__(256) void k_sum_groups(const float *__restrict__ part, int nparts,
                                                    int64_t n, float *__restrict__ out) {
  __shared__ float sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t k = int64_t(blockIdx.x) * 64 + lane;
  float s = 0.f;
  if (k < n)
    for (int c = w * kGrp; c < nparts; c += 4 * kGrp) s += part[c * n + k];
  const float t = sum4_fixed(sh, lane, s, w);
  if (w == 0 && k < n) out[k] = t;
}

// out = fixed-order sum of the nparts partial vectors of length n (part is overwritten)
static int sum_parts(float *part, int nparts, int64_t n, float *out, hipStream_t s) {
  const unsigned kb = unsigned((n + 63) / 64), ng = unsigned((nparts + kGrp - 1) / kGrp);
  hipLaunchKernelGGL(k_sum_parts_grp, dim3(kb, ng), dim3(256), 0, s, part, nparts, n);
  hipLaunchKernelGGL(k_sum_groups, dim3(kb), dim3(256), 0, s, part, nparts, n, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

// ---- weight packing ----------------------------------------------------------------------

// The chunk-major K order of k_conv_fwd for an input of cin channels: global
// group q = (cc * KSC + ks) * 4 + kg; within the chunk G = 4 ks + kg, tap =
// G / HG, half h = G % HG (channel cc CC + 8 h + jj); G >= 27 HG is padding.
struct KOrder {
  int CC, HG, KSC;
  __host__ __device__ explicit KOrder(int cin)
      : CC(cin < 16 ? 8 : 16), HG(cin < 16 ? 1 : 2), KSC((27 * (cin < 16 ? 1 : 2) + 3) / 4) {}
  // tap (27 = padding) and first channel of group q
  __host__ __device__ void group(int q, int &tap, int &c) const {
    const int cc = q / (4 * KSC), G = q - cc * 4 * KSC;
    tap = G < 27 * HG ? G / HG : 27;
    c = cc * CC + (G - (G / HG) * HG) * 8;
  }
};

int conv_ksteps(int cin) {
  const KOrder k(cin);
  return (cin / k.CC) * k.KSC;
}

// forward: wp[q][co][jj] = W[tap][c + jj][co] for group q = (tap, c) of the
// chunk-major order over cin_pad channels; zero for padding groups and
// channels past cin_real.  W is [27][cin_real][cout] FP32.
__global__ void k_pack_fwd(const float *__restrict__ W, int cin_real, int cin_pad, int cout,
                           int ngroups_pad, bf16 *__restrict__ wp) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(ngroups_pad) * cout * 8;
  if (i >= n) return;
  const int jj = int(i & 7);
  const int co = int((i >> 3) % cout);
  const int q = int((i >> 3) / cout);
  int tap, c;
  KOrder(cin_pad).group(q, tap, c);
  c += jj;
  const float v = (tap < 27 && c < cin_real) ? W[(size_t(tap) * cin_real + c) * cout + co] : 0.f;
  wp[i] = f2bf(v);
}

// backward-data: the correlation with reversed taps and swapped channels over
// an input of cout channels (the forward's outputs), output ci:
// wq[q][ci][jj] = W[26 - tap][ci][c + jj] for group q = (tap, c).
__global__ void k_pack_bwd(const float *__restrict__ W, int cin, int cout, int ngroups_pad,
                           bf16 *__restrict__ wq) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(ngroups_pad) * cin * 8;
  if (i >= n) return;
  const int jj = int(i & 7);
  const int ci = int((i >> 3) % cin);
  const int q = int((i >> 3) / cin);
  int tap, c;
  KOrder(cout).group(q, tap, c);
  c += jj;
  const float v = tap < 27 ? W[(size_t(26 - tap) * cin + ci) * cout + c] : 0.f;
  wq[i] = f2bf(v);
}

// ---- layout changes, pooling, upsampling adjoints, masks ------------------------------

// decompose a logical element index over [B][D][H][W][C]
struct Elem {
  int b, z, y, x, c;
};
__device__ __forceinline__ Elem decompose(int64_t i, const PGrid &g, int C) {
  Elem e;
  e.c = int(i % C);
  int64_t v = i / C;
  e.x = int(v % g.W);
  v /= g.W;
  e.y = int(v % g.H);
  v /= g.H;
  e.z = int(v % g.D);
  e.b = int(v / g.D);
  return e;
}

// padded concatenation of unpadded a (half grid when up_a) and b, 8 channels per thread
__global__ void k_gather_padded(const bf16 *__restrict__ a, int ca, int up_a,
                                const bf16 *__restrict__ b, int cb, PGrid g,
                                bf16 *__restrict__ out) {
  const int C8 = (ca + cb) >> 3;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.B) * g.D * g.H * g.W * C8) return;
  const Elem e = decompose(i, g, C8);
  const int c = e.c * 8;
  const bf16 *src;
  if (c < ca) {
    if (up_a) {
      const int Dc = g.D / 2, Hc = g.H / 2, Wc = g.W / 2;
      src = a + ((((int64_t)e.b * Dc + (e.z >> 1)) * Hc + (e.y >> 1)) * Wc + (e.x >> 1)) * ca + c;
    } else {
      src = a + ((((int64_t)e.b * g.D + e.z) * g.H + e.y) * g.W + e.x) * ca + c;
    }
  } else {
    src = b + ((((int64_t)e.b * g.D + e.z) * g.H + e.y) * g.W + e.x) * cb + (c - ca);
  }
  *reinterpret_cast<uint4 *>(out + g.at(e.b, e.z, e.y, e.x) * (ca + cb) + c) =
      *reinterpret_cast<const uint4 *>(src);
}

__global__ void k_unpad_f32(const float *__restrict__ in, PGrid g, int C, float *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.B) * g.D * g.H * g.W * C) return;
  const Elem e = decompose(i, g, C);
  out[i] = in[g.at(e.b, e.z, e.y, e.x) * C + e.c];
}

// 2x2x2 average pooling of a channel window into a padded coarse tensor [C]
__global__ void k_pool2(Slice in, PGrid f, int C, bf16 *__restrict__ out) {
  const PGrid g = f.half();
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.B) * g.D * g.H * g.W * C) return;
  const Elem e = decompose(i, g, C);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    s += bf2f(in.p[f.at(e.b, 2 * e.z + (k >> 2), 2 * e.y + ((k >> 1) & 1), 2 * e.x + (k & 1)) * in.cs +
                   in.co + e.c]);
  out[g.at(e.b, e.z, e.y, e.x) * C + e.c] = f2bf(s * 0.125f);
}

// coarse gpre = (sum of the 8 children of gup) * (mask > 0); gup FP32 padded fine [C];
// the mask is the coarse activation, stored upsampled (read at the first child)
__global__ void k_up_adjoint_mask(const float *__restrict__ gup, Slice mask, PGrid g, int C,
                                  bf16 *__restrict__ out) {
  const PGrid f = g.twice();
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.B) * g.D * g.H * g.W * C) return;
  const Elem e = decompose(i, g, C);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    s += gup[f.at(e.b, 2 * e.z + (k >> 2), 2 * e.y + ((k >> 1) & 1), 2 * e.x + (k & 1)) * C + e.c];
  const float m = bf2f(mask.p[f.at(e.b, 2 * e.z, 2 * e.y, 2 * e.x) * mask.cs + mask.co + e.c]);
  out[g.at(e.b, e.z, e.y, e.x) * C + e.c] = f2bf(m > 0.f ? s : 0.f);
}

// fine gpre = (gskip + gp[parent] / 8) * (mask > 0), all padded
__global__ void k_pool_adjoint_add_mask(const float *__restrict__ gskip,
                                        const float *__restrict__ gp, Slice mask, PGrid f, int C,
                                        bf16 *__restrict__ out) {
  const PGrid g = f.half();
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(f.B) * f.D * f.H * f.W * C) return;
  const Elem e = decompose(i, f, C);
  const int64_t v = f.at(e.b, e.z, e.y, e.x);
  const float s = gskip[v * C + e.c] + 0.125f * gp[g.at(e.b, e.z >> 1, e.y >> 1, e.x >> 1) * C + e.c];
  const float m = bf2f(mask.p[v * mask.cs + mask.co + e.c]);
  out[v * C + e.c] = f2bf(m > 0.f ? s : 0.f);
}

// ---- head, loss -------------------------------------------------------------------------

// out[b][z][y][x] (unpadded) = sum_c t[v][c] wh[c] + bh, t padded [16]
__global__ void k_head_fwd(const bf16 *__restrict__ t, PGrid g, const float *__restrict__ wh,
                           float *__restrict__ out) {
  constexpr int C = 16;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.B) * g.D * g.H * g.W) return;
  const Elem e = decompose(i, g, 1);
  const bf16 *tv = t + g.at(e.b, e.z, e.y, e.x) * C;
  float s = wh[C];
#pragma unroll
  for (int c = 0; c < C; ++c) s += bf2f(tv[c]) * wh[c];
  out[i] = s;
}

constexpr int kHB = 256;  // threads per block of the head / loss reductions

// gpre[v][c] = dout[v] wh[c] (t[v][c] > 0); per-block partials of
// dL/dwh[c] = sum_v dout[v] t[v][c] and dL/dbh = sum_v dout[v]
__global__ __launch_bounds__(kHB) void k_head_bwd(const float *__restrict__ dout,
                                                 const bf16 *__restrict__ t, PGrid g,
                                                 const float *__restrict__ wh,
                                                 bf16 *__restrict__ gpre,
                                                 float *__restrict__ part /*[nblk][17]*/) {
  constexpr int C = 16;
  __shared__ float sh[C + 1][kHB / 64];
  float acc[C + 1];
#pragma unroll
  for (int c = 0; c <= C; ++c) acc[c] = 0.f;
  const int64_t nv = int64_t(g.B) * g.D * g.H * g.W;
  for (int64_t i = int64_t(blockIdx.x) * kHB + threadIdx.x; i < nv; i += int64_t(gridDim.x) * kHB) {
    const Elem e = decompose(i, g, 1);
    const int64_t v = g.at(e.b, e.z, e.y, e.x);
    const float d = dout[i];
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
static inline int64_t logical(const PGrid &g) { return int64_t(g.B) * g.D * g.H * g.W; }

int conv_forward(const ConvArgs &a, hipStream_t s) {
  Q1_CHECK(a.cin % 8 == 0 && a.cin >= 8 && (a.cin == 8 || a.cin % 16 == 0) && a.cin <= 96,
           Q1_EUNSUPPORTED, "conv: %d input channels", a.cin);
  Q1_CHECK(a.nchunks == conv_ksteps(a.cin), Q1_EINVAL, "conv: %d K-steps for %d channels",
           a.nchunks, a.cin);
  Q1_CHECK(a.cout % 16 == 0 && a.cout >= 16 && a.cout <= 96, Q1_EUNSUPPORTED,
           "conv: %d output channels (16, 32, 48, 64, 96)", a.cout);
  const int64_t tiles = int64_t(a.g.B) * ((a.g.D + kTZ - 1) / kTZ) * ((a.g.H + kTY - 1) / kTY) *
                        ((a.g.W + kTX - 1) / kTX);
  // row blocks per wavefront: all of them when that still gives 512 workgroups,
  // else fewer (more workgroups, each staging its input tile once more)
  // (the chunk's weights of two row blocks fill 28 KB of LDS beside the 19 KB input tile)
  const int rb = a.cout / 16;
  const int nb = rb % 2 == 0 && tiles * (rb / 2) >= 512 ? 2 : 1;
  const unsigned blocks = unsigned(tiles * (rb / nb));
  auto launch = [&](auto k8, auto k16) {
    if (a.cin == 8)
      hipLaunchKernelGGL(k8, dim3(blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(k16, dim3(blocks), dim3(256), 0, s, a);
  };
  if (nb == 2)
    launch(k_conv_fwd<2, 8>, k_conv_fwd<2, 16>);
  else
    launch(k_conv_fwd<1, 8>, k_conv_fwd<1, 16>);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int wgrad_chunks(const ConvWArgs &a) {
  const int64_t nbr = int64_t(a.g.B) * ((a.g.D + 1) / 2) * ((a.g.H + 3) / 4) * ((a.g.W + 3) / 4);
  const int units = (a.cout / 16) * ((a.cin + 15) / 16);
  return int(std::max<int64_t>(1, std::min<int64_t>(nbr, std::max(1, 4096 / units))));
}

int conv_wgrad(ConvWArgs a, float *gw, float *gb, hipStream_t s) {
  const int64_t waves = int64_t(a.nchunks) * (a.cout / 16) * ((a.cin + 15) / 16);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, s, a);
  const int64_t nk = int64_t(27) * a.cin_real * a.cout;
  Q1_HIP(hipGetLastError());
  int rc = sum_parts(a.part, a.nchunks, nk, gw, s);
  return rc ? rc : sum_parts(a.bpart, a.nchunks, int64_t(a.cout), gb, s);
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

int gather_padded(const bf16 *a, int ca, int up_a, const bf16 *b, int cb, const PGrid &g, bf16 *out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_gather_padded, g1(logical(g) * ((ca + cb) / 8)), dim3(256), 0, s, a, ca, up_a,
                     b, cb, g, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int unpad_f32(const float *in, const PGrid &g, int C, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_unpad_f32, g1(logical(g) * C), dim3(256), 0, s, in, g, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pool2(Slice in, const PGrid &fine, int C, bf16 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2, g1(logical(fine.half()) * C), dim3(256), 0, s, in, fine, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int up_adjoint_mask(const float *gup, Slice mask_fine, const PGrid &coarse, int C, bf16 *out,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_up_adjoint_mask, g1(logical(coarse) * C), dim3(256), 0, s, gup, mask_fine,
                     coarse, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int pool_adjoint_add_mask(const float *gskip, const float *gp, Slice mask, const PGrid &fine, int C,
                          bf16 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_adjoint_add_mask, g1(logical(fine) * C), dim3(256), 0, s, gskip, gp,
                     mask, fine, C, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int head_forward(const bf16 *t, const PGrid &g, const float *wh, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_head_fwd, g1(logical(g)), dim3(256), 0, s, t, g, wh, out);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int head_backward(const float *dout, const bf16 *t, const PGrid &g, const float *wh, bf16 *gpre,
                  float *part, int nblk, float *gwh, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nblk), dim3(kHB), 0, s, dout, t, g, wh, gpre, part);
  Q1_HIP(hipGetLastError());
  return sum_parts(part, nblk, int64_t(17), gwh, s);
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
