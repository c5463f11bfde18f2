// The learned preconditioner: a 3-level 3-D convolutional U-Net on the node
// grid (channels 16/32/64, two 3x3x3 convolutions with ReLU per level, 2x2x2
// average pooling down, nearest upsampling and concatenation with the skip
// tensor up, 1x1 head), trained with Adam on residual -> error pairs and used
// as z = N(r) inside flexible PCG.  The paper's conclusions (Section 7) name
// matrix-free preconditioners as future work and say nothing of learned
// ones: the network, its encoding and its training are this project's own.
//
// Storage: BF16 activations and packed BF16 weights for the matrix cores,
// FP32 master weights, gradients and Adam moments in one flat vector whose
// layout is, per convolution, W[27][Cin][Cout] then b[Cout], and for the head
// w[16] then b.  Activations are kept from the last forward for the backward.
// Every tensor a convolution reads has a zero halo (PGrid).  The skip and
// upsampled tensors are written by their producers straight into the
// concatenation buffers the decoder reads (cat1 = [up(t2), s1] on the finest
// grid, cat2 = [up(b3), s2] on the middle one), so no convolution reads two
// tensors or upsamples on the fly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "q1_conv.hpp"
#include "q1_internal.hpp"

namespace q1 {

namespace {

struct LayerSpec {
  int cin_real, cin, cout, level;
};
// enc1a enc1b enc2a enc2b enc3a enc3b dec2a dec2b dec1a dec1b
constexpr LayerSpec kSpec[10] = {{2, 8, 16, 1},   {16, 16, 16, 1}, {16, 16, 32, 2},
                                 {32, 32, 32, 2}, {32, 32, 64, 3}, {64, 64, 64, 3},
                                 {96, 96, 32, 2}, {32, 32, 32, 2}, {48, 48, 16, 1},
                                 {16, 16, 16, 1}};
constexpr int kInC = 8;  // stored input channels (2 used)

struct Layer {
  LayerSpec s;
  int64_t wo = 0, bo = 0;
  int ngroups = 0, nchunks = 0, ngroups_b = 0, nchunks_b = 0;
  bf16 *wp = nullptr, *wq = nullptr;
};

}  // namespace

struct UNet {
  int D = 0, H = 0, W = 0, B = 0;
  int64_t nparams = 0, head_o = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  Layer L[10];
  // padded activations: input, own outputs, concatenations, pooled tensors
  bf16 *xin = nullptr, *act0 = nullptr, *act2 = nullptr, *act4 = nullptr, *act6 = nullptr,
       *act8 = nullptr, *act9 = nullptr, *cat1 = nullptr, *cat2 = nullptr, *p1 = nullptr,
       *p2 = nullptr;
  bf16 *g1a = nullptr, *g1b = nullptr, *g2a = nullptr, *g2b = nullptr, *g3a = nullptr,
       *g3b = nullptr;
  float *gup1 = nullptr, *gskip1 = nullptr, *gup2 = nullptr, *gskip2 = nullptr, *gp2 = nullptr,
        *gp1 = nullptr;
  float *part = nullptr, *bpart = nullptr, *hpart = nullptr;
  double *mpart = nullptr;
  int last_nb = 0;
  std::vector<void *> allocs;

  PGrid grid(int level, int nb) const {
    const int f = 1 << (level - 1);
    return PGrid(nb, D / f, H / f, W / f);
  }
  ~UNet() {
    for (void *p : allocs) (void)hipFree(p);
  }
};

struct UNetPC {
  UNet *net = nullptr;
  int nx = 0, ny = 0, nz = 0;
  int64_t nn = 0, n_free = 0;
  const uint8_t *mask = nullptr;
  bf16 *in = nullptr;   // one input sample [D][H][W][8] with the coefficient channel set
  float *out = nullptr;  // [D][H][W]
  float *kap = nullptr;  // nodal channel-1 values [nn]
  double *part = nullptr;
  // two-level form: Jacobi smoothing around the network's coarse correction
  Op *op = nullptr;
  double omega = 0.0;
  double *w = nullptr, *z1 = nullptr, *r1 = nullptr, *d = nullptr, *q = nullptr;
  // schedule: the network on calls 0, period, 2 period, ... since the last
  // reset; the plain Jacobi step z = w r on the others
  int period = 1;
  int64_t calls = 0;
  ~UNetPC() {
    for (void *p : {(void *)in, (void *)out, (void *)kap, (void *)part, (void *)w, (void *)z1,
                    (void *)r1, (void *)d, (void *)q})
      if (p) (void)hipFree(p);
  }
};

namespace {

template <typename T>
int dalloc(UNet &n, T **p, size_t count) {
  void *q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
    return fail(Q1_ENOMEM, "q1_unet: device allocation of %zu bytes failed", count * sizeof(T));
  n.allocs.push_back(q);
  if (hipMemset(q, 0, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
    return fail(Q1_EHIP, "q1_unet: clearing a buffer failed");
  *p = static_cast<T *>(q);
  return Q1_OK;
}

// SplitMix64 + Box-Muller for the initial weights
inline uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double u01(uint64_t seed, uint64_t i) {
  return (double(mix(seed ^ mix(i)) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

int pack_all(UNet &n, hipStream_t s) {
  for (int l = 0; l < 10; ++l) {
    Layer &L = n.L[l];
    int rc = pack_forward(n.theta + L.wo, L.s.cin_real, L.s.cin, L.s.cout, L.nchunks * 4, L.wp, s);
    if (rc) return rc;
    if (L.wq && (rc = pack_backward(n.theta + L.wo, L.s.cin_real, L.s.cout, L.nchunks_b * 4, L.wq, s)))
      return rc;
  }
  return Q1_OK;
}

struct LayerIO {
  const bf16 *in;
  Slice out;
  int up;
};

// where each layer reads and writes (see the header comment)
LayerIO layer_io(const UNet &n, int l) {
  switch (l) {
    case 0: return {n.xin, {n.act0, 16, 0}, 0};
    case 1: return {n.act0, {n.cat1, 48, 32}, 0};
    case 2: return {n.p1, {n.act2, 32, 0}, 0};
    case 3: return {n.act2, {n.cat2, 96, 64}, 0};
    case 4: return {n.p2, {n.act4, 64, 0}, 0};
    case 5: return {n.act4, {n.cat2, 96, 0}, 1};
    case 6: return {n.cat2, {n.act6, 32, 0}, 0};
    case 7: return {n.act6, {n.cat1, 48, 0}, 1};
    case 8: return {n.cat1, {n.act8, 16, 0}, 0};
    default: return {n.act8, {n.act9, 16, 0}, 0};
  }
}

int layer_forward(UNet &n, int l, int nb, hipStream_t s) {
  const Layer &L = n.L[l];
  const LayerIO io = layer_io(n, l);
  ConvArgs c;
  c.x = io.in;
  c.cin = L.s.cin;
  c.g = n.grid(L.s.level, nb);
  c.wp = L.wp;
  c.ngroups = L.ngroups;
  c.nchunks = L.nchunks;
  c.cout = L.s.cout;
  c.bias = n.theta + L.bo;
  c.relu = 1;
  c.out = io.out;
  c.out_up = io.up;
  return conv_forward(c, s);
}

// input gradient of layer l from its pre-activation gradient g (padded [cout])
int layer_backward_data(UNet &n, int l, int nb, const bf16 *g, Slice mask, bf16 *out_bf,
                        float *o32, int split, float *o32b, hipStream_t s) {
  const Layer &L = n.L[l];
  ConvArgs c;
  c.x = g;
  c.cin = L.s.cout;
  c.g = n.grid(L.s.level, nb);
  c.wp = L.wq;
  c.ngroups = L.ngroups_b;
  c.nchunks = L.nchunks_b;
  c.cout = L.s.cin;
  c.mask = mask;
  c.out = Slice{out_bf, L.s.cin, 0};
  c.o32 = o32;
  c.split = split;
  c.o32b = o32b;
  return conv_forward(c, s);
}

int layer_wgrad(UNet &n, int l, int nb, const bf16 *g, hipStream_t s) {
  const Layer &L = n.L[l];
  ConvWArgs w;
  w.x = layer_io(n, l).in;
  w.cin = L.s.cin;
  w.g = n.grid(L.s.level, nb);
  w.gy = g;
  w.cout = L.s.cout;
  w.cin_real = L.s.cin_real;
  w.nchunks = wgrad_chunks(w);
  w.part = n.part;
  w.bpart = n.bpart;
  return conv_wgrad(w, n.grad + L.wo, n.grad + L.bo, s);
}

int unet_forward(UNet &n, const bf16 *in, float *out, int nb, hipStream_t s) {
  int rc;
  const PGrid g1 = n.grid(1, nb), g2 = n.grid(2, nb);
  if ((rc = gather_padded(in, kInC, 0, nullptr, 0, g1, n.xin, s))) return rc;
  for (int l = 0; l < 10; ++l) {
    if ((rc = layer_forward(n, l, nb, s))) return rc;
    if (l == 1 && (rc = pool2(Slice{n.cat1, 48, 32}, g1, 16, n.p1, s))) return rc;
    if (l == 3 && (rc = pool2(Slice{n.cat2, 96, 64}, g2, 32, n.p2, s))) return rc;
  }
  if ((rc = head_forward(n.act9, g1, n.theta + n.head_o, out, s))) return rc;
  n.last_nb = nb;
  return Q1_OK;
}

int unet_backward(UNet &n, const float *dout, hipStream_t s) {
  int rc;
  const int nb = n.last_nb;
  const PGrid g1 = n.grid(1, nb), g2 = n.grid(2, nb), g3 = n.grid(3, nb);
  const int64_t v1 = int64_t(nb) * n.D * n.H * n.W;
  const int hblk = int(std::min<int64_t>(1024, (v1 + 255) / 256));
  const Slice none{};
  if ((rc = head_backward(dout, n.act9, g1, n.theta + n.head_o, n.g1a, n.hpart, hblk,
                          n.grad + n.head_o, s)))
    return rc;
  // level 1 decoder
  if ((rc = layer_wgrad(n, 9, nb, n.g1a, s))) return rc;
  if ((rc = layer_backward_data(n, 9, nb, n.g1a, Slice{n.act8, 16, 0}, n.g1b, nullptr, 0,
                                nullptr, s)))
    return rc;
  if ((rc = layer_wgrad(n, 8, nb, n.g1b, s))) return rc;
  if ((rc = layer_backward_data(n, 8, nb, n.g1b, none, nullptr, n.gup1, 32, n.gskip1, s)))
    return rc;
  if ((rc = up_adjoint_mask(n.gup1, Slice{n.cat1, 48, 0}, g2, 32, n.g2a, s))) return rc;
  // level 2 decoder
  if ((rc = layer_wgrad(n, 7, nb, n.g2a, s))) return rc;
  if ((rc = layer_backward_data(n, 7, nb, n.g2a, Slice{n.act6, 32, 0}, n.g2b, nullptr, 0,
                                nullptr, s)))
    return rc;
  if ((rc = layer_wgrad(n, 6, nb, n.g2b, s))) return rc;
  if ((rc = layer_backward_data(n, 6, nb, n.g2b, none, nullptr, n.gup2, 64, n.gskip2, s)))
    return rc;
  if ((rc = up_adjoint_mask(n.gup2, Slice{n.cat2, 96, 0}, g3, 64, n.g3a, s))) return rc;
  // level 3
  if ((rc = layer_wgrad(n, 5, nb, n.g3a, s))) return rc;
  if ((rc = layer_backward_data(n, 5, nb, n.g3a, Slice{n.act4, 64, 0}, n.g3b, nullptr, 0,
                                nullptr, s)))
    return rc;
  if ((rc = layer_wgrad(n, 4, nb, n.g3b, s))) return rc;
  if ((rc = layer_backward_data(n, 4, nb, n.g3b, none, nullptr, n.gp2, 0, nullptr, s))) return rc;
  if ((rc = pool_adjoint_add_mask(n.gskip2, n.gp2, Slice{n.cat2, 96, 64}, g2, 32, n.g2a, s)))
    return rc;
  // level 2 encoder
  if ((rc = layer_wgrad(n, 3, nb, n.g2a, s))) return rc;
  if ((rc = layer_backward_data(n, 3, nb, n.g2a, Slice{n.act2, 32, 0}, n.g2b, nullptr, 0,
                                nullptr, s)))
    return rc;
  if ((rc = layer_wgrad(n, 2, nb, n.g2b, s))) return rc;
  if ((rc = layer_backward_data(n, 2, nb, n.g2b, none, nullptr, n.gp1, 0, nullptr, s))) return rc;
  if ((rc = pool_adjoint_add_mask(n.gskip1, n.gp1, Slice{n.cat1, 48, 32}, g1, 16, n.g1a, s)))
    return rc;
  // level 1 encoder
  if ((rc = layer_wgrad(n, 1, nb, n.g1a, s))) return rc;
  if ((rc = layer_backward_data(n, 1, nb, n.g1a, Slice{n.act0, 16, 0}, n.g1b, nullptr, 0,
                                nullptr, s)))
    return rc;
  return layer_wgrad(n, 0, nb, n.g1b, s);
}

// ---- preconditioner encoding ---------------------------------------------------------

constexpr int kEB = 256;

// mean of ln k over the cells adjacent to each node, halved (input channel 1)
__global__ void k_kappa(const double *__restrict__ k, int nx, int ny, int nz,
                        float *__restrict__ kap) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nn = int64_t(nx + 1) * (ny + 1) * (nz + 1);
  if (id >= nn) return;
  const int i = int(id % (nx + 1)), j = int((id / (nx + 1)) % (ny + 1)),
            kk = int(id / (int64_t(nx + 1) * (ny + 1)));
  double s = 0.0;
  int c = 0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = i + dx, ey = j + dy, ez = kk + dz;
        if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
        s += log(k[(int64_t(ez) * ny + ey) * nx + ex]);
        ++c;
      }
  kap[id] = float(0.5 * s / c);
}

// per-block partials of sum over free nodes of v^2
__global__ __launch_bounds__(kEB) void k_free_norm(const double *__restrict__ v,
                                                  const uint8_t *__restrict__ mask, int64_t nn,
                                                  double *__restrict__ part) {
  __shared__ double sh[kEB / 64];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kEB + threadIdx.x; i < nn; i += int64_t(gridDim.x) * kEB)
    if (!mask || !mask[i]) s += v[i] * v[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kEB / 64; ++k) t += sh[k];
    part[blockIdx.x] = t;
  }
}

__device__ __forceinline__ double scale_from(const double *part, int nparts, int64_t n_free) {
  double s = 0.0;
  for (int k = 0; k < nparts; ++k) s += part[k];
  return s > 0.0 ? sqrt(double(n_free) / s) : 0.0;
}

// full input sample [D][H][W][8]: channel 0 = r scaled to unit RMS on free nodes,
// channel 1 = kappa on mesh nodes, zero elsewhere
__global__ void k_encode(const double *__restrict__ r, const uint8_t *__restrict__ mask,
                         const float *__restrict__ kap, const double *__restrict__ part, int nparts,
                         int64_t n_free, int nx, int ny, int nz, int D, int H, int W,
                         bf16 *__restrict__ in) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= int64_t(D) * H * W) return;
  const int x = int(v % W), y = int((v / W) % H), z = int(v / (int64_t(W) * H));
  unsigned short c0 = 0, c1 = 0;
  if (x <= nx && y <= ny && z <= nz) {
    const int64_t id = (int64_t(z) * (ny + 1) + y) * (nx + 1) + x;
    const double sc = scale_from(part, nparts, n_free);
    if (!mask || !mask[id]) c0 = __builtin_bit_cast(unsigned short, static_cast<__bf16>(float(r[id] * sc)));
    c1 = __builtin_bit_cast(unsigned short, static_cast<__bf16>(kap[id]));
  }
  uint4 o;
  o.x = unsigned(c0) | (unsigned(c1) << 16);
  o.y = o.z = o.w = 0u;
  *reinterpret_cast<uint4 *>(in + v * kInC) = o;
}

// target on the grid: e scaled to unit RMS on free nodes; weight 1 there, else 0
__global__ void k_encode_target(const double *__restrict__ e, const uint8_t *__restrict__ mask,
                                const double *__restrict__ part, int nparts, int64_t n_free,
                                int nx, int ny, int nz, int D, int H, int W,
                                float *__restrict__ tgt, float *__restrict__ wgt) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= int64_t(D) * H * W) return;
  const int x = int(v % W), y = int((v / W) % H), z = int(v / (int64_t(W) * H));
  float t = 0.f, w = 0.f;
  if (x <= nx && y <= ny && z <= nz) {
    const int64_t id = (int64_t(z) * (ny + 1) + y) * (nx + 1) + x;
    if (!mask || !mask[id]) {
      t = float(e[id] * scale_from(part, nparts, n_free));
      w = 1.f;
    }
  }
  tgt[v] = t;
  if (wgt) wgt[v] = w;
}

// z on the nodes: the network output on free nodes, 0 on Dirichlet nodes
__global__ void k_decode(const float *__restrict__ out, const uint8_t *__restrict__ mask, int nx,
                         int ny, int nz, int H, int W, double *__restrict__ z) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nn = int64_t(nx + 1) * (ny + 1) * (nz + 1);
  if (id >= nn) return;
  const int x = int(id % (nx + 1)), y = int((id / (nx + 1)) % (ny + 1)),
            zz = int(id / (int64_t(nx + 1) * (ny + 1)));
  z[id] = (mask && mask[id]) ? 0.0 : double(out[(int64_t(zz) * H + y) * W + x]);
}

// z = w r
__global__ void k_jacobi_step(int64_t n, const double *__restrict__ w, const double *__restrict__ r,
                              double *__restrict__ z) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[i] = w[i] * r[i];
}
// training pair from an iterate: e = xs - xk (the error)
__global__ void k_pair_error(int64_t n, const double *__restrict__ xs,
                             const double *__restrict__ xk, double *__restrict__ e) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) e[i] = xs[i] - xk[i];
}
// e -= omega w r (one damped-Jacobi step on the error)
__global__ void k_pair_smooth(int64_t n, const double *__restrict__ w,
                              const double *__restrict__ r, double omega,
                              double *__restrict__ e) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) e[i] -= omega * w[i] * r[i];
}
// FP32 copies of the pair
__global__ void k_pair_store(int64_t n, const double *__restrict__ e,
                             const double *__restrict__ r, float *__restrict__ eo,
                             float *__restrict__ ro) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    eo[i] = float(e[i]);
    ro[i] = float(r[i]);
  }
}

__global__ void k_inv(int64_t n, const double *__restrict__ d, double *__restrict__ w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;  // 0 on zero rows (unreferenced nodes)
}
// z1 = omega w r ; (w = 1 / diag A)
__global__ void k_smooth(int64_t n, const double *__restrict__ w, const double *__restrict__ r,
                         double omega, double *__restrict__ z) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[i] = omega * w[i] * r[i];
}
// r1 = r - q
__global__ void k_sub(int64_t n, const double *__restrict__ r, const double *__restrict__ q,
                      double *__restrict__ r1) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) r1[i] = r[i] - q[i];
}
// per-block partials of d.r1 and d.q
__global__ __launch_bounds__(kEB) void k_dot2(int64_t n, const double *__restrict__ d,
                                             const double *__restrict__ r1,
                                             const double *__restrict__ q,
                                             double *__restrict__ part) {
  __shared__ double sh[2][kEB / 64];
  double a = 0.0, b = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kEB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kEB) {
    a += d[i] * r1[i];
    b += d[i] * q[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int k = 0; k < kEB / 64; ++k) t += sh[threadIdx.x][k];
    part[2 * blockIdx.x + threadIdx.x] = t;
  }
}
// c = (d.r1) / (d.A d) (0 when not positive and finite); z = z1 + c d + omega w (r1 - c A d)
__global__ void k_two_level_combine(int64_t n, const double *__restrict__ part, int nparts,
                                    const double *__restrict__ z1, const double *__restrict__ d,
                                    const double *__restrict__ r1, const double *__restrict__ q,
                                    const double *__restrict__ w, double omega,
                                    double *__restrict__ z) {
  double dr = 0.0, dq = 0.0;
  for (int k = 0; k < nparts; ++k) {
    dr += part[2 * k];
    dq += part[2 * k + 1];
  }
  const double c = (dq > 0.0 && isfinite(dr / dq)) ? dr / dq : 0.0;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[i] = z1[i] + c * d[i] + omega * w[i] * (r1[i] - c * q[i]);
}

inline dim3 grid_for(int64_t n, int bs = 256) { return dim3(unsigned((n + bs - 1) / bs)); }

int pc_norm(UNetPC &pc, const double *v, hipStream_t s, int *nparts) {
  const int nb = int(std::min<int64_t>(256, (pc.nn + kEB - 1) / kEB));
  hipLaunchKernelGGL(k_free_norm, dim3(nb), dim3(kEB), 0, s, v, pc.mask, pc.nn, pc.part);
  Q1_HIP(hipGetLastError());
  *nparts = nb;
  return Q1_OK;
}

int pc_encode(UNetPC &pc, const double *r, bf16 *in, hipStream_t s) {
  int np = 0, rc = pc_norm(pc, r, s, &np);
  if (rc) return rc;
  const UNet &n = *pc.net;
  hipLaunchKernelGGL(k_encode, grid_for(int64_t(n.D) * n.H * n.W), dim3(256), 0, s, r, pc.mask,
                     pc.kap, pc.part, np, pc.n_free, pc.nx, pc.ny, pc.nz, n.D, n.H, n.W, in);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace
}  // namespace q1

using namespace q1;

struct q1_unet : public q1::UNet {};
struct q1_unet_pc : public q1::UNetPC {};

extern "C" {

int q1_unet_create(q1_unet **out, int D, int H, int W, int batch, uint64_t seed, void *stream) {
  Q1_CHECK(out, Q1_EINVAL, "q1_unet_create: NULL argument");
  *out = nullptr;
  Q1_CHECK(D >= 4 && H >= 4 && W >= 4 && D % 4 == 0 && H % 4 == 0 && W % 4 == 0 && batch >= 1,
           Q1_EINVAL, "q1_unet_create: grid %dx%dx%d must be multiples of 4, batch >= 1", D, H, W);
  hipStream_t s = static_cast<hipStream_t>(stream);
  q1_unet *np = new (std::nothrow) q1_unet();
  Q1_CHECK(np, Q1_ENOMEM, "q1_unet_create: out of host memory");
  UNet &n = *np;
  n.D = D;
  n.H = H;
  n.W = W;
  n.B = batch;
  int64_t off = 0;
  size_t part_cap = 0, bpart_cap = 0;
  for (int l = 0; l < 10; ++l) {
    Layer &L = n.L[l];
    L.s = kSpec[l];
    L.wo = off;
    L.bo = off + int64_t(27) * L.s.cin_real * L.s.cout;
    off = L.bo + L.s.cout;
    L.ngroups = 27 * L.s.cin / 8;
    L.nchunks = conv_ksteps(L.s.cin);
    L.ngroups_b = 27 * L.s.cout / 8;
    L.nchunks_b = conv_ksteps(L.s.cout);
    ConvWArgs w;
    w.g = n.grid(L.s.level, batch);
    w.cin = L.s.cin;
    w.cout = L.s.cout;
    const int nch = wgrad_chunks(w);
    part_cap = std::max(part_cap, size_t(nch) * 27 * L.s.cin_real * L.s.cout);
    bpart_cap = std::max(bpart_cap, size_t(nch) * L.s.cout);
  }
  n.head_o = off;
  n.nparams = off + 17;
  int rc = Q1_OK;
  auto A = [&](auto **p, size_t cnt) {
    if (!rc) rc = dalloc(n, p, cnt);
  };
  A(&n.theta, n.nparams);
  A(&n.grad, n.nparams);
  A(&n.m, n.nparams);
  A(&n.v, n.nparams);
  for (int l = 0; l < 10; ++l) {
    Layer &L = n.L[l];
    A(&L.wp, size_t(L.nchunks) * 4 * L.s.cout * 8);
    if (l > 0) A(&L.wq, size_t(L.nchunks_b) * 4 * L.s.cin * 8);
  }
  const size_t v1 = size_t(n.grid(1, batch).voxels()), v2 = size_t(n.grid(2, batch).voxels()),
               v3 = size_t(n.grid(3, batch).voxels());
  A(&n.xin, v1 * kInC);
  A(&n.act0, v1 * 16);
  A(&n.act2, v2 * 32);
  A(&n.act4, v3 * 64);
  A(&n.act6, v2 * 32);
  A(&n.act8, v1 * 16);
  A(&n.act9, v1 * 16);
  A(&n.cat1, v1 * 48);
  A(&n.cat2, v2 * 96);
  A(&n.p1, v2 * 16);
  A(&n.p2, v3 * 32);
  A(&n.g1a, v1 * 16);
  A(&n.g1b, v1 * 16);
  A(&n.g2a, v2 * 32);
  A(&n.g2b, v2 * 32);
  A(&n.g3a, v3 * 64);
  A(&n.g3b, v3 * 64);
  A(&n.gup1, v1 * 32);
  A(&n.gskip1, v1 * 16);
  A(&n.gup2, v2 * 64);
  A(&n.gskip2, v2 * 32);
  A(&n.gp2, v3 * 32);
  A(&n.gp1, v2 * 16);
  A(&n.part, part_cap);
  A(&n.bpart, bpart_cap);
  A(&n.hpart, size_t(1024) * 17);
  A(&n.mpart, size_t(1024) * 2);
  if (!rc) {
    // He-normal weights (std sqrt(2 / fan_in)), zero biases, zero moments
    std::vector<float> th(size_t(n.nparams), 0.f);
    uint64_t key = mix(seed ^ 0x5eed5eedull);
    for (int l = 0; l < 10; ++l) {
      const Layer &L = n.L[l];
      const double sd = std::sqrt(2.0 / (27.0 * L.s.cin_real));
      for (int64_t i = L.wo; i < L.bo; ++i) {
        const double u1 = u01(key, 2 * uint64_t(i)), u2 = u01(key, 2 * uint64_t(i) + 1);
        th[size_t(i)] = float(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
      }
    }
    for (int64_t i = n.head_o; i < n.head_o + 16; ++i) {
      const double u1 = u01(key, 2 * uint64_t(i)), u2 = u01(key, 2 * uint64_t(i) + 1);
      th[size_t(i)] = float(std::sqrt(2.0 / 16.0) * std::sqrt(-2.0 * std::log(u1)) *
                            std::cos(6.283185307179586 * u2));
    }
    if (hipMemcpyAsync(n.theta, th.data(), th.size() * sizeof(float), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemsetAsync(n.m, 0, size_t(n.nparams) * sizeof(float), s) != hipSuccess ||
        hipMemsetAsync(n.v, 0, size_t(n.nparams) * sizeof(float), s) != hipSuccess ||
        hipMemsetAsync(n.grad, 0, size_t(n.nparams) * sizeof(float), s) != hipSuccess)
      rc = fail(Q1_EHIP, "q1_unet_create: initialisation failed");
    if (!rc) rc = pack_all(n, s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess)
      rc = fail(Q1_EHIP, "q1_unet_create: initialisation failed");
  }
  if (rc) {
    delete np;
    return rc;
  }
  *out = np;
  return Q1_OK;
}

int q1_unet_destroy(q1_unet *net) {
  delete net;
  return Q1_OK;
}

int q1_unet_info(const q1_unet *net, int64_t *nparams, int *D, int *H, int *W, int *batch) {
  Q1_CHECK(net, Q1_EINVAL, "q1_unet_info: NULL network");
  if (nparams) *nparams = net->nparams;
  if (D) *D = net->D;
  if (H) *H = net->H;
  if (W) *W = net->W;
  if (batch) *batch = net->B;
  return Q1_OK;
}

int q1_unet_params(q1_unet *net, float **theta_d, float **grad_d) {
  Q1_CHECK(net, Q1_EINVAL, "q1_unet_params: NULL network");
  if (theta_d) *theta_d = net->theta;
  if (grad_d) *grad_d = net->grad;
  return Q1_OK;
}

int q1_unet_commit(q1_unet *net, void *stream) {
  Q1_CHECK(net, Q1_EINVAL, "q1_unet_commit: NULL network");
  return pack_all(*net, static_cast<hipStream_t>(stream));
}

int q1_unet_copy(q1_unet *net, int which, int to_net, float *buf_d, void *stream) {
  Q1_CHECK(net && buf_d, Q1_EINVAL, "q1_unet_copy: NULL argument");
  Q1_CHECK((which == 0 || which == 1) && (to_net == 0 || to_net == 1), Q1_EINVAL,
           "q1_unet_copy: which %d to_net %d", which, to_net);
  float *lib_buf = which == 0 ? net->theta : net->grad;
  const size_t bytes = size_t(net->nparams) * sizeof(float);
  Q1_HIP(hipMemcpyAsync(to_net ? lib_buf : buf_d, to_net ? buf_d : lib_buf, bytes,
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return Q1_OK;
}

int q1_unet_forward(q1_unet *net, const uint16_t *in_d, float *out_d, int nbatch, void *stream) {
  Q1_CHECK(net && in_d && out_d, Q1_EINVAL, "q1_unet_forward: NULL argument");
  Q1_CHECK(nbatch >= 1 && nbatch <= net->B, Q1_EINVAL, "q1_unet_forward: nbatch %d not in [1, %d]",
           nbatch, net->B);
  return unet_forward(*net, in_d, out_d, nbatch, static_cast<hipStream_t>(stream));
}

int q1_unet_mse(q1_unet *net, const float *out_d, const float *target_d, const float *weight_d,
                float *dout_d, float *loss_d, void *stream) {
  Q1_CHECK(net && out_d && target_d && weight_d && dout_d, Q1_EINVAL, "q1_unet_mse: NULL argument");
  Q1_CHECK(net->last_nb >= 1, Q1_EINVAL, "q1_unet_mse: no forward pass yet");
  const int64_t n = int64_t(net->last_nb) * net->D * net->H * net->W;
  const int nblk = int(std::min<int64_t>(1024, (n + 255) / 256));
  return mse(out_d, target_d, weight_d, n, net->mpart, nblk, dout_d, loss_d,
             static_cast<hipStream_t>(stream));
}

int q1_unet_backward(q1_unet *net, const float *dout_d, void *stream) {
  Q1_CHECK(net && dout_d, Q1_EINVAL, "q1_unet_backward: NULL argument");
  Q1_CHECK(net->last_nb >= 1, Q1_EINVAL, "q1_unet_backward: no forward pass yet");
  return unet_backward(*net, dout_d, static_cast<hipStream_t>(stream));
}

int q1_unet_adam_step(q1_unet *net, float lr, float b1, float b2, float eps, int step,
                      void *stream) {
  Q1_CHECK(net, Q1_EINVAL, "q1_unet_adam_step: NULL network");
  Q1_CHECK(step >= 1 && lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0, Q1_EINVAL,
           "q1_unet_adam_step: bad hyper-parameters");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = adam(net->theta, net->grad, net->m, net->v, net->nparams, lr, b1, b2, eps, step, s);
  return rc ? rc : pack_all(*net, s);
}

// ---- single-layer primitives (synchronous: they pack the weights into temporaries) ----

namespace {
struct TmpBuf {
  void *p = nullptr;
  ~TmpBuf() {
    if (p) (void)hipFree(p);
  }
};
bool conv_cout_ok(int c) { return c == 16 || c == 32 || c == 48 || c == 64 || c == 96; }
}  // namespace

int q1_conv3d_forward(int B, int D, int H, int W, const uint16_t *a_d, int ca, int up_a,
                      const uint16_t *b_d, int cb, const float *w_d, const float *bias_d, int cout,
                      int relu, float *y_d, void *stream) {
  Q1_CHECK(a_d && w_d && y_d && (cb == 0 || b_d), Q1_EINVAL, "q1_conv3d_forward: NULL argument");
  Q1_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1 && ca >= 8 && ca % 8 == 0 && cb >= 0 && cb % 8 == 0,
           Q1_EINVAL, "q1_conv3d_forward: bad sizes (channels must be multiples of 8)");
  Q1_CHECK(!up_a || (D % 2 == 0 && H % 2 == 0 && W % 2 == 0), Q1_EINVAL,
           "q1_conv3d_forward: upsampled input needs an even grid");
  Q1_CHECK(conv_cout_ok(cout), Q1_EUNSUPPORTED, "q1_conv3d_forward: cout %d", cout);
  Q1_CHECK(ca + cb <= 96, Q1_EUNSUPPORTED, "q1_conv3d_forward: more than 96 input channels");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int cin = ca + cb, ngroups = 27 * cin / 8, nchunks = conv_ksteps(cin);
  const PGrid g(B, D, H, W);
  TmpBuf wp, xp, yp;
  Q1_HIP(hipMalloc(&wp.p, size_t(nchunks) * 4 * cout * 8 * sizeof(bf16)));
  Q1_HIP(hipMalloc(&xp.p, size_t(g.voxels()) * cin * sizeof(bf16)));
  Q1_HIP(hipMalloc(&yp.p, size_t(g.voxels()) * cout * sizeof(float)));
  Q1_HIP(hipMemsetAsync(xp.p, 0, size_t(g.voxels()) * cin * sizeof(bf16), s));
  int rc = pack_forward(w_d, cin, cin, cout, nchunks * 4, static_cast<bf16 *>(wp.p), s);
  if (!rc) rc = gather_padded(a_d, ca, up_a, b_d, cb, g, static_cast<bf16 *>(xp.p), s);
  if (rc) return rc;
  ConvArgs c;
  c.x = static_cast<bf16 *>(xp.p);
  c.cin = cin;
  c.g = g;
  c.wp = static_cast<bf16 *>(wp.p);
  c.ngroups = ngroups;
  c.nchunks = nchunks;
  c.cout = cout;
  c.bias = bias_d;
  c.relu = relu;
  c.o32 = static_cast<float *>(yp.p);
  if ((rc = conv_forward(c, s))) return rc;
  if ((rc = unpad_f32(static_cast<float *>(yp.p), g, cout, y_d, s))) return rc;
  Q1_HIP(hipStreamSynchronize(s));
  return Q1_OK;
}

int q1_conv3d_backward_data(int B, int D, int H, int W, const uint16_t *gy_d, int cout,
                            const float *w_d, int cin, float *gx_d, void *stream) {
  Q1_CHECK(gy_d && w_d && gx_d, Q1_EINVAL, "q1_conv3d_backward_data: NULL argument");
  Q1_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1 && cout % 8 == 0 && cout >= 8 && cout <= 96,
           Q1_EINVAL, "q1_conv3d_backward_data: bad sizes");
  Q1_CHECK(conv_cout_ok(cin), Q1_EUNSUPPORTED, "q1_conv3d_backward_data: cin %d", cin);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ngroups = 27 * cout / 8, nchunks = conv_ksteps(cout);
  const PGrid g(B, D, H, W);
  TmpBuf wq, gp, xp;
  Q1_HIP(hipMalloc(&wq.p, size_t(nchunks) * 4 * cin * 8 * sizeof(bf16)));
  Q1_HIP(hipMalloc(&gp.p, size_t(g.voxels()) * cout * sizeof(bf16)));
  Q1_HIP(hipMalloc(&xp.p, size_t(g.voxels()) * cin * sizeof(float)));
  Q1_HIP(hipMemsetAsync(gp.p, 0, size_t(g.voxels()) * cout * sizeof(bf16), s));
  int rc = pack_backward(w_d, cin, cout, nchunks * 4, static_cast<bf16 *>(wq.p), s);
  if (!rc) rc = gather_padded(gy_d, cout, 0, nullptr, 0, g, static_cast<bf16 *>(gp.p), s);
  if (rc) return rc;
  ConvArgs c;
  c.x = static_cast<bf16 *>(gp.p);
  c.cin = cout;
  c.g = g;
  c.wp = static_cast<bf16 *>(wq.p);
  c.ngroups = ngroups;
  c.nchunks = nchunks;
  c.cout = cin;
  c.o32 = static_cast<float *>(xp.p);
  if ((rc = conv_forward(c, s))) return rc;
  if ((rc = unpad_f32(static_cast<float *>(xp.p), g, cin, gx_d, s))) return rc;
  Q1_HIP(hipStreamSynchronize(s));
  return Q1_OK;
}

int q1_conv3d_backward_weight(int B, int D, int H, int W, const uint16_t *a_d, int ca, int up_a,
                              const uint16_t *b_d, int cb, const uint16_t *gy_d, int cout,
                              float *gw_d, float *gb_d, void *stream) {
  Q1_CHECK(a_d && gy_d && gw_d && gb_d && (cb == 0 || b_d), Q1_EINVAL,
           "q1_conv3d_backward_weight: NULL argument");
  Q1_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1 && ca >= 8 && ca % 8 == 0 && cb >= 0 &&
               cb % 8 == 0 && cout % 16 == 0 && cout >= 16 && cout <= 96,
           Q1_EINVAL, "q1_conv3d_backward_weight: bad sizes");
  Q1_CHECK(!up_a || (D % 2 == 0 && H % 2 == 0 && W % 2 == 0), Q1_EINVAL,
           "q1_conv3d_backward_weight: upsampled input needs an even grid");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int cin = ca + cb;
  const PGrid g(B, D, H, W);
  ConvWArgs w;
  w.cin = cin;
  w.g = g;
  w.cout = cout;
  w.cin_real = cin;
  w.nchunks = wgrad_chunks(w);
  TmpBuf xp, gp, part, bpart;
  Q1_HIP(hipMalloc(&xp.p, size_t(g.voxels()) * cin * sizeof(bf16)));
  Q1_HIP(hipMalloc(&gp.p, size_t(g.voxels()) * cout * sizeof(bf16)));
  Q1_HIP(hipMalloc(&part.p, size_t(w.nchunks) * 27 * cin * cout * sizeof(float)));
  Q1_HIP(hipMalloc(&bpart.p, size_t(w.nchunks) * cout * sizeof(float)));
  Q1_HIP(hipMemsetAsync(xp.p, 0, size_t(g.voxels()) * cin * sizeof(bf16), s));
  Q1_HIP(hipMemsetAsync(gp.p, 0, size_t(g.voxels()) * cout * sizeof(bf16), s));
  int rc = gather_padded(a_d, ca, up_a, b_d, cb, g, static_cast<bf16 *>(xp.p), s);
  if (!rc) rc = gather_padded(gy_d, cout, 0, nullptr, 0, g, static_cast<bf16 *>(gp.p), s);
  if (rc) return rc;
  w.x = static_cast<bf16 *>(xp.p);
  w.gy = static_cast<bf16 *>(gp.p);
  w.part = static_cast<float *>(part.p);
  w.bpart = static_cast<float *>(bpart.p);
  if ((rc = conv_wgrad(w, gw_d, gb_d, s))) return rc;
  Q1_HIP(hipStreamSynchronize(s));
  return Q1_OK;
}

int q1_unet_pc_create(q1_unet_pc **out, q1_unet *net, int nx, int ny, int nz, const double *k_d,
                      const uint8_t *mask_d, void *stream) {
  Q1_CHECK(out && net && k_d, Q1_EINVAL, "q1_unet_pc_create: NULL argument");
  *out = nullptr;
  Q1_CHECK(nx >= 1 && ny >= 1 && nz >= 1 && nx + 1 <= net->W && ny + 1 <= net->H &&
               nz + 1 <= net->D,
           Q1_EINVAL, "q1_unet_pc_create: %dx%dx%d-element mesh does not fit the %dx%dx%d grid",
           nx, ny, nz, net->W, net->H, net->D);
  hipStream_t s = static_cast<hipStream_t>(stream);
  q1_unet_pc *pc = new (std::nothrow) q1_unet_pc();
  Q1_CHECK(pc, Q1_ENOMEM, "q1_unet_pc_create: out of host memory");
  pc->net = net;
  pc->nx = nx;
  pc->ny = ny;
  pc->nz = nz;
  pc->nn = int64_t(nx + 1) * (ny + 1) * (nz + 1);
  pc->mask = mask_d;
  const int64_t nv = int64_t(net->D) * net->H * net->W;
  int rc = Q1_OK;
  if (hipMalloc(&pc->in, size_t(nv) * kInC * sizeof(bf16)) != hipSuccess ||
      hipMalloc(&pc->out, size_t(nv) * sizeof(float)) != hipSuccess ||
      hipMalloc(&pc->kap, size_t(pc->nn) * sizeof(float)) != hipSuccess ||
      hipMalloc(&pc->part, 256 * sizeof(double)) != hipSuccess)
    rc = fail(Q1_ENOMEM, "q1_unet_pc_create: device allocation failed");
  if (!rc) {
    hipLaunchKernelGGL(k_kappa, grid_for(pc->nn), dim3(256), 0, s, k_d, nx, ny, nz, pc->kap);
    if (hipGetLastError() != hipSuccess) rc = fail(Q1_EHIP, "q1_unet_pc_create: launch failed");
  }
  if (!rc) {
    pc->n_free = pc->nn;
    if (mask_d) {
      std::vector<uint8_t> m(size_t(pc->nn));
      if (hipMemcpyAsync(m.data(), mask_d, m.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        rc = fail(Q1_EHIP, "q1_unet_pc_create: mask copy failed");
      else
        pc->n_free = pc->nn - std::count_if(m.begin(), m.end(), [](uint8_t c) { return c != 0; });
    }
  }
  if (rc) {
    delete pc;
    return rc;
  }
  *out = pc;
  return Q1_OK;
}

int q1_unet_pc_two_level(q1_unet_pc *pc, q1_op *op, double omega, void *stream) {
  Q1_CHECK(pc && op, Q1_EINVAL, "q1_unet_pc_two_level: NULL argument");
  Op &o = *reinterpret_cast<Op *>(op);
  Q1_CHECK(o.physics == 1 && o.dtype == Q1_F64 && o.n_nodes == pc->nn, Q1_EINVAL,
           "q1_unet_pc_two_level: needs the FP64 scalar operator of the context's mesh");
  Q1_CHECK(omega > 0.0 && omega < 2.0, Q1_EINVAL, "q1_unet_pc_two_level: omega %g", omega);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t b = size_t(pc->nn) * sizeof(double);
  if (!pc->w) {
    if (hipMalloc(&pc->w, b) != hipSuccess || hipMalloc(&pc->z1, b) != hipSuccess ||
        hipMalloc(&pc->r1, b) != hipSuccess || hipMalloc(&pc->d, b) != hipSuccess ||
        hipMalloc(&pc->q, b) != hipSuccess)
      return fail(Q1_ENOMEM, "q1_unet_pc_two_level: device allocation failed");
  }
  int rc = launch_diag(o, pc->q, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_inv, grid_for(pc->nn), dim3(256), 0, s, pc->nn, pc->q, pc->w);
  Q1_HIP(hipGetLastError());
  pc->op = &o;
  pc->omega = omega;
  return Q1_OK;
}

int q1_unet_pc_schedule(q1_unet_pc *pc, int period) {
  Q1_CHECK(pc && period >= 1, Q1_EINVAL, "q1_unet_pc_schedule: need a context and period >= 1");
  Q1_CHECK(period == 1 || pc->op, Q1_EINVAL,
           "q1_unet_pc_schedule: a period above 1 needs the two-level form (its Jacobi weights)");
  pc->period = period;
  pc->calls = 0;
  return Q1_OK;
}

int q1_unet_pairs(q1_op *op, const double *xstar_d, int npairs, const double *const *xk_d,
                  double omega, float *const *e_d, float *const *r_d, void *stream) {
  Q1_CHECK(op && xstar_d && npairs >= 0 && (npairs == 0 || (xk_d && e_d && r_d)), Q1_EINVAL,
           "q1_unet_pairs: NULL argument");
  Op &o = *reinterpret_cast<Op *>(op);
  Q1_CHECK(o.physics == Q1_LAPLACE && o.dtype == Q1_F64, Q1_EINVAL,
           "q1_unet_pairs: needs an FP64 scalar-Laplace operator");
  Q1_CHECK(omega >= 0.0 && omega < 2.0, Q1_EINVAL, "q1_unet_pairs: omega %g", omega);
  for (int i = 0; i < npairs; ++i)
    Q1_CHECK(xk_d[i] && e_d[i] && r_d[i], Q1_EINVAL, "q1_unet_pairs: NULL vector %d", i);
  if (npairs == 0) return Q1_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = o.n_nodes;
  double *ws = nullptr;  // e, r and (with omega) the Jacobi weights
  Q1_HIP(hipMalloc(&ws, size_t(3 * n) * sizeof(double)));
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } fr{ws};
  double *e = ws, *r = ws + n, *w = ws + 2 * n;
  const dim3 g = grid_for(n);
  int rc;
  if (omega > 0.0) {
    if ((rc = launch_diag(o, r, s))) return rc;
    hipLaunchKernelGGL(k_inv, g, dim3(256), 0, s, n, r, w);
  }
  for (int i = 0; i < npairs; ++i) {
    hipLaunchKernelGGL(k_pair_error, g, dim3(256), 0, s, n, xstar_d, xk_d[i], e);
    if ((rc = launch_apply(o, e, r, s))) return rc;
    if (omega > 0.0) {
      hipLaunchKernelGGL(k_pair_smooth, g, dim3(256), 0, s, n, w, r, omega, e);
      if ((rc = launch_apply(o, e, r, s))) return rc;
    }
    hipLaunchKernelGGL(k_pair_store, g, dim3(256), 0, s, n, e, r, e_d[i], r_d[i]);
  }
  Q1_HIP(hipGetLastError());
  Q1_HIP(hipStreamSynchronize(s));  // the workspace is freed on return
  return Q1_OK;
}

int q1_unet_pc_destroy(q1_unet_pc *pc) {
  delete pc;
  return Q1_OK;
}

int q1_unet_encode(q1_unet_pc *pc, const double *r_d, uint16_t *in_d, void *stream) {
  Q1_CHECK(pc && r_d && in_d, Q1_EINVAL, "q1_unet_encode: NULL argument");
  return pc_encode(*pc, r_d, in_d, static_cast<hipStream_t>(stream));
}

int q1_unet_encode_target(q1_unet_pc *pc, const double *e_d, float *target_d, float *weight_d,
                          void *stream) {
  Q1_CHECK(pc && e_d && target_d, Q1_EINVAL, "q1_unet_encode_target: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int np = 0, rc = pc_norm(*pc, e_d, s, &np);
  if (rc) return rc;
  const UNet &n = *pc->net;
  hipLaunchKernelGGL(k_encode_target, grid_for(int64_t(n.D) * n.H * n.W), dim3(256), 0, s, e_d,
                     pc->mask, pc->part, np, pc->n_free, pc->nx, pc->ny, pc->nz, n.D, n.H, n.W,
                     target_d, weight_d);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int q1_unet_precond(void *ctx, const void *r_d, void *z_d, void *stream) {
  Q1_CHECK(ctx && r_d && z_d, Q1_EINVAL, "q1_unet_precond: NULL argument");
  q1_unet_pc &pc = *static_cast<q1_unet_pc *>(ctx);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double *r = static_cast<const double *>(r_d);
  double *z = static_cast<double *>(z_d);
  const dim3 g = grid_for(pc.nn);
  int rc;
  const bool net_call = pc.calls++ % pc.period == 0;
  if (!net_call) {  // the scheduled plain Jacobi step
    hipLaunchKernelGGL(k_jacobi_step, g, dim3(256), 0, s, pc.nn, pc.w, r, z);
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  }
  if (!pc.op) {  // z = N(r)
    if ((rc = pc_encode(pc, r, pc.in, s))) return rc;
    if ((rc = unet_forward(*pc.net, pc.in, pc.out, 1, s))) return rc;
    hipLaunchKernelGGL(k_decode, g, dim3(256), 0, s, pc.out, pc.mask, pc.nx, pc.ny, pc.nz,
                       pc.net->H, pc.net->W, z);
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  }
  // two-level: pre-smooth, network correction scaled to minimise the energy
  // norm of the error, post-smooth
  hipLaunchKernelGGL(k_smooth, g, dim3(256), 0, s, pc.nn, pc.w, r, pc.omega, pc.z1);
  if ((rc = launch_apply(*pc.op, pc.z1, pc.q, s))) return rc;
  hipLaunchKernelGGL(k_sub, g, dim3(256), 0, s, pc.nn, r, pc.q, pc.r1);
  if ((rc = pc_encode(pc, pc.r1, pc.in, s))) return rc;
  if ((rc = unet_forward(*pc.net, pc.in, pc.out, 1, s))) return rc;
  hipLaunchKernelGGL(k_decode, g, dim3(256), 0, s, pc.out, pc.mask, pc.nx, pc.ny, pc.nz,
                     pc.net->H, pc.net->W, pc.d);
  if ((rc = launch_apply(*pc.op, pc.d, pc.q, s))) return rc;
  const int nb = int(std::min<int64_t>(256, (pc.nn + kEB - 1) / kEB));
  hipLaunchKernelGGL(k_dot2, dim3(nb), dim3(kEB), 0, s, pc.nn, pc.d, pc.r1, pc.q, pc.part);
  hipLaunchKernelGGL(k_two_level_combine, g, dim3(256), 0, s, pc.nn, pc.part, nb, pc.z1, pc.d,
                     pc.r1, pc.q, pc.w, pc.omega, z);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // extern "C"
