// LDS-tiled apply: tile-resident accumulators.
//
// Set-up (once per operator, host).  Elements are grouped into tiles by their
// centroids: an (x, y) patch of PATCH x PATCH elements and a z-range of
// LAYERS element layers (a 32x2xLAYERS brick on a Cartesian grid).  A tile is
// processed by ONE wavefront in steps of at most 64 elements (one per lane),
// ordered by layer and then lexicographically.  Per tile the set-up stores the
// sorted list of its distinct nodes (global id, plus a flag for nodes that
// other tiles also touch and a flag for Dirichlet nodes), and per element the
// 8 indices of its corners in that list.  Nothing depends on the mesh being
// Cartesian; the grouping only decides how much reuse there is.
//
// Apply.  The wave clears an LDS accumulator for the tile's nodes; per step
// each lane gathers its element's coordinates and input values from global
// memory (neighbouring lanes share nodes, so the gathers coalesce and hit in
// L2), computes the element product (Section 3, step 2; q1_elem.hpp) and adds
// it into the accumulator.  After the last step the wave writes the tile's
// nodes once (Section 3, step 3): plain stores for nodes owned by this tile
// alone, global atomic adds for shared nodes.  The step loop issues no global
// stores, so its load waits never queue behind writes.  A small kernel first
// resets the shared and Dirichlet nodes (y = x on Dirichlet nodes, 0 on shared
// ones).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <numeric>
#include <vector>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {

constexpr int kLanes = 64;
constexpr uint32_t kSharedBit = 0x80000000u;
constexpr uint32_t kFixedBit = 0x40000000u;
constexpr uint32_t kIdMask = 0x3fffffffu;
// steps per wave of the split accumulation (held in registers): two for the
// scalar kind's 16 x 8 x 4 tiles, one for the 3-DOF kinds' 16 x 4 x 4
__host__ __device__ constexpr int split_steps(int dpn) { return dpn == 1 ? 2 : 1; }

// i / d for 0 <= i < 2^16 and 0 < d < 2^16: the single-precision quotient is
// within one of the exact one, and one correction each way makes it exact.
__host__ __device__ inline int div_small(int i, int d) {
  int q = int(float(i) * (1.0f / float(d)));
  q -= q * d > i ? 1 : 0;
  q += (q + 1) * d <= i ? 1 : 0;
  return q;
}

// Corner indices of lane `lane` at position `rel` of a lattice tile (the
// interleaved layout; see lattice_of); false for an empty lane.
__host__ __device__ inline bool corner_lattice(uint32_t lat, int rel, int lane, int (&lc)[8]) {
  const int A = int(lat & 0xff), B = int((lat >> 8) & 0xff), spl = int((lat >> 16) & 0xff),
            C = int(lat >> 24);
  const int w = rel & 3, k = rel >> 2, kl = div_small(k, spl);
  const int iz = w + 4 * kl, e = (k - kl * spl) * kLanes + lane;
  if (iz >= C || e >= A * B) return false;
  const int a1 = A + 1, ab1 = (A + 1) * (B + 1), ey = div_small(e, A);
  const int base = (e - ey * A) + a1 * ey + ab1 * iz;
#pragma unroll
  for (int a = 0; a < 8; ++a) lc[a] = base + (a & 1) + a1 * ((a >> 1) & 1) + ab1 * (a >> 2);
  return true;
}

// Lattice-addressed tiles (a lattice tile without Dirichlet nodes whose node
// list is the box g0 + ix + iy sy + iz sz of the mesh's own numbering): entry
// i's global id and shared flag follow from i, the tile origin g0, the mesh
// strides (sy, sz) and which of the six faces border another tile (bits 0-5:
// x-low, x-high, y-low, y-high, z-low, z-high), so the node words are not
// loaded.  i = ix + (A+1)(iy + (B+1) iz).
constexpr uint32_t kAddrValid = 0x80000000u;
__host__ __device__ inline uint32_t lattice_word(int i, uint32_t lat, uint32_t addr, int64_t g0,
                                                 int64_t sy, int64_t sz) {
  const int A = int(lat & 0xff), B = int((lat >> 8) & 0xff), C = int(lat >> 24);
  const int a1 = A + 1, ab1 = (A + 1) * (B + 1);
  const int iz = div_small(i, ab1), r = i - iz * ab1, iy = div_small(r, a1), ix = r - iy * a1;
  const bool sh = (ix == 0 && (addr & 1)) || (ix == A && (addr & 2)) ||
                  (iy == 0 && (addr & 4)) || (iy == B && (addr & 8)) ||
                  (iz == 0 && (addr & 16)) || (iz == C && (addr & 32));
  return uint32_t(g0 + ix + iy * sy + iz * sz) | (sh ? kSharedBit : 0u);
}

// The default tile of each kind as compile-time constants: 16 x 8 x 4
// elements (765 nodes, two steps per layer) for the scalar kind, 16 x 4 x 4
// (425 nodes, one step per layer) for the 3-DOF kinds.  When every tile of an
// operator is that lattice tile, a kernel instance with the shape built in
// computes corner indices, LDS offsets and lattice addresses from constants
// (the LDS reads of an element share one address register and differ by
// immediate offsets), which removes most of the integer work per element.
template <int DPN>
struct FxTile {
  static constexpr int A = 16, B = DPN == 1 ? 8 : 4, C = 4;
  static constexpr int SPL = A * B / 64;  // steps per layer; one layer per wave
  static constexpr int STEPS = C * SPL;
  static constexpr int NODES = (A + 1) * (B + 1) * (C + 1);
  static constexpr uint32_t LAT =
      uint32_t(A) | uint32_t(B) << 8 | uint32_t(SPL) << 16 | uint32_t(C) << 24;
  static_assert(A == 16 && A * B == SPL * 64 && C == 4 && SPL == split_steps(DPN),
                "one layer per wave, whole steps");
};

// corner_lattice for the fixed tile: position rel = 4k + w is step k of layer w
template <int DPN>
__host__ __device__ inline void corner_fixed(int rel, int lane, int (&lc)[8]) {
  using F = FxTile<DPN>;
  constexpr int a1 = F::A + 1, ab1 = (F::A + 1) * (F::B + 1);
  const int e = (rel >> 2) * 64 + lane;
  const int base = (e & (F::A - 1)) + a1 * (e >> 4) + ab1 * (rel & 3);
#pragma unroll
  for (int a = 0; a < 8; ++a) lc[a] = base + (a & 1) + a1 * ((a >> 1) & 1) + ab1 * (a >> 2);
}

// lattice_word for the fixed tile (ids below 2^30, so 32-bit arithmetic gives them exactly)
template <int DPN>
__host__ __device__ inline uint32_t lattice_word_fixed(int i, uint32_t addr, int64_t g0,
                                                       int64_t sy, int64_t sz) {
  using F = FxTile<DPN>;
  constexpr unsigned a1 = F::A + 1, ab1 = (F::A + 1) * (F::B + 1);
  const unsigned ui = unsigned(i);
  const unsigned iz = ui / ab1, r = ui - iz * ab1, iy = r / a1, ix = r - iy * a1;
  const bool sh = (ix == 0 && (addr & 1)) || (ix == unsigned(F::A) && (addr & 2)) ||
                  (iy == 0 && (addr & 4)) || (iy == unsigned(F::B) && (addr & 8)) ||
                  (iz == 0 && (addr & 16)) || (iz == unsigned(F::C) && (addr & 32));
  return (uint32_t(g0) + ix + iy * uint32_t(sy) + iz * uint32_t(sz)) | (sh ? kSharedBit : 0u);
}

__device__ __forceinline__ int xcd_block_t(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, local = bid >> 3;
  return x * q + min(x, r) + local;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(float *p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gbl_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void gbl_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// y on the reset list: x on Dirichlet nodes, 0 elsewhere
template <typename T, int DPN>
__global__ void k_reset_nodes(int64_t n, const int32_t *__restrict__ ids,
                              const uint8_t *__restrict__ mask, const T *__restrict__ x,
                              T *__restrict__ y, const int *__restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t g = ids[i];
  const bool fx = mask && mask[g];
#pragma unroll
  for (int j = 0; j < DPN; ++j) y[g * DPN + j] = fx ? x[g * DPN + j] : T(0);
}

// Accumulation: with LDS_ATOMIC the corner contributions are added with LDS
// atomics; otherwise corner by corner with plain read-add-write, which the
// set-up allows only when no two lanes of a step share a node at the same
// local corner (true on any consistently numbered structured grid).
// The plain read-add-write accumulation relies on one property: within one
// corner's instruction no two lanes touch the same node, while the next
// corner's instruction of the same wavefront may touch nodes that other lanes
// have just written.  A wavefront's LDS instructions execute in order, so the
// only thing to prevent is the compiler moving a later corner's read above an
// earlier corner's write (it may, where the addresses differ within one
// lane).  This is that compiler-only barrier; it emits no instruction.
__device__ __forceinline__ void lane_order() { asm volatile("" ::: "memory"); }

// Sum of one value per thread over a 256-thread workgroup in a fixed order (a
// wavefront shuffle tree, then the four wavefront sums in order); the result
// is valid in thread 0.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double wsum[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  return (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

template <typename T, bool LDS_ATOMIC>
__device__ __forceinline__ void acc_add(T *p, T v) {
  if constexpr (LDS_ATOMIC)
    lds_add(p, v);
  else
    *p += v;
}

template <typename T, int PH, bool LDS_ATOMIC>
__global__ __launch_bounds__(64) void k_apply_tile(
    int max_nodes, int64_t nn, const int32_t *__restrict__ node_ptr,  // [n_tiles+1]
    const uint32_t *__restrict__ nodes,                                 // ids | flags
    const int32_t *__restrict__ tile_step,                              // [n_tiles+1]
    const uint4 *__restrict__ lconn,                                    // [n_steps*64]
    const T *__restrict__ coef_t, int64_t coef_stride, const T *__restrict__ xyz,
    const T *__restrict__ x, T *__restrict__ y, const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sV = reinterpret_cast<T *>(smem_raw);                             // [DPN][max_nodes]
  uint32_t *sId = reinterpret_cast<uint32_t *>(sV + DPN * max_nodes);  // [max_nodes]
  const int lane = threadIdx.x;
  const int tile = xcd_block_t(blockIdx.x, gridDim.x);
  const int n0 = node_ptr[tile], nm = node_ptr[tile + 1] - n0;
  const int s0 = tile_step[tile], s1 = tile_step[tile + 1];
  // first step's corner indices and coefficients
  uint4 pk_n = lconn[int64_t(s0) * kLanes + lane];
  T c0_n = coef_t[int64_t(s0) * kLanes + lane];
  T c1_n = PH == 3 ? coef_t[coef_stride + int64_t(s0) * kLanes + lane] : T(0);
  for (int i = lane; i < nm; i += kLanes) {
    sId[i] = nodes[n0 + i];
#pragma unroll
    for (int j = 0; j < DPN; ++j) sV[j * max_nodes + i] = T(0);
  }
  __syncthreads();
  for (int s = s0; s < s1; ++s) {
    const uint4 pk = pk_n;
    const T c0 = c0_n, c1 = c1_n;
    {  // prefetch the next step's (clamped to this tile's last step)
      const int64_t nslot = int64_t(min(s + 1, s1 - 1)) * kLanes + lane;
      pk_n = lconn[nslot];
      c0_n = coef_t[nslot];
      if constexpr (PH == 3) c1_n = coef_t[coef_stride + nslot];
    }
    if (pk.x == 0xffffffffu) continue;  // empty lane
    const int lc[8] = {int(pk.x & 0xffff), int(pk.x >> 16), int(pk.y & 0xffff), int(pk.y >> 16),
                       int(pk.z & 0xffff), int(pk.z >> 16), int(pk.w & 0xffff), int(pk.w >> 16)};
    int64_t g[8];
    bool fixed[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const uint32_t raw = sId[lc[a]];
      g[a] = raw & kIdMask;
      fixed[a] = (raw & kFixedBit) != 0;
    }
    T X[3][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      X[0][a] = xyz[g[a]];
      X[1][a] = xyz[nn + g[a]];
      X[2][a] = xyz[2 * nn + g[a]];
    }
    T u[DPN][8], v[DPN][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int j = 0; j < DPN; ++j) u[j][a] = fixed[a] ? T(0) : x[g[a] * DPN + j];
    element_apply<T, PH>(X, u, c0, c1, v);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int j = 0; j < DPN; ++j) acc_add<T, LDS_ATOMIC>(&sV[j * max_nodes + lc[a]], v[j][a]);
      if constexpr (!LDS_ATOMIC) lane_order();
    }
  }
  __syncthreads();
  for (int i = lane; i < nm; i += kLanes) {
    const uint32_t raw = sId[i];
    if (raw & kFixedBit) continue;  // y = x written by the reset kernel
    const int64_t gg = raw & kIdMask;
    if (raw & kSharedBit) {
#pragma unroll
      for (int j = 0; j < DPN; ++j) gbl_add(&y[gg * DPN + j], sV[j * max_nodes + i]);
    } else {
#pragma unroll
      for (int j = 0; j < DPN; ++j) y[gg * DPN + j] = sV[j * max_nodes + i];
    }
  }
}

// Block-staged variant: one workgroup of four wavefronts per tile.  The
// tile's node records (coordinates and input values; zero input on Dirichlet
// nodes) are loaded once into LDS with bulk loads, so the element loop reads
// corners from LDS instead of gathering them from memory.  Wave w takes the
// tile's steps w, w + 4, ... and accumulates into LDS: in FP64 into one copy
// shared by the four waves (LDS atomics), in FP32 into its own copy, the copies
// being added in a fixed order when the tile's nodes are written.
// One element step of a wave: corners from the staged records, element
// product.  PAR: the element is known to be a parallelepiped, so only corners
// 0, 1, 2, 4 give geometry.  PA: partial assembly, the element's quadrature
// data (qdata[8 * 6][coef_stride] for the Laplace kinds, qdata[8 * 9][coef_stride]
// for elasticity) replaces its geometry (the staged records then hold the
// input only).  Returns false for an empty lane.
template <typename T, int PH, bool PAR, bool PA, bool FX = false>
__device__ __forceinline__ bool step_element(int s, int lane, int max_nodes,
                                             const T *__restrict__ sR, uint4 pk, T c0, T c1,
                                             int64_t coef_stride, const T *__restrict__ qdata,
                                             uint32_t lat, int s_first, int (&lc)[8],
                                             T (&v)[phys_dpn(PH)][8]) {
  constexpr int DPN = phys_dpn(PH);
  constexpr int UOFF = PA ? 0 : 3;  // first input field of a staged record
  if constexpr (FX) {  // the fixed tile: no empty lanes
    corner_fixed<DPN>(s - s_first, lane, lc);
  } else if (lat) {  // lattice tile: corner indices from (step, lane), no corner-index loads
    if (!corner_lattice(lat, s - s_first, lane, lc)) return false;
  } else {
    if (pk.x == 0xffffffffu) return false;
    lc[0] = int(pk.x & 0xffff); lc[1] = int(pk.x >> 16);
    lc[2] = int(pk.y & 0xffff); lc[3] = int(pk.y >> 16);
    lc[4] = int(pk.z & 0xffff); lc[5] = int(pk.z >> 16);
    lc[6] = int(pk.w & 0xffff); lc[7] = int(pk.w >> 16);
  }
  T X[3][8], u[DPN][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T *r = sR + lc[a];
    if (!PA && (!PAR || a == 0 || a == 1 || a == 2 || a == 4)) {
#pragma unroll
      for (int k = 0; k < 3; ++k) X[k][a] = r[size_t(k) * max_nodes];
    }
#pragma unroll
    for (int j = 0; j < DPN; ++j) u[j][a] = r[size_t(UOFF + j) * max_nodes];
  }
  if constexpr (PA && PH == 3) {
    const T *qs = qdata + int64_t(s) * kLanes + lane;
    elasticity_element_pa<T>(
        [&](int q, int m) { return qs[(q * 9 + m) * coef_stride]; }, u, c0, c1, v);
  } else if constexpr (PA) {
    const int64_t slot = int64_t(s) * kLanes + lane;
    T qd[8][6];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int m = 0; m < 6; ++m) qd[q][m] = qdata[(q * 6 + m) * coef_stride + slot];
    laplace_element_pa_n<T, DPN>(qd, u, v);
  } else if constexpr (PAR && PH != 3) {
    laplace_element_parallelepiped_n<T, DPN>(X, u, c0, v);
  } else if constexpr (PAR) {
    elasticity_element_parallelepiped<T>(X, u, c0, c1, v);
  } else {
    element_apply<T, PH>(X, u, c0, c1, v);
  }
  return true;
}

// A wave's steps s, s + 4, ... < s1 of a tile, each added into the LDS
// accumulator myV at once (LDS_ATOMIC: with LDS atomics).
template <typename T, int PH, bool LDS_ATOMIC, bool PAR, bool PA>
__device__ __forceinline__ void block_steps(int s, int s1, int lane, int max_nodes,
                                            const T *__restrict__ sR, T *__restrict__ myV,
                                            const uint4 *__restrict__ lconn,
                                            const T *__restrict__ coef_t, int64_t coef_stride,
                                            uint4 pk_n, T c0_n, T c1_n,
                                            const T *__restrict__ qdata, uint32_t lat,
                                            int s_first) {
  constexpr int DPN = phys_dpn(PH);
  // pk_n, c0_n, c1_n: this wave's first step, loaded by the caller before staging
  for (; s < s1; s += 4) {
    const uint4 pk = pk_n;
    const T c0 = c0_n, c1 = c1_n;
    {  // prefetch this wave's next step (clamped to the current one)
      const int64_t slot = int64_t(s + 4 < s1 ? s + 4 : s) * kLanes + lane;
      if (!lat) pk_n = lconn[slot];
      c0_n = coef_t[slot];
      if constexpr (PH == 3) c1_n = coef_t[coef_stride + slot];
    }
    int lc[8];
    T v[DPN][8];
    if (!step_element<T, PH, PAR, PA>(s, lane, max_nodes, sR, pk, c0, c1, coef_stride, qdata,
                                      lat, s_first, lc, v))
      continue;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int j = 0; j < DPN; ++j) acc_add<T, LDS_ATOMIC>(&myV[j * max_nodes + lc[a]], v[j][a]);
      if constexpr (!LDS_ATOMIC) lane_order();
    }
  }
}

// The split accumulation (bitwise reproducible; the planner's split_ok): the
// wave's steps s0 + w + 4k, k < split_steps(dpn), add their lower corners (a < 4)
// into sV at once and keep the upper ones in registers; after a barrier of
// the whole workgroup they are added in the same order.  All four waves call
// this (it contains the barrier).  par_tile: the tile's elements are all
// parallelepipeds (taken only where PAR_OK; GEN_OK: the general element is
// compiled in).
template <typename T, int PH, bool PAR_OK, bool GEN_OK, bool PA, bool FX = false>
__device__ __forceinline__ void block_steps_split(int s0, int s1, int w, int lane, int max_nodes,
                                                  const T *__restrict__ sR, T *__restrict__ sV,
                                                  const uint4 *__restrict__ lconn,
                                                  const T *__restrict__ coef_t,
                                                  int64_t coef_stride, uint4 pk_n, T c0_n, T c1_n,
                                                  const T *__restrict__ qdata, uint32_t lat,
                                                  bool par_tile) {
  constexpr int DPN = phys_dpn(PH);
  constexpr int kSplitSteps = split_steps(DPN);
  T hold[kSplitSteps][4][DPN];
  int hidx[kSplitSteps][4];
#pragma unroll
  for (int k = 0; k < kSplitSteps; ++k) {
    const int s = s0 + w + 4 * k;
    const uint4 pk = pk_n;
    const T c0 = c0_n, c1 = c1_n;
    if (k + 1 < kSplitSteps) {  // prefetch the wave's next step (clamped, unconditional)
      const int64_t slot = int64_t(min(s + 4, s1 - 1)) * kLanes + lane;
      if (!lat) pk_n = lconn[slot];
      c0_n = coef_t[slot];
      if constexpr (PH == 3) c1_n = coef_t[coef_stride + slot];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) hidx[k][a] = -1;
    if (s >= s1) continue;
    int lc[8];
    T v[DPN][8];
    bool live;
    if constexpr (PA)
      live = step_element<T, PH, false, true>(s, lane, max_nodes, sR, pk, c0, c1, coef_stride,
                                              qdata, lat, s0, lc, v);
    else if constexpr (!GEN_OK)
      live = step_element<T, PH, true, false, FX>(s, lane, max_nodes, sR, pk, c0, c1,
                                                  coef_stride, qdata, lat, s0, lc, v);
    else if (PAR_OK && par_tile)
      live = step_element<T, PH, true, false, FX>(s, lane, max_nodes, sR, pk, c0, c1,
                                                  coef_stride, qdata, lat, s0, lc, v);
    else
      live = step_element<T, PH, false, false, FX>(s, lane, max_nodes, sR, pk, c0, c1,
                                                   coef_stride, qdata, lat, s0, lc, v);
    if (!live) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int j = 0; j < DPN; ++j) sV[j * max_nodes + lc[a]] += v[j][a];
      lane_order();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      hidx[k][a] = lc[4 + a];
#pragma unroll
      for (int j = 0; j < DPN; ++j) hold[k][a][j] = v[j][4 + a];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSplitSteps; ++k)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (hidx[k][a] >= 0) {
#pragma unroll
        for (int j = 0; j < DPN; ++j) sV[j * max_nodes + hidx[k][a]] += hold[k][a][j];
        lane_order();
      }
}

// Accumulation modes of the block kernel: kAccSplit, one LDS accumulator
// filled in two race-free passes (bitwise reproducible; every tile must pass
// split_ok); kAccShared, one accumulator that the four waves add into with
// LDS atomics (FP64 fallback: order of additions varies); kAccCopies, one
// copy per wave, the copies summed in a fixed order (FP32 fallback).
// ALLPAR: every tile of the operator is a parallelepiped tile (flagged at
// set-up), so only the parallelepiped element is compiled in (fewer registers).
// FX: every tile is the kind's fixed lattice tile (FxTile, with the split
// accumulation), whose shape is built in.
constexpr int kAccSplit = 0, kAccShared = 1, kAccCopies = 2;
template <typename T, int PH, bool LDS_ATOMIC, int ACC, bool PA, bool ALLPAR, bool FX = false>
__global__ __launch_bounds__(256) void k_apply_block(
    int max_nodes, int64_t nn, const int32_t *__restrict__ node_ptr,
    const uint32_t *__restrict__ nodes, const int32_t *__restrict__ tile_step,
    const uint4 *__restrict__ lconn, const T *__restrict__ coef_t, int64_t coef_stride,
    const T *__restrict__ xyz, const T *__restrict__ x, T *__restrict__ y,
    const int *__restrict__ stop, const uint8_t *__restrict__ tile_affine,
    const int32_t *__restrict__ slot, T *__restrict__ halo, const T *__restrict__ qdata,
    const uint32_t *__restrict__ tile_lat, const uint32_t *__restrict__ tile_addr,
    const int32_t *__restrict__ tile_g0, int64_t sy, int64_t sz, double *__restrict__ dot_part) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  constexpr int UOFF = PA ? 0 : 3;
  constexpr int NR = UOFF + DPN;  // [x, y, z,] u[DPN], stored field by field
  using FT = FxTile<DPN>;
  // node records per thread issued together (all of a fixed tile, else 1024 per round)
  constexpr int KN = FX ? (FT::NODES + 255) / 256 : 4;
  static_assert(!FX || (ACC == kAccSplit && !PA), "FX instance");
  // the LDS stride of a field: a constant on the fixed tile
  const int MN = FX ? FT::NODES : max_nodes;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sR = reinterpret_cast<T *>(smem_raw);  // [NR][MN]
  constexpr bool ONEACC = ACC != kAccCopies;
  constexpr int NACC = ONEACC ? 1 : 4;
  T *sV = sR + size_t(NR) * MN;              // [NACC][DPN][MN]
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int tile = xcd_block_t(blockIdx.x, gridDim.x);
  const int n0 = node_ptr[tile], nm = FX ? FT::NODES : node_ptr[tile + 1] - n0;
  const int s0 = tile_step[tile], s1 = FX ? s0 + FT::STEPS : tile_step[tile + 1];
  const uint32_t lat = FX ? FT::LAT : tile_lat[tile], addr = tile_addr[tile];
  const int64_t g0 = tile_g0[tile];
  // node word of entry i: computed on lattice-addressed tiles, else loaded
  auto word = [&](int i) -> uint32_t {
    if constexpr (FX)
      return addr ? lattice_word_fixed<DPN>(i, addr, g0, sy, sz) : nodes[n0 + i];
    else
      return addr ? lattice_word(i, lat, addr, g0, sy, sz) : nodes[n0 + i];
  };
  // the wave's first step: requested after the first staging round's loads, so
  // that the waits of that round's LDS writes do not include it (its latency
  // overlaps them and the barrier)
  uint4 pk0 = make_uint4(0xffffffffu, 0u, 0u, 0u);
  T c00 = T(0), c10 = T(0);
  // (unconditional, at a clamped step, since a load under a branch makes the
  // compiler wait for it at the branch's end; a wave without steps never uses it)
  auto first_step = [&]() {
    const int64_t slot = int64_t(min(s0 + w, s1 - 1)) * kLanes + lane;
    if (!lat) pk0 = lconn[slot];
    c00 = coef_t[slot];
    if constexpr (PH == 3) c10 = coef_t[coef_stride + slot];
  };
  // stage the node records: all loads of a round are issued (unconditionally,
  // at clamped indices) before any LDS write, so the round costs one latency.
  // The first round's node words stay in registers for the write-back.
  uint32_t keep[KN];
  int32_t kslot[KN];
  for (int base = 0; base < nm; base += KN * 256) {
    uint32_t raw[KN];
    T rec[KN][NR];
#pragma unroll
    for (int k = 0; k < KN; ++k) raw[k] = word(min(base + k * 256 + tid, nm - 1));
    if (base == 0) {
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        keep[k] = raw[k];
        // slots are only used for shared entries (known at once on lattice-addressed
        // tiles): the other lanes load the tile's first slot, one line per wavefront.
        // The load is unconditional so that nothing waits for it before the write-back.
        const int sl = n0 + min(k * 256 + tid, nm - 1);
        kslot[k] = slot[!addr || (raw[k] & kSharedBit) ? sl : n0];
      }
    }
#pragma unroll
    for (int k = 0; k < KN; ++k) {
      const int64_t g = raw[k] & kIdMask;
      if constexpr (!PA) {
        rec[k][0] = xyz[g];
        rec[k][1] = xyz[nn + g];
        rec[k][2] = xyz[2 * nn + g];
      }
#pragma unroll
      for (int j = 0; j < DPN; ++j) rec[k][UOFF + j] = x[g * DPN + j];
    }
    if (base == 0) first_step();
#pragma unroll
    for (int k = 0; k < KN; ++k) {
      const int i = base + k * 256 + tid;
      if (i < nm) {
        const bool fixed = (raw[k] & kFixedBit) != 0;
#pragma unroll
        for (int f = 0; f < UOFF; ++f) sR[size_t(f) * MN + i] = rec[k][f];
#pragma unroll
        for (int j = 0; j < DPN; ++j)
          sR[size_t(UOFF + j) * MN + i] = fixed ? T(0) : rec[k][UOFF + j];
#pragma unroll
        for (int c = 0; c < NACC * DPN; ++c) sV[size_t(c) * MN + i] = T(0);
      }
    }
  }
  __syncthreads();
  if constexpr (ACC == kAccSplit) {
    block_steps_split<T, PH, !PA, !ALLPAR, PA, FX>(s0, s1, w, lane, MN, sR, sV, lconn, coef_t,
                                                   coef_stride, pk0, c00, c10, qdata, lat,
                                                   !PA && !ALLPAR && tile_affine[tile]);
  } else {
    constexpr bool AT = LDS_ATOMIC || ACC == kAccShared;
    T *myV = ONEACC ? sV : sV + size_t(w) * DPN * max_nodes;
    if constexpr (ALLPAR && !PA) {
      block_steps<T, PH, AT, true, false>(s0 + w, s1, lane, max_nodes, sR, myV, lconn, coef_t,
                                          coef_stride, pk0, c00, c10, qdata, lat, s0);
    } else {
      if (!PA && tile_affine[tile])
        block_steps<T, PH, AT, true, PA>(s0 + w, s1, lane, max_nodes, sR, myV, lconn, coef_t,
                                         coef_stride, pk0, c00, c10, qdata, lat, s0);
      else
        block_steps<T, PH, AT, false, PA>(s0 + w, s1, lane, max_nodes, sR, myV, lconn, coef_t,
                                          coef_stride, pk0, c00, c10, qdata, lat, s0);
    }
  }
  __syncthreads();
  // nodes of this tile only: y; nodes shared with other tiles: this tile's halo
  // slot (summed by k_halo_sum); Dirichlet nodes: written by k_halo_sum.
  // dot_part: this tile's share of x.y, over the nodes it writes to y
  double dsum = 0.0;
  auto write_node = [&](int i, uint32_t raw, int32_t sl) {
    if (raw & kFixedBit) return;
    const int64_t gg = raw & kIdMask;
#pragma unroll
    for (int j = 0; j < DPN; ++j) {
      const size_t o = size_t(j) * MN + i, cs = size_t(DPN) * MN;
      T v;
      if constexpr (ONEACC)
        v = sV[o];
      else
        v = (sV[o] + sV[cs + o]) + (sV[2 * cs + o] + sV[3 * cs + o]);
      if (raw & kSharedBit) {
        halo[int64_t(sl) * DPN + j] = v;
      } else {
        y[gg * DPN + j] = v;
        if (dot_part) dsum += double(sR[size_t(UOFF + j) * MN + i]) * double(v);
      }
    }
  };
#pragma unroll
  for (int k = 0; k < KN; ++k)
    if (k * 256 + tid < nm) write_node(k * 256 + tid, keep[k], kslot[k]);
  for (int i = KN * 256 + tid; i < nm; i += 256) write_node(i, word(i), slot[n0 + i]);
  if (dot_part) {
    const double t = block_sum_256(dsum);
    if (tid == 0) dot_part[tile] = t;
  }
}

// ---------------------------------------------------------------------------
// Owner-computes tiles: the scalar Laplace operator on a box lattice of
// parallelepipeds (element e = ex + nx (ey + ny ez), node i + (nx+1)(j +
// (ny+1) k), local corner a = i + 2j + 4k), nx, ny, nz multiples of 16, 8, 4.
// A workgroup owns a 16 x 8 x 4 box of nodes (the last tile in a direction
// also owns the mesh's last node plane in it) and computes every element that
// touches them: 17 x 9 x 5 elements over the 18 x 10 x 6 staged nodes.  What
// an element adds to a node outside the box is dropped, so every entry of y is
// written once, with a plain store, by the tile that owns it: no halo slots
// and no second kernel, for 765 element evaluations per 512 owned nodes (the
// shell of elements around the box is computed by both tiles beside it).
//
// Order of the additions (bitwise reproducible).  Wave w computes element
// layer w + 1 of the box (153 elements, box row-major) and the w-th quarter of
// layer 0 (elements [38w, 38(w+1)) of it, the last quarter up to 153), in three
// steps of 64 lanes.  Pass L adds the lower corners of layer w + 1 into node
// plane w + 1 (at once, as each step is computed); after a barrier pass U1 adds
// the upper corners of layer w + 1 into plane w + 2 and those of the layer-0
// quarters of waves 0 and 2 into plane 1; after another, pass U2 adds those of
// the quarters of waves 1 and 3 into plane 1.  A quarter spans more than two
// element rows, so quarters 0 and 2 (and 1 and 3) share no node; in every pass
// each node receives additions from one wavefront, whose LDS adds execute in
// program order, and within one instruction the lanes' nodes are distinct.
// The accumulator is FP64 in both precisions (FP32 LDS atomic adds measured
// slow here).
// Loads and stores at a 32-bit byte offset from a base pointer held in scalar
// registers (one address operand per access instead of a 64-bit vector address).
template <typename E>
__device__ __forceinline__ E ld_off(const E *base, uint32_t byte_off) {
  return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename E>
__device__ __forceinline__ void st_off(E *base, uint32_t byte_off, E v) {
  *reinterpret_cast<E *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

struct OwnTile {
  static constexpr int OX = 16, OY = 8, OZ = 4;              // owned nodes
  static constexpr int AX = OX + 1, AY = OY + 1, AZ = OZ + 1;  // accumulator box
  static constexpr int EX = OX + 1, EY = OY + 1;              // elements per layer
  static constexpr int SX = OX + 2, SY = OY + 2, SZ = OZ + 2;  // staged nodes
  static constexpr int NS = SX * SY * SZ;
  static constexpr int NL = EX * EY;                          // 153
  static constexpr int NA = AX * AY * AZ;
  static constexpr int KN = (NS + 255) / 256;
  static_assert((KN - 1) * 256 <= NS, "staging rounds before the last are full");
  static constexpr int NQ = NL / 4;  // elements of a layer-0 quarter (the last one: the rest)
  static_assert(NL <= 192 && NL + (NL - 3 * NQ) <= 192, "three steps per wave");
  static_assert(NQ > 2 * EX, "quarters 0 and 2 (1 and 3) share no node");
};

__device__ __forceinline__ void lds_add_own(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Element kinds of the owner-computes tiles: the parallelepiped hexahedron; the
// general hexahedron (isoparametric geometry at each Gauss point, all 8 corners'
// coordinates), taken on small meshes whose elements are not all parallelepipeds,
// where one kernel per apply matters more than the element work; the six linear
// tetrahedra of a cell's Kuhn split (tetrahedron t of cell e is element 6e + t,
// with the cell corners of kKuhn[t]), their sum acting as the cell's element; and
// the diagonal of that sum (no input; y is the diagonal, 1 on Dirichlet nodes).
constexpr int kOwnPar = 0, kOwnGen = 1, kOwnKuhn = 2, kOwnKuhnDiag = 3;
__device__ constexpr int kKuhn[6][4] = {{0, 1, 3, 7}, {0, 5, 1, 7}, {0, 3, 2, 7},
                                        {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}};

template <typename T, bool MASK, int EK>
__global__ __launch_bounds__(256) void k_apply_owner(int nx, int ny, int nz,
                                                     const T *__restrict__ xyz,
                                                     const T *__restrict__ coef,
                                                     const uint8_t *__restrict__ mask,
                                                     const T *__restrict__ x, T *__restrict__ y,
                                                     const int *__restrict__ stop,
                                                     double *__restrict__ dot_part) {
  using F = OwnTile;
  constexpr int NC = EK >= kOwnKuhn ? 6 : 1;  // cell coefficients
  constexpr bool ALLX = EK != kOwnPar;          // all 8 corners' coordinates
  if (stop && *stop) return;
  __shared__ T sR[4 * F::NS];   // x, y, z, input (0 on Dirichlet nodes), field by field
  __shared__ double sV[F::NA];  // accumulator over the owned box
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int tile = xcd_block_t(blockIdx.x, gridDim.x);
  const int ntx = nx / F::OX, nty = ny / F::OY, ntz = nz / F::OZ;
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int hx = F::OX + (tx == ntx - 1), hy = F::OY + (ty == nty - 1),
            hz = F::OZ + (tz == ntz - 1);
  const int n1x = nx + 1, n1y = ny + 1;
  const int64_t nn = int64_t(n1x) * n1y * (nz + 1);
  // global lattice position of local node / element (0, 0, 0)
  const int gx0 = tx * F::OX - 1, gy0 = ty * F::OY - 1, gz0 = tz * F::OZ - 1;
  // ids and byte offsets in 32 bits (the host takes this kernel for fewer than
  // 2^32 bytes per field), each field's base in scalar registers
  const T *X0 = xyz, *X1 = xyz + nn, *X2 = xyz + 2 * nn;
  // stage the node records: every load issued (at clamped positions) before any
  // LDS write.  gk, ak: the record's node id, and its accumulator entry when this
  // tile owns the node (else -1); kept with the record for the write-back.
  T rec[F::KN][4];
  uint32_t fx[F::KN];  // the Dirichlet byte, kept raw: a compare at the load would wait for it
  uint32_t gk[F::KN];
  int ak[F::KN];
#pragma unroll
  for (int k = 0; k < F::KN; ++k) {
    const int ii = k * 256 + tid, i = min(ii, F::NS - 1);
    const int c = i / (F::SX * F::SY), r = i - c * (F::SX * F::SY), b = r / F::SX,
              a = r - b * F::SX;
    // 24-bit products (the host checks the factors' range): a 32-bit multiply-add
    // in the wider form reads a neighbouring register, which then waits for a load
    const uint32_t g = __umul24(uint32_t(n1x), __umul24(uint32_t(n1y),
                                                        uint32_t(min(max(gz0 + c, 0), nz))) +
                                                   uint32_t(min(max(gy0 + b, 0), ny))) +
                       uint32_t(min(max(gx0 + a, 0), nx));
    const uint32_t o = g * uint32_t(sizeof(T));
    rec[k][0] = ld_off(X0, o);
    rec[k][1] = ld_off(X1, o);
    rec[k][2] = ld_off(X2, o);
    rec[k][3] = EK == kOwnKuhnDiag ? T(0) : ld_off(x, o);
    fx[k] = MASK ? uint32_t(ld_off(mask, g)) : 0u;
    gk[k] = g;
    // (range tests as unsigned compares joined without short-circuit: no branches)
    const bool own = (ii < F::NS) & (unsigned(a - 1) < unsigned(hx)) &
                     (unsigned(b - 1) < unsigned(hy)) & (unsigned(c - 1) < unsigned(hz));
    ak[k] = own ? (a - 1) + F::AX * ((b - 1) + F::AY * (c - 1)) : -1;
  }
  // the wave's three steps: element (ea, eb, ec) of the box, its mask of owned
  // corners (bits 0-3 lower, 4-7 upper; the layer-0 quarters of odd waves
  // carry their upper corners in bits 8-11, for pass U2) and its cell's byte offset
  const int q0 = F::NQ * w, q1 = w == 3 ? F::NL : F::NQ * (w + 1);
  int ea[3], eb[3], ec[3];
  unsigned msk[3];
  uint32_t eo[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int j = k * 64 + lane;
    const bool own_layer = j < F::NL;
    const int qj = q0 + j - F::NL;
    const int lin = own_layer ? j : min(qj, F::NL - 1);
    ec[k] = own_layer ? w + 1 : 0;
    eb[k] = lin / F::EX;
    ea[k] = lin - eb[k] * F::EX;
    const int gx = gx0 + ea[k], gy = gy0 + eb[k], gz = gz0 + ec[k];
    const bool live = (own_layer | (qj < q1)) & (unsigned(gx) < unsigned(nx)) &
                      (unsigned(gy) < unsigned(ny)) & (unsigned(gz) < unsigned(nz));
    // corner a = i + 2j + 4k is owned when its x, y and z positions are: the
    // corners with i = 0 are bits 0x55, i = 1 0xaa; j = 0 0x33, j = 1 0xcc; k = 0
    // 0x0f, k = 1 0xf0
    const unsigned bx = (ea[k] >= 1 ? 0x55u : 0u) | (ea[k] + 1 <= hx ? 0xaau : 0u);
    const unsigned by = (eb[k] >= 1 ? 0x33u : 0u) | (eb[k] + 1 <= hy ? 0xccu : 0u);
    const unsigned bz = (ec[k] >= 1 ? 0x0fu : 0u) | (ec[k] + 1 <= hz ? 0xf0u : 0u);
    unsigned m = bx & by & bz;
    if (!own_layer && (w & 1)) m = (m & 0x0fu) | ((m & 0xf0u) << 4);
    msk[k] = live ? m : 0u;
    eo[k] = (__umul24(uint32_t(nx), __umul24(uint32_t(ny), uint32_t(min(max(gz, 0), nz - 1))) +
                                        uint32_t(min(max(gy, 0), ny - 1))) +
             uint32_t(min(max(gx, 0), nx - 1))) *
            uint32_t(NC * sizeof(T));
  }
  T cnext[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) cnext[t] = ld_off(coef, eo[0] + uint32_t(t * sizeof(T)));
#pragma unroll
  for (int k = 0; k < F::KN; ++k) {
    const int i = k * 256 + tid;
    if (k < F::KN - 1 || i < F::NS) {  // only the last round is partial
#pragma unroll
      for (int f = 0; f < 3; ++f) sR[f * F::NS + i] = rec[k][f];
      sR[3 * F::NS + i] = fx[k] != 0 ? T(0) : rec[k][3];
    }
  }
  for (int i = tid; i < F::NA; i += 256) sV[i] = 0.0;
  __syncthreads();
  double hold[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T c[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) c[t] = cnext[t];
    if (k < 2) {
#pragma unroll
      for (int t = 0; t < NC; ++t) cnext[t] = ld_off(coef, eo[k + 1] + uint32_t(t * sizeof(T)));
    }
    const T *r = sR + (ea[k] + F::SX * (eb[k] + F::SY * ec[k]));
    T X[3][8], u[1][8], v[1][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int o = (a & 1) + F::SX * ((a >> 1) & 1) + F::SX * F::SY * (a >> 2);
      if (ALLX || a == 0 || a == 1 || a == 2 || a == 4) {
#pragma unroll
        for (int d = 0; d < 3; ++d) X[d][a] = r[d * F::NS + o];
      }
      u[0][a] = r[3 * F::NS + o];
    }
    if constexpr (EK == kOwnGen) {
      laplace_element_n<T, 1>(X, u, c[0], v);
    } else if constexpr (EK == kOwnPar) {
      laplace_element_parallelepiped_n<T, 1>(X, u, c[0], v);
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a) v[0][a] = T(0);
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        T Xt[3][4], ut[1][4], vt[1][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int d = 0; d < 3; ++d) Xt[d][q] = X[d][kKuhn[t][q]];
          ut[0][q] = u[0][kKuhn[t][q]];
        }
        if constexpr (EK == kOwnKuhn) {
          tet_element<T, 1>(Xt, ut, c[t], T(0), vt);
        } else {  // diagonal: k |c_q|^2 / (6 det) with c_q the scaled gradient of corner q
          const T E1[3] = {Xt[0][1] - Xt[0][0], Xt[1][1] - Xt[1][0], Xt[2][1] - Xt[2][0]};
          const T E2[3] = {Xt[0][2] - Xt[0][0], Xt[1][2] - Xt[1][0], Xt[2][2] - Xt[2][0]};
          const T E3[3] = {Xt[0][3] - Xt[0][0], Xt[1][3] - Xt[1][0], Xt[2][3] - Xt[2][0]};
          T g[4][3];
          cross(E2, E3, g[1]);
          cross(E3, E1, g[2]);
          cross(E1, E2, g[3]);
#pragma unroll
          for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
          const T ks = c[t] * rcp(T(6) * dot3(E1, g[1]));
#pragma unroll
          for (int q = 0; q < 4; ++q) vt[0][q] = ks * dot3(g[q], g[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v[0][kKuhn[t][q]] += vt[0][q];
      }
    }
    // accumulator entry of the element's corner 0 (may lie outside the box; only
    // owned corners are addressed)
    double *acc = sV + ((ea[k] - 1) + F::AX * ((eb[k] - 1) + F::AY * (ec[k] - 1)));
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (msk[k] & (1u << a)) lds_add_own(acc + (a & 1) + F::AX * ((a >> 1) & 1), double(v[0][a]));
#pragma unroll
    for (int a = 0; a < 4; ++a) hold[k][a] = double(v[0][4 + a]);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double *acc = sV + ((ea[k] - 1) + F::AX * ((eb[k] - 1) + F::AY * ec[k]));
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (msk[k] & (16u << a)) lds_add_own(acc + (a & 1) + F::AX * ((a >> 1) & 1), hold[k][a]);
  }
  __syncthreads();
  if (w & 1) {  // layer-0 lanes are in the last step only
    double *acc = sV + ((ea[2] - 1) + F::AX * ((eb[2] - 1) + F::AY * ec[2]));
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (msk[2] & (256u << a)) lds_add_own(acc + (a & 1) + F::AX * ((a >> 1) & 1), hold[2][a]);
  }
  __syncthreads();
  // write-back: each thread stores the owned nodes among the records it staged
  // (their ids, Dirichlet flags and input values are still in registers), so no
  // global load waits at the end; dot_part: this tile's share of x.y
  double dsum = 0.0;
#pragma unroll
  for (int k = 0; k < F::KN; ++k) {
    if (ak[k] >= 0) {
      const T yv = fx[k] != 0 ? (EK == kOwnKuhnDiag ? T(1) : rec[k][3]) : T(sV[ak[k]]);
      st_off(y, gk[k] * uint32_t(sizeof(T)), yv);
      if (dot_part) dsum += double(rec[k][3]) * double(yv);
    }
  }
  if (dot_part) {
    const double t = block_sum_256(dsum);
    if (tid == 0) dot_part[tile] = t;
  }
}

// Byte offset of the tetrahedron kernel's FP64 accumulator after the node
// records (rec_bytes per node), rounded up to 8 bytes.
__host__ __device__ inline size_t tet_acc_offset(int max_nodes, size_t rec_bytes) {
  return (size_t(max_nodes) * rec_bytes + 7) & ~size_t(7);
}

// Block apply of linear tetrahedra: the block kernel's staging, write-back
// and halo slots with the tetrahedron's element (tet_element); a tile is a
// brick of cells' tetrahedra, wave w takes its steps w, w + 4, ... and adds
// each tetrahedron's 4 corner contributions into one FP64 LDS accumulator with
// LDS atomics (the order of those additions varies; FP64 in both precisions,
// since the FP32 LDS atomic add measured twice as slow here).
template <typename T, int PH>
__global__ __launch_bounds__(256) void k_apply_block_tet(
    int max_nodes, int64_t nn, const int32_t *__restrict__ node_ptr,
    const uint32_t *__restrict__ nodes, const int32_t *__restrict__ tile_step,
    const uint4 *__restrict__ lconn, const T *__restrict__ coef_t, int64_t coef_stride,
    const T *__restrict__ xyz, const T *__restrict__ x, T *__restrict__ y,
    const int *__restrict__ stop, const int32_t *__restrict__ slot, T *__restrict__ halo) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  constexpr int NR = 3 + DPN;
  constexpr int KN = 4;  // node records per thread issued together (1024 per round)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sR = reinterpret_cast<T *>(smem_raw);  // [NR][max_nodes]
  // the accumulator is FP64 in both precisions ([DPN][max_nodes], 8-byte aligned)
  double *sV = reinterpret_cast<double *>(smem_raw + tet_acc_offset(max_nodes, NR * sizeof(T)));
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int tile = xcd_block_t(blockIdx.x, gridDim.x);
  const int n0 = node_ptr[tile], nm = node_ptr[tile + 1] - n0;
  const int s0 = tile_step[tile], s1 = tile_step[tile + 1];
  // staging: all loads of a round (node words, then coordinates, input and the
  // halo slots of shared entries) are issued before any LDS write; the first
  // round's words and slots stay in registers for the write-back
  uint32_t keep[KN];
  int32_t kslot[KN];
  for (int base = 0; base < nm; base += KN * 256) {
    uint32_t raw[KN];
    int32_t sl[KN];
    T rec[KN][NR];
#pragma unroll
    for (int k = 0; k < KN; ++k) raw[k] = nodes[n0 + min(base + k * 256 + tid, nm - 1)];
#pragma unroll
    for (int k = 0; k < KN; ++k) {
      const int64_t g = raw[k] & kIdMask;
#pragma unroll
      for (int r = 0; r < 3; ++r) rec[k][r] = xyz[r * nn + g];
#pragma unroll
      for (int j = 0; j < DPN; ++j) rec[k][3 + j] = x[g * DPN + j];
      sl[k] = slot[raw[k] & kSharedBit ? n0 + min(base + k * 256 + tid, nm - 1) : n0];
    }
    if (base == 0) {
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        keep[k] = raw[k];
        kslot[k] = sl[k];
      }
    }
#pragma unroll
    for (int k = 0; k < KN; ++k) {
      const int i = base + k * 256 + tid;
      if (i < nm) {
        const bool fixed = (raw[k] & kFixedBit) != 0;
#pragma unroll
        for (int r = 0; r < 3; ++r) sR[size_t(r) * max_nodes + i] = rec[k][r];
#pragma unroll
        for (int j = 0; j < DPN; ++j) {
          sR[size_t(3 + j) * max_nodes + i] = fixed ? T(0) : rec[k][3 + j];
          sV[size_t(j) * max_nodes + i] = 0.0;
        }
      }
    }
  }
  __syncthreads();
  // steps w, w + 4, ...: each step's corner indices and coefficients are
  // requested one step ahead (at a clamped step, unconditionally)
  int s = s0 + w;
  int64_t sl0 = int64_t(min(s, s1 - 1)) * kLanes + lane;
  uint4 pk = lconn[sl0];
  T c0 = coef_t[sl0], c1 = PH == 3 ? coef_t[coef_stride + sl0] : T(0);
  for (; s < s1; s += 4) {
    const int64_t sn = int64_t(min(s + 4, s1 - 1)) * kLanes + lane;
    const uint4 pkn = lconn[sn];
    const T c0n = coef_t[sn], c1n = PH == 3 ? coef_t[coef_stride + sn] : T(0);
    if (pk.x != 0xffffffffu) {  // empty lanes skip
      const int lc[4] = {int(pk.x & 0xffff), int(pk.x >> 16), int(pk.y & 0xffff),
                         int(pk.y >> 16)};
      T X[3][4], u[DPN][4], v[DPN][4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int r = 0; r < 3; ++r) X[r][a] = sR[size_t(r) * max_nodes + lc[a]];
#pragma unroll
        for (int j = 0; j < DPN; ++j) u[j][a] = sR[size_t(3 + j) * max_nodes + lc[a]];
      }
      tet_element<T, PH>(X, u, c0, c1, v);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < DPN; ++j)
          lds_add(&sV[size_t(j) * max_nodes + lc[a]], double(v[j][a]));
    }
    pk = pkn;
    c0 = c0n;
    c1 = c1n;
  }
  __syncthreads();
  auto write_node = [&](int i, uint32_t raw, int32_t sl) {
    if (raw & kFixedBit) return;  // y = x written by k_halo_sum
    const int64_t g = raw & kIdMask;
#pragma unroll
    for (int j = 0; j < DPN; ++j) {
      const T v = T(sV[size_t(j) * max_nodes + i]);
      if (raw & kSharedBit)
        halo[int64_t(sl) * DPN + j] = v;
      else
        y[g * DPN + j] = v;
    }
  };
#pragma unroll
  for (int k = 0; k < KN; ++k)
    if (k * 256 + tid < nm) write_node(k * 256 + tid, keep[k], kslot[k]);
  for (int i = KN * 256 + tid; i < nm; i += 256) write_node(i, nodes[n0 + i], slot[n0 + i]);
}

// Diagonal of A on the block variants' tiles with the split accumulation
// (bitwise reproducible): one workgroup per tile stages the coordinates,
// each element's diagonal entries (element_diag) are added into LDS in the
// two race-free passes of the apply, and the tile's nodes are written like
// the apply's (tile-private nodes to d, shared ones to halo slots summed by
// k_halo_sum, which writes 1 on Dirichlet nodes).
template <typename T, int PH>
__global__ __launch_bounds__(256) void k_diag_block(
    int max_nodes, int64_t nn, const int32_t *__restrict__ node_ptr,
    const uint32_t *__restrict__ nodes, const int32_t *__restrict__ tile_step,
    const uint4 *__restrict__ lconn, const T *__restrict__ coef_t, int64_t coef_stride,
    const T *__restrict__ xyz, T *__restrict__ d, const int32_t *__restrict__ slot,
    T *__restrict__ halo, const uint32_t *__restrict__ tile_lat) {
  constexpr int DPN = phys_dpn(PH);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sR = reinterpret_cast<T *>(smem_raw);  // [3][max_nodes]
  T *sV = sR + size_t(3) * max_nodes;       // [DPN][max_nodes]
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int tile = blockIdx.x;
  const int n0 = node_ptr[tile], nm = node_ptr[tile + 1] - n0;
  const int s0 = tile_step[tile], s1 = tile_step[tile + 1];
  const uint32_t lat = tile_lat[tile];
  for (int i = tid; i < nm; i += 256) {
    const int64_t g = nodes[n0 + i] & kIdMask;
#pragma unroll
    for (int r = 0; r < 3; ++r) sR[size_t(r) * max_nodes + i] = xyz[r * nn + g];
#pragma unroll
    for (int j = 0; j < DPN; ++j) sV[size_t(j) * max_nodes + i] = T(0);
  }
  __syncthreads();
  constexpr int kSplitSteps = split_steps(DPN);
  T hold[kSplitSteps][4][DPN];
  int hidx[kSplitSteps][4];
#pragma unroll
  for (int k = 0; k < kSplitSteps; ++k) {
    const int s = s0 + w + 4 * k;
#pragma unroll
    for (int a = 0; a < 4; ++a) hidx[k][a] = -1;
    if (s >= s1) continue;
    const int64_t sl = int64_t(s) * kLanes + lane;
    int lc[8];
    if (lat) {
      if (!corner_lattice(lat, s - s0, lane, lc)) continue;
    } else {
      const uint4 pk = lconn[sl];
      if (pk.x == 0xffffffffu) continue;
      lc[0] = int(pk.x & 0xffff); lc[1] = int(pk.x >> 16);
      lc[2] = int(pk.y & 0xffff); lc[3] = int(pk.y >> 16);
      lc[4] = int(pk.z & 0xffff); lc[5] = int(pk.z >> 16);
      lc[6] = int(pk.w & 0xffff); lc[7] = int(pk.w >> 16);
    }
    T X[3][8], v[DPN][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int r = 0; r < 3; ++r) X[r][a] = sR[size_t(r) * max_nodes + lc[a]];
    element_diag<T, PH>(X, coef_t[sl], PH == 3 ? coef_t[coef_stride + sl] : T(0), v);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int j = 0; j < DPN; ++j) sV[j * max_nodes + lc[a]] += v[j][a];
      lane_order();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      hidx[k][a] = lc[4 + a];
#pragma unroll
      for (int j = 0; j < DPN; ++j) hold[k][a][j] = v[j][4 + a];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSplitSteps; ++k)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (hidx[k][a] >= 0) {
#pragma unroll
        for (int j = 0; j < DPN; ++j) sV[j * max_nodes + hidx[k][a]] += hold[k][a][j];
        lane_order();
      }
  __syncthreads();
  for (int i = tid; i < nm; i += 256) {
    const uint32_t raw = nodes[n0 + i];
    if (raw & kFixedBit) continue;
    const int64_t g = raw & kIdMask;
    const int32_t sl = slot[n0 + i];
#pragma unroll
    for (int j = 0; j < DPN; ++j) {
      const T v = sV[size_t(j) * max_nodes + i];
      if (raw & kSharedBit)
        halo[int64_t(sl) * DPN + j] = v;
      else
        d[g * DPN + j] = v;
    }
  }
}

// Second pass of the block variant over the reset list: y = x on Dirichlet
// nodes (1 when x is NULL: the diagonal), 0 on nodes that no element references, otherwise the sum of the
// node's halo slots in tile order (slots j and
// n + j, then the extra slots of edge and corner nodes), so every entry of y
// is written exactly once.  Each thread takes kHaloNpt nodes (a block's nodes
// are contiguous) and issues all their loads before summing; two per thread
// measured faster than four (more waves in flight for the one memory round).
constexpr int kHaloNpt = 2;
template <typename T, int DPN>
__global__ __launch_bounds__(256) void k_halo_sum(int64_t n, const int32_t *__restrict__ hnode,
                                                  const int32_t *__restrict__ hptr,
                                                  const T *__restrict__ x,
                                                  const T *__restrict__ halo,
                                                  T *__restrict__ y,
                                                  const int *__restrict__ stop,
                                                  double *__restrict__ dot_part,
                                                  const double *__restrict__ tile_part,
                                                  int64_t n_tiles) {
  if (stop && *stop) return;
  const int64_t base = int64_t(blockIdx.x) * 256 * kHaloNpt + threadIdx.x;
  int64_t jj[kHaloNpt];
  int32_t h[kHaloNpt], e0[kHaloNpt], e1[kHaloNpt];
#pragma unroll
  for (int p = 0; p < kHaloNpt; ++p) {
    jj[p] = min(base + p * 256, n - 1);
    h[p] = hnode[jj[p]];
    e0[p] = hptr[jj[p]];
    e1[p] = hptr[jj[p] + 1];
  }
  T acc[kHaloNpt][DPN];
#pragma unroll
  for (int p = 0; p < kHaloNpt; ++p)
#pragma unroll
    for (int c = 0; c < DPN; ++c)  // (read but unused on Dirichlet nodes)
      acc[p][c] = halo[jj[p] * DPN + c] + halo[(n + jj[p]) * DPN + c];
#pragma unroll
  for (int p = 0; p < kHaloNpt; ++p)
    for (int32_t k = e0[p]; k < e1[p]; ++k)
#pragma unroll
      for (int c = 0; c < DPN; ++c) acc[p][c] += halo[(2 * n + k) * DPN + c];
  double dsum = 0.0;
#pragma unroll
  for (int p = 0; p < kHaloNpt; ++p) {
    if (base + p * 256 >= n) continue;
    const bool fixed = h[p] < 0, orphan = (h[p] & 0x40000000) != 0;
    const int64_t g = h[p] & 0x3fffffff;
#pragma unroll
    for (int c = 0; c < DPN; ++c) {
      const T v = fixed ? (x ? x[g * DPN + c] : T(1)) : orphan ? T(0) : acc[p][c];
      y[g * DPN + c] = v;
      if (dot_part) dsum += double(x[g * DPN + c]) * double(v);
    }
  }
  // dot_part: x.y over this workgroup's nodes plus its range of the tile partials
  if (dot_part) {
    const int64_t t0 = n_tiles * blockIdx.x / gridDim.x;
    const int64_t t1 = n_tiles * (blockIdx.x + 1) / gridDim.x;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) dsum += tile_part[t];
    const double tot = block_sum_256(dsum);
    if (threadIdx.x == 0) dot_part[blockIdx.x] = tot;
  }
}

// Partial-assembly set-up: the quadrature data of the element in each lane
// slot (zero for empty slots), stored [8 * NQ][n_slots] so that a step's loads
// are contiguous: NQ = 6 (Laplace kinds, the cell coefficient folded in) or 9
// (elasticity, the scaled adjugate; lambda and mu stay per cell).
template <typename T, int NQ>
__global__ void k_pa_setup(int64_t n_slots, const int32_t *__restrict__ slot_elem, int64_t ne,
                           int64_t nn, const int32_t *__restrict__ conn,
                           const T *__restrict__ xyz, const T *__restrict__ coef,
                           T *__restrict__ qdata) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const int32_t e = slot_elem[i];
  T qd[8][NQ];
  if (e < 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int m = 0; m < NQ; ++m) qd[q][m] = T(0);
  } else {
    T X[3][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int64_t g = conn[a * ne + e];
#pragma unroll
      for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + g];
    }
    if constexpr (NQ == 6)
      laplace_qdata<T>(X, coef[e], qd);
    else
      elasticity_qdata<T>(X, qd);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int m = 0; m < NQ; ++m) qdata[(q * NQ + m) * n_slots + i] = qd[q][m];
}

namespace {

struct HostTiles {
  std::vector<int32_t> node_ptr{0}, tile_step{0}, reset;
  std::vector<uint32_t> nodes;
  std::vector<uint16_t> lconn;
  std::vector<int32_t> step_elem;  // element of each lane slot (-1 = empty)
  int max_nodes = 0;
  bool corner_collision = false;   // two lanes of a step share a node at one corner
  std::vector<uint8_t> tile_affine;  // every element of the tile is a parallelepiped
  std::vector<int32_t> slot, hptr, hnode;  // halo slots of the block variant
  std::vector<uint32_t> tile_lat;    // lattice description of each tile (0: none)
  bool split = true;                 // every tile admits the split accumulation
  std::vector<uint32_t> tile_addr;   // lattice addressing: kAddrValid | face bits, or 0
  std::vector<int32_t> tile_g0;      // global id of a lattice-addressed tile's entry 0
  int64_t sy = 0, sz = 0;            // the mesh strides lattice addressing uses
};

// Lattice tiles: the tile's elements form an A x B x C brick, its node list is
// the (A+1) x (B+1) x (C+1) lattice in x-fastest order, and each layer's A*B
// elements are taken x-fastest in runs of 64 (spl steps per layer) in the
// interleaved layout (layer l on wave l mod 4, wave w's k-th step at position
// 4k + w).  Then the corner indices of lane l at position p follow from (p, l)
// alone (corner_lattice) and the kernel computes them instead of loading
// them.  Returns A | B << 8 | spl << 16 | C << 24 when every element, corner
// and empty lane of tile t matches, else 0.
uint32_t lattice_of(const HostTiles &H, int t) {
  const int s0 = H.tile_step[t], s1 = H.tile_step[t + 1];
  const int nm = H.node_ptr[t + 1] - H.node_ptr[t];
  const uint16_t *L0 = &H.lconn[size_t(s0) * kLanes * 8];
  if (L0[0] == 0xffff) return 0;
  const int a1 = L0[2] - L0[0], ab1 = L0[4] - L0[0];  // A+1, (A+1)(B+1)
  if (a1 < 2 || ab1 < 2 * a1 || ab1 % a1) return 0;
  const int A = a1 - 1, B = ab1 / a1 - 1;
  if (A > 255 || B > 255) return 0;
  const int spl = (A * B + kLanes - 1) / kLanes;
  if (nm % ab1) return 0;
  const int C = nm / ab1 - 1;
  if (spl > 255 || C < 1 || C > 255) return 0;
  if (s1 - s0 != 4 * spl * ((C + 3) / 4)) return 0;
  const uint32_t lat = uint32_t(A) | uint32_t(B) << 8 | uint32_t(spl) << 16 | uint32_t(C) << 24;
  for (int s = s0; s < s1; ++s)
    for (int l = 0; l < kLanes; ++l) {
      const uint16_t *lc = &H.lconn[(size_t(s) * kLanes + l) * 8];
      int want[8];
      if (!corner_lattice(lat, s - s0, l, want)) {
        if (lc[0] != 0xffff) return 0;
        continue;
      }
      for (int a = 0; a < 8; ++a)
        if (lc[a] != want[a]) return 0;
    }
  return lat;
}

// The split accumulation of the block variants (bitwise reproducible): in a
// first pass every wave adds the lower corners (local a = 0..3) of its
// elements into the tile's LDS accumulator, in a second pass (after a
// barrier) the upper corners (a = 4..7), which it kept in registers.  Each
// pass is race-free, and its order fixed, when every node of the tile receives
// lower-corner additions from one wave at most and upper-corner additions
// from one wave at most, a wave has at most split_steps(dpn) steps (its registers),
// and no two lanes of a step share a node at one corner (checked separately).
bool split_ok(const HostTiles &H, int t, int nm, int dpn) {
  const int s0 = H.tile_step[t], s1 = H.tile_step[t + 1];
  if (s1 - s0 > 4 * split_steps(dpn)) return false;
  std::vector<int8_t> lo(nm, -1), hi(nm, -1);
  for (int s = s0; s < s1; ++s) {
    const int8_t w = int8_t((s - s0) & 3);
    for (int l = 0; l < kLanes; ++l) {
      const uint16_t *lc = &H.lconn[(size_t(s) * kLanes + l) * 8];
      if (lc[0] == 0xffff) continue;
      for (int a = 0; a < 8; ++a) {
        int8_t &o = a < 4 ? lo[lc[a]] : hi[lc[a]];
        if (o >= 0 && o != w) return false;
        o = w;
      }
    }
  }
  return true;
}

// Whether every tile is the kind's fixed lattice tile (FxTile<DPN>), and the
// built-in shape reproduces what the planner verified: the corner indices of
// every (position, lane), and every entry's word on lattice-addressed tiles.
template <int DPN>
bool fixed_tiles(const HostTiles &H) {
  using F = FxTile<DPN>;
  if (H.max_nodes != F::NODES || H.tile_lat.empty() ||
      !std::all_of(H.tile_lat.begin(), H.tile_lat.end(), [](uint32_t l) { return l == F::LAT; }))
    return false;
  for (int rel = 0; rel < F::STEPS; ++rel)
    for (int l = 0; l < kLanes; ++l) {
      int a[8], b[8];
      corner_fixed<DPN>(rel, l, a);
      if (!corner_lattice(F::LAT, rel, l, b) || !std::equal(a, a + 8, b)) return false;
    }
  for (size_t t = 0; t < H.tile_addr.size(); ++t)
    if (H.tile_addr[t])
      for (int i = 0; i < F::NODES; ++i)
        if (lattice_word_fixed<DPN>(i, H.tile_addr[t], H.tile_g0[t], H.sy, H.sz) !=
            lattice_word(i, F::LAT, H.tile_addr[t], H.tile_g0[t], H.sy, H.sz))
          return false;
  return true;
}

// Group elements into tiles and steps; record node lists and corner indices.
template <typename T>
// nloc: nodes per element (8 hexahedra, 4 tetrahedra; a tetrahedron's corner
// indices fill the first 4 of its 8 lane entries); cell_elems: elements per
// cell of the size estimate (6 for tetrahedra, as in a cube's split).
int plan_tiles(const std::vector<int32_t> &conn, const std::vector<T> &xyz,
               const std::vector<uint8_t> &mask, int64_t nn, int64_t ne, int patch_x,
               int patch_y, int layers, bool interleave, int dpn, HostTiles &H, int nloc = 8,
               double cell_elems = 1.0) {
  std::vector<double> cen(size_t(3) * ne);
  double lo[3] = {1e300, 1e300, 1e300};
  for (int64_t e = 0; e < ne; ++e)
    for (int r = 0; r < 3; ++r) {
      double c = 0;
      for (int a = 0; a < nloc; ++a) c += double(xyz[r * nn + conn[a * ne + e]]);
      c /= nloc;
      cen[3 * e + r] = c;
      lo[r] = std::min(lo[r], c);
    }
  // element size from the node bounding box
  double vol = 1.0;
  int live = 0;
  for (int r = 0; r < 3; ++r) {
    double nlo = 1e300, nhi = -1e300;
    for (int64_t n = 0; n < nn; ++n) {
      nlo = std::min(nlo, double(xyz[r * nn + n]));
      nhi = std::max(nhi, double(xyz[r * nn + n]));
    }
    if (nhi > nlo) { vol *= nhi - nlo; ++live; }
  }
  double h = live ? std::pow(vol * cell_elems / double(ne), 1.0 / live) : 1.0;
  if (!(h > 0)) h = 1.0;
  std::vector<int32_t> lz(ne), iy(ne), ix(ne);
  int64_t npx = 1, npy = 1;
  for (int64_t e = 0; e < ne; ++e) {
    ix[e] = int32_t(std::floor((cen[3 * e + 0] - lo[0]) / h + 0.5));
    iy[e] = int32_t(std::floor((cen[3 * e + 1] - lo[1]) / h + 0.5));
    lz[e] = int32_t(std::floor((cen[3 * e + 2] - lo[2]) / h + 0.5));
    npx = std::max<int64_t>(npx, ix[e] / patch_x + 1);
    npy = std::max<int64_t>(npy, iy[e] / patch_y + 1);
  }
  std::vector<uint64_t> tkey(ne);
  for (int64_t e = 0; e < ne; ++e) {
    const uint64_t px = ix[e] / patch_x, py = iy[e] / patch_y, cz = lz[e] / layers;
    tkey[e] = (cz * uint64_t(npy) + py) * uint64_t(npx) + px;
  }  std::vector<int32_t> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (tkey[a] != tkey[b]) return tkey[a] < tkey[b];
    if (lz[a] != lz[b]) return lz[a] < lz[b];
    if (iy[a] != iy[b]) return iy[a] < iy[b];
    return ix[a] < ix[b];
  });
  // tiles = runs of equal tile key; steps = runs of one layer, <= 64 elements
  std::vector<int64_t> tb;
  for (int64_t k = 0; k < ne; ++k)
    if (k == 0 || tkey[order[k]] != tkey[order[k - 1]]) tb.push_back(k);
  tb.push_back(ne);
  const int n_tiles = int(tb.size()) - 1;
  std::vector<int32_t> stamp(nn, -1), ntile(nn, 0);
  for (int t = 0; t < n_tiles; ++t)
    for (int64_t k = tb[t]; k < tb[t + 1]; ++k)
      for (int a = 0; a < nloc; ++a) {
        const int32_t g = conn[a * ne + order[k]];
        if (stamp[g] != t) { stamp[g] = t; ++ntile[g]; }
      }
  for (int64_t n = 0; n < nn; ++n)
    if (ntile[n] != 1 || (!mask.empty() && mask[n])) H.reset.push_back(int32_t(n));
  std::vector<int32_t> local(nn, -1), list;
  for (int t = 0; t < n_tiles; ++t) {
    list.clear();
    for (int64_t k = tb[t]; k < tb[t + 1]; ++k)
      for (int a = 0; a < nloc; ++a) list.push_back(conn[a * ne + order[k]]);
    std::sort(list.begin(), list.end());
    list.erase(std::unique(list.begin(), list.end()), list.end());
    if (list.size() >= 65535) return fail(Q1_EUNSUPPORTED, "tile with %zu nodes", list.size());
    H.max_nodes = std::max<int>(H.max_nodes, int(list.size()));
    for (size_t i = 0; i < list.size(); ++i) {
      const int32_t g = list[i];
      local[g] = int32_t(i);
      uint32_t v = uint32_t(g);
      if (ntile[g] > 1) v |= kSharedBit;
      if (!mask.empty() && mask[g]) v |= kFixedBit;
      H.nodes.push_back(v);
    }
    H.node_ptr.push_back(int32_t(H.nodes.size()));
    // steps: runs of one layer, at most 64 elements; (first, end, layer) with
    // the layer counted within the tile
    struct Run {
      int64_t j, je;
      int layer;
    };
    std::vector<Run> runs;
    for (int64_t j = tb[t], layer = -1; j < tb[t + 1];) {
      int64_t je = j;
      while (je < tb[t + 1] && lz[order[je]] == lz[order[j]] && je - j < kLanes) ++je;
      if (j == tb[t] || lz[order[j]] != lz[order[j - 1]]) ++layer;
      runs.push_back({j, je, int(layer)});
      for (int a = 0; a < nloc && !H.corner_collision; ++a) {
        std::vector<int32_t> cs;
        for (int64_t k = j; k < je; ++k) cs.push_back(conn[a * ne + order[k]]);
        std::sort(cs.begin(), cs.end());
        H.corner_collision = std::adjacent_find(cs.begin(), cs.end()) != cs.end();
      }
      j = je;
    }
    // interleaved layout (block variants): the steps of layer l belong to
    // wave l mod 4, and wave w's k-th step sits at position 4k + w (padded
    // with empty steps)
    std::vector<int> pos_run;  // run of each position, -1 = empty step
    if (interleave) {
      std::vector<int> per_wave[4];
      for (size_t r = 0; r < runs.size(); ++r) per_wave[runs[r].layer & 3].push_back(int(r));
      size_t kmax = 0;
      for (auto &v : per_wave) kmax = std::max(kmax, v.size());
      for (size_t k = 0; k < kmax; ++k)
        for (int w = 0; w < 4; ++w) pos_run.push_back(k < per_wave[w].size() ? per_wave[w][k] : -1);
    } else {
      for (size_t r = 0; r < runs.size(); ++r) pos_run.push_back(int(r));
    }
    for (int r : pos_run)
      for (int64_t k = 0; k < kLanes; ++k) {
        if (r >= 0 && runs[r].j + k < runs[r].je) {
          const int32_t e = order[runs[r].j + k];
          H.step_elem.push_back(e);
          for (int a = 0; a < 8; ++a)
            H.lconn.push_back(a < nloc ? uint16_t(local[conn[a * ne + e]]) : uint16_t(0));
        } else {
          H.step_elem.push_back(-1);
          for (int a = 0; a < 8; ++a) H.lconn.push_back(0xffff);
        }
      }
    H.tile_step.push_back(int32_t(H.step_elem.size() / kLanes));
    H.tile_lat.push_back(interleave ? lattice_of(H, t) : 0u);
    if (interleave && !split_ok(H, t, int(list.size()), dpn)) H.split = false;
    bool aff = nloc == 8;  // the kernel's own exact test, in the operator's precision
    for (int64_t k = tb[t]; k < tb[t + 1] && aff; ++k) {
      T X[3][8];
      for (int r = 0; r < 3; ++r) {
        for (int a = 0; a < 8; ++a) X[r][a] = xyz[r * nn + conn[a * ne + order[k]]];
        butterfly_fwd(X[r]);
      }
      aff = is_affine(X);
    }
    H.tile_affine.push_back(aff ? 1 : 0);
    for (int32_t g : list) local[g] = -1;
  }
  // halo slots.  Reset node j (a free node shared by c_j >= 2 tiles) receives the
  // contributions of the tiles touching it in tile order: the first in slot j,
  // the second in slot n_reset + j (so each tile's writes along a shared face are
  // contiguous), the others in the extra region 2 n_reset + [hptr[j], hptr[j+1]).
  // hnode[j] is the node id with bit 31 set on Dirichlet nodes (y = x) and
  // bit 30 set on free nodes that no element references (y = 0); neither
  // kind has slots written.
  const int64_t nr = int64_t(H.reset.size());
  std::vector<int64_t> hp(nr + 1, 0);
  H.hnode.assign(nr, 0);
  for (int64_t j = 0; j < nr; ++j) {
    const int32_t g = H.reset[j];
    const bool fixed = !mask.empty() && mask[g];
    hp[j + 1] = hp[j] + (fixed ? 0 : std::max(0, ntile[g] - 2));
    H.hnode[j] = fixed            ? int32_t(uint32_t(g) | 0x80000000u)
                 : ntile[g] == 0 ? int32_t(uint32_t(g) | 0x40000000u)
                                 : g;
    local[g] = int32_t(j);  // reset index (local[] is free again here)
  }
  if (2 * nr + hp[nr] >= (int64_t(1) << 31)) return fail(Q1_EUNSUPPORTED, "too many halo slots");
  H.hptr.assign(hp.begin(), hp.end());
  H.slot.assign(H.nodes.size(), -1);
  std::vector<int32_t> rank(nr, 0);
  for (size_t i = 0; i < H.nodes.size(); ++i) {
    const uint32_t v = H.nodes[i];
    if (!(v & kSharedBit) || (v & kFixedBit)) continue;
    const int32_t jj = local[v & kIdMask], r = rank[jj]++;
    H.slot[i] = r < 2 ? int32_t(r * nr + jj) : int32_t(2 * nr + H.hptr[jj] + (r - 2));
  }
  return Q1_OK;
}

// Lattice addressing (see lattice_word) for every lattice tile of the block
// variants without Dirichlet nodes whose words all match: the strides come
// from the first such tile, the face bits from one entry inside each face
// (faces without such an entry are taken as not shared), and every entry of
// the tile is then checked against the formula.
// Q1_TILE_ADDRESSING=0 keeps every tile on loaded node words (for comparison).
void plan_addressing(HostTiles &H) {
  const int nt = int(H.tile_lat.size());
  H.tile_addr.assign(nt, 0u);
  H.tile_g0.assign(nt, 0);
  if (const char *e = std::getenv("Q1_TILE_ADDRESSING"))
    if (e[0] == '0') return;
  for (int t = 0; t < nt; ++t) {
    const uint32_t lat = H.tile_lat[t];
    if (!lat) continue;
    const int A = int(lat & 0xff), B = int((lat >> 8) & 0xff), C = int(lat >> 24);
    const int a1 = A + 1, b1 = B + 1, n0 = H.node_ptr[t], nm = H.node_ptr[t + 1] - n0;
    const uint32_t *w = &H.nodes[n0];
    auto at = [&](int ix, int iy, int iz) { return w[ix + a1 * (iy + b1 * iz)]; };
    bool fixed = false;
    for (int i = 0; i < nm; ++i) fixed = fixed || (w[i] & kFixedBit);
    if (fixed) continue;
    const int64_t g0 = at(0, 0, 0) & kIdMask;
    if (!H.sy) {
      H.sy = int64_t(at(0, 1, 0) & kIdMask) - g0;
      H.sz = int64_t(at(0, 0, 1) & kIdMask) - g0;
      if (H.sy <= 0 || H.sz <= 0) return;
    }
    uint32_t f = 0;
    auto face = [&](bool ok, uint32_t word, uint32_t bit) {
      if (ok && (word & kSharedBit)) f |= bit;
    };
    face(B >= 2 && C >= 2, at(0, 1, 1), 1u);
    face(B >= 2 && C >= 2, at(A, 1, 1), 2u);
    face(A >= 2 && C >= 2, at(1, 0, 1), 4u);
    face(A >= 2 && C >= 2, at(1, B, 1), 8u);
    face(A >= 2 && B >= 2, at(1, 1, 0), 16u);
    face(A >= 2 && B >= 2, at(1, 1, C), 32u);
    const uint32_t addr = kAddrValid | f;
    bool ok = g0 + A + B * H.sy + C * H.sz <= int64_t(kIdMask);
    for (int i = 0; i < nm && ok; ++i) ok = lattice_word(i, lat, addr, g0, H.sy, H.sz) == w[i];
    if (ok) {
      H.tile_addr[t] = addr;
      H.tile_g0[t] = int32_t(g0);
    }
  }
}

// The mesh of an owner-computes operator: a box lattice in the generator's
// numbering (element e = ex + nx (ey + ny ez) with corner a at node
// (ex + a_x) + (nx+1)((ey + a_y) + (ny+1)(ez + a_z))), checked entry by entry,
// with nx, ny, nz multiples of the owned box, fewer than 2^29 nodes and
// (ny+1)(nz+1) below 2^24.
bool owner_box(const std::vector<int32_t> &conn, int64_t ne, int64_t nn, int &nx, int &ny,
               int &nz) {
  if (ne <= 0 || conn.size() != size_t(8) * ne || conn[0] != 0 || conn[ne] != 1) return false;
  const int64_t bx = int64_t(conn[2 * ne]) - 1;
  if (bx < 1 || int64_t(conn[4 * ne]) % (bx + 1)) return false;
  const int64_t by = int64_t(conn[4 * ne]) / (bx + 1) - 1;
  if (by < 1 || ne % (bx * by)) return false;
  const int64_t bz = ne / (bx * by);
  if ((bx + 1) * (by + 1) * (bz + 1) != nn) return false;
  if (nn * 8 >= (int64_t(1) << 32)) return false;  // the kernel's 32-bit byte offsets
  if ((by + 1) * (bz + 1) >= (int64_t(1) << 24) || bx + 1 >= (int64_t(1) << 24))
    return false;  // and its 24-bit products
  if (bx % OwnTile::OX || by % OwnTile::OY || bz % OwnTile::OZ) return false;
  const int64_t sy = bx + 1, sz = (bx + 1) * (by + 1);
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t ex = e % bx, ey = (e / bx) % by, ez = e / (bx * by);
    const int64_t b = ex + sy * ey + sz * ez;
    for (int a = 0; a < 8; ++a)
      if (conn[size_t(a) * ne + e] != b + (a & 1) + sy * ((a >> 1) & 1) + sz * (a >> 2))
        return false;
  }
  nx = int(bx);
  ny = int(by);
  nz = int(bz);
  return true;
}

// The tetrahedra of an owner-computes operator: the Kuhn split of a box lattice
// (tetrahedron t of cell e is element 6e + t, its corners the cell corners kKuhn[t]
// of the lattice cell e = ex + nx (ey + ny ez)), checked entry by entry, with the
// limits of owner_box.
bool owner_kuhn(const std::vector<int32_t> &conn, int64_t ne, int64_t nn, int &nx, int &ny,
                int &nz) {
  static constexpr int kt[6][4] = {{0, 1, 3, 7}, {0, 5, 1, 7}, {0, 3, 2, 7},
                                   {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}};
  if (ne <= 0 || ne % 6 || conn.size() != size_t(4) * ne) return false;
  const int64_t nc = ne / 6;
  // cell 0's corners 1, 3 and 7 are tetrahedron 0's vertices 1, 2 and 3
  if (conn[0] != 0 || conn[ne] != 1) return false;
  const int64_t bx = int64_t(conn[2 * ne]) - 2;  // corner 3 = 1 + (nx + 1)
  if (bx < 1) return false;
  const int64_t c7 = int64_t(conn[3 * ne]) - 1 - (bx + 1);  // (nx + 1)(ny + 1)
  if (c7 <= 0 || c7 % (bx + 1)) return false;
  const int64_t by = c7 / (bx + 1) - 1;
  if (by < 1 || nc % (bx * by)) return false;
  const int64_t bz = nc / (bx * by);
  if ((bx + 1) * (by + 1) * (bz + 1) != nn) return false;
  if (nn * 8 >= (int64_t(1) << 32) || ne * 8 >= (int64_t(1) << 32)) return false;
  if ((by + 1) * (bz + 1) >= (int64_t(1) << 24) || bx + 1 >= (int64_t(1) << 24)) return false;
  if (bx % OwnTile::OX || by % OwnTile::OY || bz % OwnTile::OZ) return false;
  const int64_t sy = bx + 1, sz = (bx + 1) * (by + 1);
  for (int64_t e = 0; e < nc; ++e) {
    const int64_t ex = e % bx, ey = (e / bx) % by, ez = e / (bx * by);
    const int64_t b = ex + sy * ey + sz * ez;
    for (int t = 0; t < 6; ++t)
      for (int q = 0; q < 4; ++q) {
        const int a = kt[t][q];
        if (conn[size_t(q) * ne + 6 * e + t] != b + (a & 1) + sy * ((a >> 1) & 1) + sz * (a >> 2))
          return false;
      }
  }
  nx = int(bx);
  ny = int(by);
  nz = int(bz);
  return true;
}

// Largest mesh of general hexahedra that takes the owner-computes tiles: measured
// on jittered n^3 Laplace FP64 (owner / halo-slot tiles, us per apply streaming):
// 32^3 9.6 / 11.4, 48^3 10.2 / 11.9, 64^3 17.0 / 16.7, 128^3 99.8 / 80.6; the 16^3
// Jacobi-PCG to 1e-8 2.23 / 2.40 ms.
constexpr int64_t kOwnerGeneralElems = 128 * 1024;

int64_t own_tiles(const TileMap &tm) {
  return int64_t(tm.own_nx / OwnTile::OX) * (tm.own_ny / OwnTile::OY) * (tm.own_nz / OwnTile::OZ);
}

template <typename T>
int build_tiles_t(Op &op, hipStream_t s, int patch_x, int patch_y, int layers) {
  const int64_t ne = op.n_elems, nn = op.n_nodes;
  const int ncoef = phys_ncoef(op.physics);
  TileMap &tm = op.tiles;
  Q1_CHECK(nn <= int64_t(kIdMask), Q1_EUNSUPPORTED, "LDS-tile variant supports < 2^30 nodes");
  Q1_HIP(hipStreamSynchronize(s));
  const int nloc = op.nloc();
  std::vector<int32_t> conn(size_t(nloc) * ne);
  std::vector<T> xyz(size_t(3) * nn), coef(size_t(ncoef) * ne);
  std::vector<uint8_t> mask;
  Q1_HIP(hipMemcpy(conn.data(), op.conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(xyz.data(), op.xyz, xyz.size() * sizeof(T), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(coef.data(), op.coef, coef.size() * sizeof(T), hipMemcpyDeviceToHost));
  if (op.mask) {
    mask.resize(nn);
    Q1_HIP(hipMemcpy(mask.data(), op.mask, size_t(nn), hipMemcpyDeviceToHost));
  }
  for (size_t i = 0; i < conn.size(); ++i)
    Q1_CHECK(conn[i] >= 0 && conn[i] < nn, Q1_EINVAL, "connectivity entry %zu out of range", i);
  HostTiles H;
  const bool block = op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA;
  const bool hex = op.elem == Q1_HEX8;
  int rc = plan_tiles<T>(conn, xyz, mask, nn, ne, patch_x, patch_y, layers, block && hex,
                         op.dpn(), H, nloc, hex ? 1.0 : 6.0);
  if (rc) return rc;
  // lattice addressing for the scalar kind only: measured on 128^3 Laplace FP64
  // (applies streaming from HBM) 46.8 against 44.9 GDOF/s, while the 3-DOF kinds
  // (fewer nodes per element, more arithmetic per node) ran 3-5% slower with it;
  // in their fixed-shape instance it gains 2-3% streaming from HBM but nothing
  // (FP64) or -5% (FP32) on MALL-resident data, where a solver's applies run
  if (block && hex && op.dpn() == 1) plan_addressing(H);
  else {
    H.tile_addr.assign(H.tile_lat.size(), 0u);
    H.tile_g0.assign(H.tile_lat.size(), 0);
  }
  tm.sy = H.sy;
  tm.sz = H.sz;
  const int64_t n_slots = int64_t(H.step_elem.size());
  std::vector<T> coef_t(size_t(ncoef) * n_slots, T(0));
  for (int64_t k = 0; k < n_slots; ++k)
    if (H.step_elem[k] >= 0)
      for (int c = 0; c < ncoef; ++c) coef_t[c * n_slots + k] = coef[c * ne + H.step_elem[k]];
  tm.n_tiles = int(H.node_ptr.size()) - 1;
  tm.n_steps = n_slots / kLanes;
  tm.max_nodes = H.max_nodes;
  tm.n_reset = int64_t(H.reset.size());
  tm.n_entries = int64_t(H.nodes.size());
  tm.lds_atomic = H.corner_collision;
  tm.split = block && hex && H.split && !H.corner_collision;
  tm.all_affine = std::all_of(H.tile_affine.begin(), H.tile_affine.end(),
                              [](uint8_t a) { return a != 0; });
  tm.fixed = op.dpn() == 1 ? fixed_tiles<1>(H) : fixed_tiles<3>(H);
  tm.fixed = tm.fixed && tm.split && op.variant == Q1_V_BLOCK && op.elem == Q1_HEX8;
  if (const char *e = std::getenv("Q1_FIXED_TILE"))  // "0": the general-shape instances
    if (e[0] == '0') tm.fixed = false;
  // owner-computes tiles for the scalar kind on a box lattice ("Q1_OWNER_TILE=0": the
  // halo-slot tiles); the diagonal keeps the split tiles.  Meshes of general hexahedra
  // take them only when small (at most kOwnerGeneralElems elements), where the apply is
  // bound by the latency of its kernels rather than by the element work that the
  // owner tiles repeat on the shell ("Q1_OWNER_GENERAL=0" or "1" overrides).
  // Tetrahedra of a lattice's Kuhn split take them too, each cell's six as one element
  // (scalar kind; bitwise reproducible, unlike their block tiles).
  tm.own_nx = tm.own_ny = tm.own_nz = 0;
  tm.own_elem = tm.all_affine ? 0 : 1;
  bool own_ok = tm.all_affine || ne <= kOwnerGeneralElems;
  if (const char *e = std::getenv("Q1_OWNER_GENERAL")) own_ok = tm.all_affine || e[0] == '1';
  const char *own_env = std::getenv("Q1_OWNER_TILE");
  const bool own_on = op.variant == Q1_V_BLOCK && op.physics == Q1_LAPLACE &&
                      !(own_env && own_env[0] == '0');
  if (own_on && hex && own_ok && tm.split)
    owner_box(conn, ne, nn, tm.own_nx, tm.own_ny, tm.own_nz);
  if (own_on && op.elem == Q1_TET4 && owner_kuhn(conn, ne, nn, tm.own_nx, tm.own_ny, tm.own_nz))
    tm.own_elem = 2;
  auto up = [&](auto **dst, const auto &v) -> int {
    using E = typename std::remove_reference<decltype(v)>::type::value_type;
    const size_t b = std::max<size_t>(1, v.size()) * sizeof(E);
    Q1_HIP(hipMalloc(reinterpret_cast<void **>(dst), b));
    if (!v.empty()) Q1_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice));
    tm.bytes += b;
    return Q1_OK;
  };
  T *coef_dev = nullptr;
  if ((rc = up(&tm.node_ptr, H.node_ptr)) || (rc = up(&tm.nodes, H.nodes)) ||
      (rc = up(&tm.tile_step, H.tile_step)) || (rc = up(&tm.lconn, H.lconn)) ||
      (rc = up(&tm.reset, H.reset)) || (rc = up(&coef_dev, coef_t)) ||
      (rc = up(&tm.tile_affine, H.tile_affine)) || (rc = up(&tm.tile_lat, H.tile_lat)) ||
      (rc = up(&tm.tile_addr, H.tile_addr)) || (rc = up(&tm.tile_g0, H.tile_g0)))
    return rc;
  tm.coef_t = coef_dev;
  if (op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA) {
    if ((rc = up(&tm.slot, H.slot)) || (rc = up(&tm.hptr, H.hptr)) ||
        (rc = up(&tm.hnode, H.hnode)))
      return rc;
    tm.n_halo = 2 * int64_t(H.reset.size()) + H.hptr.back();
    const size_t hb = std::max<int64_t>(1, tm.n_halo) * op.dpn() * sizeof(T);
    Q1_HIP(hipMalloc(&tm.halo, hb));
    tm.bytes += hb;
  }
  if (op.variant == Q1_V_PA) {
    // quadrature data of every element slot, computed once on the device
    int32_t *d_elem = nullptr;
    Q1_HIP(hipMalloc(&d_elem, size_t(n_slots) * sizeof(int32_t)));
    Q1_HIP(hipMemcpy(d_elem, H.step_elem.data(), size_t(n_slots) * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    const int nq = op.physics == Q1_ELASTICITY ? 9 : 6;
    const size_t qb = size_t(8 * nq) * n_slots * sizeof(T);
    hipError_t e = hipMalloc(&tm.qdata, qb);
    if (e != hipSuccess) {
      (void)hipFree(d_elem);
      return fail(Q1_ENOMEM, "partial assembly: %zu B of quadrature data", qb);
    }
    tm.bytes += qb;
    hipLaunchKernelGGL((nq == 9 ? k_pa_setup<T, 9> : k_pa_setup<T, 6>),
                       dim3(unsigned((n_slots + 255) / 256)), dim3(256), 0, s, n_slots, d_elem,
                       ne, nn, op.conn, static_cast<const T *>(op.xyz),
                       static_cast<const T *>(op.coef), static_cast<T *>(tm.qdata));
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_elem);
    if (e != hipSuccess) return fail(Q1_EHIP, "partial assembly set-up: %s", hipGetErrorString(e));
  }
  return Q1_OK;
}

// LDS of the block-staged variant: node records (coordinates unless partial
// assembly, input), then the accumulator copies (one shared copy for FP64,
// one per wave for FP32)
size_t block_lds_bytes(const Op &op) {
  const size_t rb = op.dtype == Q1_F64 ? 8 : 4;
  if (op.elem == Q1_TET4)  // records, then the FP64 accumulator
    return tet_acc_offset(op.tiles.max_nodes, rb * (3 + op.dpn())) +
           size_t(op.tiles.max_nodes) * 8 * op.dpn();
  const size_t nacc = op.tiles.split || op.dtype == Q1_F64 || op.elem == Q1_TET4 ? 1 : 4;
  const size_t ncoord = op.variant == Q1_V_PA ? 0 : 3;
  return size_t(op.tiles.max_nodes) * rb * size_t(ncoord + op.dpn() + nacc * op.dpn());
}

// Halo-sum workgroups of an operator's block apply.
int64_t halo_blocks(const TileMap &tm) {
  return (tm.n_reset + 256 * kHaloNpt - 1) / (256 * kHaloNpt);
}

// dot: optional partials of x.y (block variants of hexahedra): on owner-computes
// tiles, one per tile at dot[0..); else with shared or Dirichlet nodes,
// halo_blocks(tm) partials at dot[0..) that include the tile partials at
// dot[halo_blocks(tm)..); without them, the tile partials at dot[0..).
template <typename T, int PH>
int apply_tile_t(Op &op, const void *xv, void *yv, hipStream_t s, const int *stop,
                 double *dot = nullptr) {
  constexpr int DPN = phys_dpn(PH);
  const TileMap &tm = op.tiles;
  const T *x = static_cast<const T *>(xv);
  T *y = static_cast<T *>(yv);
  const bool pa = op.variant == Q1_V_PA;
  const bool block = op.variant == Q1_V_BLOCK || pa;
  if (tm.n_reset > 0 && !block)
    hipLaunchKernelGGL((k_reset_nodes<T, DPN>), dim3(int((tm.n_reset + 255) / 256)), dim3(256), 0,
                       s, tm.n_reset, tm.reset, op.mask, x, y, stop);
  if (block && tm.own_nx > 0) {
    if constexpr (PH == 1) {
      auto pick = [&](auto ek) {
        constexpr int EK = decltype(ek)::value;
        return op.mask ? k_apply_owner<T, true, EK> : k_apply_owner<T, false, EK>;
      };
      auto kern = tm.own_elem == 2   ? pick(std::integral_constant<int, kOwnKuhn>{})
                  : tm.own_elem == 1 ? pick(std::integral_constant<int, kOwnGen>{})
                                     : pick(std::integral_constant<int, kOwnPar>{});
      hipLaunchKernelGGL(kern, dim3(unsigned(own_tiles(tm))), dim3(256), 0, s, tm.own_nx,
                         tm.own_ny, tm.own_nz, static_cast<const T *>(op.xyz),
                         static_cast<const T *>(op.coef), op.mask, x, y, stop, dot);
      Q1_HIP(hipGetLastError());
      return Q1_OK;
    }
  }
  const size_t lds = block ? block_lds_bytes(op) : size_t(tm.max_nodes) * (DPN * sizeof(T) + sizeof(uint32_t));
  if (block && op.elem == Q1_TET4) {
    if constexpr (PH != 2) {
      const size_t tl = block_lds_bytes(op);
      hipLaunchKernelGGL((k_apply_block_tet<T, PH>), dim3(tm.n_tiles), dim3(256), tl, s,
                         tm.max_nodes, op.n_nodes, tm.node_ptr, tm.nodes, tm.tile_step,
                         reinterpret_cast<const uint4 *>(tm.lconn),
                         static_cast<const T *>(tm.coef_t), tm.n_steps * kLanes,
                         static_cast<const T *>(op.xyz), x, y, stop, tm.slot,
                         static_cast<T *>(tm.halo));
      if (tm.n_reset > 0)
        hipLaunchKernelGGL((k_halo_sum<T, DPN>), dim3(int(halo_blocks(tm))), dim3(256), 0, s,
                           tm.n_reset, tm.hnode, tm.hptr, x, static_cast<const T *>(tm.halo), y,
                           stop, static_cast<double *>(nullptr),
                           static_cast<const double *>(nullptr), int64_t(0));
      Q1_HIP(hipGetLastError());
      return Q1_OK;
    }
    return fail(Q1_EUNSUPPORTED, "tetrahedra: scalar Laplace and elasticity");
  }
  if (block) {
    // fallback accumulation when some tile does not admit the split one
    constexpr int FB = std::is_same<T, double>::value ? kAccShared : kAccCopies;
    const bool allpar = tm.all_affine && !pa;
    auto pick = [&](auto pa_c, auto allpar_c) {
      constexpr bool P = decltype(pa_c)::value, AP = decltype(allpar_c)::value;
      return tm.split        ? k_apply_block<T, PH, false, kAccSplit, P, AP>
             : tm.lds_atomic ? k_apply_block<T, PH, true, FB, P, AP>
                             : k_apply_block<T, PH, false, FB, P, AP>;
    };
    using tt = std::true_type;
    using ff = std::false_type;
    auto kb = pa ? pick(tt{}, ff{}) : allpar ? pick(ff{}, tt{}) : pick(ff{}, ff{});
    if (tm.fixed)
      kb = allpar ? k_apply_block<T, PH, false, kAccSplit, false, true, true>
                  : k_apply_block<T, PH, false, kAccSplit, false, false, true>;
    hipLaunchKernelGGL(kb, dim3(tm.n_tiles), dim3(256), lds, s, tm.max_nodes, op.n_nodes,
                       tm.node_ptr, tm.nodes, tm.tile_step,
                       reinterpret_cast<const uint4 *>(tm.lconn),
                       static_cast<const T *>(tm.coef_t), tm.n_steps * kLanes,
                       static_cast<const T *>(op.xyz), x, y, stop, tm.tile_affine, tm.slot,
                       static_cast<T *>(tm.halo), static_cast<const T *>(tm.qdata),
                       tm.tile_lat, tm.tile_addr, tm.tile_g0, tm.sy, tm.sz,
                       dot ? dot + (tm.n_reset > 0 ? halo_blocks(tm) : 0) : nullptr);
    if (tm.n_reset > 0)
      hipLaunchKernelGGL((k_halo_sum<T, DPN>), dim3(int(halo_blocks(tm))), dim3(256), 0, s,
                         tm.n_reset, tm.hnode, tm.hptr, x, static_cast<const T *>(tm.halo), y,
                         stop, dot, dot ? dot + halo_blocks(tm) : nullptr, int64_t(tm.n_tiles));
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  }
  auto kern = tm.lds_atomic ? k_apply_tile<T, PH, true> : k_apply_tile<T, PH, false>;
  hipLaunchKernelGGL(kern, dim3(tm.n_tiles), dim3(kLanes), lds, s, tm.max_nodes,
                     op.n_nodes,
                     tm.node_ptr, tm.nodes, tm.tile_step,
                     reinterpret_cast<const uint4 *>(tm.lconn),
                     static_cast<const T *>(tm.coef_t), tm.n_steps * kLanes,
                     static_cast<const T *>(op.xyz), x, y, stop);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace

// Tile shape in elements: PATCH_X x PATCH_Y per step (one wavefront), LAYERS steps.
// Wide-in-x patches keep each wave-wide gather on few cache lines (measured:
// 32x2x4 beats 8x8x8 by 17% in FP64 and 32% in FP32 on a 128^3 grid).
static int tile_layers(const Op &op) { return op.dpn() == 1 ? 4 : 2; }
static int tile_patch_x(const Op &) { return 32; }

// Block-staged tiles: 16 x 8 x 4 elements for scalar problems (two wavefront
// steps per layer; measured on 128^3 with parallelepiped tiles: FP64 41.0 us
// and FP32 30.6 us, against 43.2 / 30.2 for 32x4x4, 41.5 / 32.7 for 8x8x8 and
// 45.2 / 34.3 for 16x16x2) and 16 x 4 x 4 for the 3-DOF kinds (96^3
// elasticity FP64 48.4 us, against 49.5 for 16x8x2 and 49.8 for 8x8x4);
// Q1_BLOCK_SHAPE="px,py,layers" overrides the shape.
static void block_shape(const Op &op, int &px, int &py, int &layers) {
  px = 16;
  py = op.dpn() == 1 ? 8 : 4;
  layers = 4;
  if (const char *e = std::getenv("Q1_BLOCK_SHAPE")) {
    int a = 0, b = 0, c = 0;
    if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0) {
      px = a;
      py = b;
      layers = c;
    }
  }
}

int build_tiles(Op &op, hipStream_t s) {
  Q1_CHECK(op.n_elems > 0, Q1_EUNSUPPORTED, "LDS-tile variant needs at least one element");
  int px, py, layers;
  if (op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA) {
    block_shape(op, px, py, layers);
  } else {
    layers = tile_layers(op);
    px = tile_patch_x(op);
    py = kLanes / px;
  }
  int rc = op.dtype == Q1_F64 ? build_tiles_t<double>(op, s, px, py, layers)
                              : build_tiles_t<float>(op, s, px, py, layers);
  if (rc) return rc;
  const size_t lds = op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA
                         ? block_lds_bytes(op)
                         : size_t(op.tiles.max_nodes) * (op.dpn() * (op.dtype == Q1_F64 ? 8 : 4) + 4);
  Q1_CHECK(lds <= 64 * 1024, Q1_EUNSUPPORTED, "tile needs %zu B of LDS", lds);
  return Q1_OK;
}

// The diagonal through the tiles (block variants whose tiles admit the split
// accumulation; Q1_EUNSUPPORTED otherwise).
int launch_diag_tile(Op &op, void *dv, hipStream_t s) {
  const TileMap &tm = op.tiles;
  const bool block = op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA;
  Q1_CHECK(block && tm.split, Q1_EUNSUPPORTED, "tile diagonal needs the split accumulation");
  return dispatch_phys(op, [&](auto t, auto ph) -> int {
    using T = decltype(t);
    constexpr int PH = decltype(ph)::value;
    constexpr int DPN = phys_dpn(PH);
    T *d = static_cast<T *>(dv);
    const size_t lds = size_t(tm.max_nodes) * sizeof(T) * (3 + DPN);
    hipLaunchKernelGGL((k_diag_block<T, PH>), dim3(tm.n_tiles), dim3(256), lds, s, tm.max_nodes,
                       op.n_nodes, tm.node_ptr, tm.nodes, tm.tile_step,
                       reinterpret_cast<const uint4 *>(tm.lconn),
                       static_cast<const T *>(tm.coef_t), tm.n_steps * kLanes,
                       static_cast<const T *>(op.xyz), d, tm.slot, static_cast<T *>(tm.halo),
                       tm.tile_lat);
    if (tm.n_reset > 0)
      hipLaunchKernelGGL((k_halo_sum<T, DPN>), dim3(int(halo_blocks(tm))), dim3(256), 0, s,
                         tm.n_reset, tm.hnode, tm.hptr, static_cast<const T *>(nullptr),
                         static_cast<const T *>(tm.halo), d, static_cast<const int *>(nullptr),
                         static_cast<double *>(nullptr), static_cast<const double *>(nullptr),
                         int64_t(0));
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  });
}

int launch_apply_tile(Op &op, const void *x, void *y, hipStream_t s, const int *stop) {
  return dispatch_phys(op, [&](auto t, auto ph) {
    return apply_tile_t<decltype(t), decltype(ph)::value>(op, x, y, s, stop);
  });
}

int64_t apply_dot_parts(const Op &op, int64_t *n_final) {
  if (op.variant == Q1_V_BLOCK && op.tiles.own_nx > 0) {  // one partial per owner tile
    if (n_final) *n_final = own_tiles(op.tiles);
    return own_tiles(op.tiles);
  }
  const bool block = (op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA) && op.elem == Q1_HEX8;
  if (!block || op.tiles.n_tiles == 0) return 0;
  const int64_t h = op.tiles.n_reset > 0 ? halo_blocks(op.tiles) : 0;
  if (n_final) *n_final = h > 0 ? h : op.tiles.n_tiles;
  return h + op.tiles.n_tiles;
}

int launch_apply_dot(Op &op, const void *x, void *y, hipStream_t s, const int *stop,
                     double *parts) {
  Q1_CHECK(apply_dot_parts(op, nullptr) > 0, Q1_EUNSUPPORTED,
           "apply with partial dot products: block variants of hexahedra only");
  return dispatch_phys(op, [&](auto t, auto ph) {
    return apply_tile_t<decltype(t), decltype(ph)::value>(op, x, y, s, stop, parts);
  });
}

int launch_diag_owner(Op &op, void *dv, hipStream_t s) {
  const TileMap &tm = op.tiles;
  Q1_CHECK(tm.own_nx > 0 && tm.own_elem == 2 && op.physics == Q1_LAPLACE, Q1_EUNSUPPORTED,
           "owner-computes diagonal: the tetrahedra of a Kuhn-split lattice");
  auto run = [&](auto t) -> int {
    using T = decltype(t);
    auto kern = op.mask ? k_apply_owner<T, true, kOwnKuhnDiag>
                        : k_apply_owner<T, false, kOwnKuhnDiag>;
    hipLaunchKernelGGL(kern, dim3(unsigned(own_tiles(tm))), dim3(256), 0, s, tm.own_nx,
                       tm.own_ny, tm.own_nz, static_cast<const T *>(op.xyz),
                       static_cast<const T *>(op.coef), op.mask, static_cast<const T *>(nullptr),
                       static_cast<T *>(dv), static_cast<const int *>(nullptr),
                       static_cast<double *>(nullptr));
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  };
  return op.dtype == Q1_F64 ? run(double{}) : run(float{});
}

void free_tiles(Op &op) {
  TileMap &t = op.tiles;
  void *ptrs[] = {t.node_ptr, t.nodes, t.tile_step, t.lconn, t.reset,
                  t.coef_t,   t.tile_affine, t.slot, t.hptr, t.halo, t.qdata, t.tile_lat,
                  t.tile_addr, t.tile_g0,
                  t.hnode};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  t = TileMap{};
}

}  // namespace q1
