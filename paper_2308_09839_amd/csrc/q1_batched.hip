// Batched persistent Jacobi-PCG: many independent scalar-Laplace problems,
// each with up to four right-hand sides, solved by ONE cooperative launch.
//
// Each problem p owns a contiguous range of single-wavefront workgroups
// (sized in proportion to its expected work).  The waves of a problem meet at
// a two-level barrier of global counters; problems never wait for each
// other.  Vectors are stored interleaved [node][R] so that one gather of a
// node serves all R right-hand sides.  Per iteration (the CG operations of
// Table 4, regrouped):
//   P1  over the operator's LDS tiles (as in q1_tile.hip): the direction
//       update p = D^{-1} r + beta p_old on each tile's nodes into LDS (the
//       node's writer entry also stores it, and q = p on Dirichlet nodes,
//       their rows of A p), then q = A p from the staged p, with the partials
//       of p^T A p (element energies sum_e p_e^T A_e p_e and p^2 on Dirichlet
//       nodes).  p alternates between two buffers, so reading p_old and
//       writing p needs no barrier in between.
//   P2  alpha = rho / p^T A p; x += alpha p; r -= alpha q; q = 0 once read;
//       partials of rho' = r^T D^{-1} r and r^T r; then the convergence test
//       and beta = rho'/rho for the next P1
// with one barrier after each phase.  In the mixed-precision form the search
// directions p, q and the applies of P1 are FP32 (the FP32 operator's
// coordinates and coefficients), while x, r and every dot product stay FP64;
// whenever the recurrence residual has fallen by delta since the last refresh
// (and before convergence is declared) the true residual r = b - A64 x is
// recomputed with an FP64 apply of x inside the same launch (two more
// barriers), and the recurrences continue from it with p kept.
// The barrier itself sums the partials in a fixed order (per sub-group of
// waves, then over sub-groups) and every wave reads the same totals, so all
// waves of a problem hold bit-identical scalars and take the same branch.  Each
// barrier wait has a spin limit: past it the kernel records an error and every
// wave returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <new>
#include <type_traits>
#include <vector>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {

namespace {

constexpr int kW = 64;            // one wavefront per workgroup
constexpr int kRmax = 4;
constexpr uint32_t kSharedBitB = 0x80000000u;
constexpr uint32_t kFixedBitB = 0x40000000u;
constexpr uint32_t kIdMaskB = 0x3fffffffu;
// In the per-problem copy of the tile node lists the search-direction phase
// reads, bit 29 marks the one entry (in the first tile holding the node) that
// writes the node's new direction; ids are then below 2^29.
constexpr uint32_t kOwnBitB = 0x20000000u;
constexpr uint32_t kIdMaskOwnB = 0x1fffffffu;
constexpr unsigned kSpinLimit = 1u << 26;  // barrier polls before giving up
// Nodes per lane per round in the vector phases: every load of a round is
// issued before its stores (gfx9 waits for loads and stores on one counter, so
// a round costs one load and one store latency whatever kU is).
constexpr int kU = 4;
constexpr int kStage = 8;  // node ids per lane per staging round of a tile

// partial-sum slots per problem: [slot][rhs][nwg]
enum { kEnergy = 0, kMp2 = 1, kRho = 2, kRR = 3, kBB = 4, kRho0 = 5, kSlots = 6 };

struct BProb {
  int64_t nn;
  int n_tiles, max_nodes;
  const int32_t *node_ptr;
  const uint32_t *nodes;
  const uint32_t *onodes;     // the node lists with the writer bit
  const int32_t *tile_step;
  const uint4 *lconn;
  const double *coef_t;
  const double *xyz;
  const int32_t *reset;
  int64_t n_reset;
  const uint8_t *mask;
  double *b, *x, *r, *q;      // [nn][R]
  double *p[2];               // [nn][R]: directions of odd and even iterations
  const double *w;            // inverse diagonal [nn]
  // mixed precision: FP32 geometry, coefficients and directions; FP64 refresh output
  const float *xyz32, *coef32;
  float *p32[2], *q32;        // [nn][R]
  double *t;                  // [nn][R]
  double *part;               // [kSlots][R][nwg]
  double *tot;                // [kSub + 1][2R] sub-group and problem totals
  unsigned *bar;              // [kBarWords]: two-level barrier counters, generation
  int wg0, nwg;
  int *iters, *status, *nref; // [R]
  double *rr, *bb;            // [R]
};

// The problem records are read from memory, so the compiler cannot tell that
// their pointers address global memory and would access them with flat
// instructions, which also count on the LDS counter: every LDS wait of the
// apply (node ids, accumulator atomics) would then wait for all outstanding
// memory loads.  The kernel therefore reads each record through a twin whose
// pointers are typed as global-address-space pointers; converting those to
// ordinary pointers keeps the fact that they address global memory, and the
// compiler emits global instructions for every access made through them.
#define Q1_GLB __attribute__((address_space(1)))
struct BProbG {
  int64_t nn;
  int n_tiles, max_nodes;
  const Q1_GLB int32_t *node_ptr;
  const Q1_GLB uint32_t *nodes;
  const Q1_GLB uint32_t *onodes;
  const Q1_GLB int32_t *tile_step;
  const Q1_GLB uint4 *lconn;
  const Q1_GLB double *coef_t;
  const Q1_GLB double *xyz;
  const Q1_GLB int32_t *reset;
  int64_t n_reset;
  const Q1_GLB uint8_t *mask;
  Q1_GLB double *b, *x, *r, *q;
  Q1_GLB double *p[2];
  const Q1_GLB double *w;
  const Q1_GLB float *xyz32, *coef32;
  Q1_GLB float *p32[2], *q32;
  Q1_GLB double *t;
  Q1_GLB double *part;
  Q1_GLB double *tot;
  Q1_GLB unsigned *bar;
  int wg0, nwg;
  Q1_GLB int *iters, *status, *nref;
  Q1_GLB double *rr, *bb;
};
static_assert(sizeof(BProbG) == sizeof(BProb) && offsetof(BProbG, bb) == offsetof(BProb, bb) &&
                  offsetof(BProbG, n_reset) == offsetof(BProb, n_reset) &&
                  offsetof(BProbG, wg0) == offsetof(BProb, wg0),
              "BProbG must mirror BProb");

__device__ __forceinline__ BProb load_problem(const BProb *src) {
  BProbG G;
  __builtin_memcpy(&G, src, sizeof(G));
  BProb P;
  P.nn = G.nn;
  P.n_tiles = G.n_tiles;
  P.max_nodes = G.max_nodes;
  P.node_ptr = (const int32_t *)G.node_ptr;
  P.nodes = (const uint32_t *)G.nodes;
  P.onodes = (const uint32_t *)G.onodes;
  P.tile_step = (const int32_t *)G.tile_step;
  P.lconn = (const uint4 *)G.lconn;
  P.coef_t = (const double *)G.coef_t;
  P.xyz = (const double *)G.xyz;
  P.reset = (const int32_t *)G.reset;
  P.n_reset = G.n_reset;
  P.mask = (const uint8_t *)G.mask;
  P.b = (double *)G.b;
  P.x = (double *)G.x;
  P.r = (double *)G.r;
  P.p[0] = (double *)G.p[0];
  P.p[1] = (double *)G.p[1];
  P.q = (double *)G.q;
  P.w = (const double *)G.w;
  P.xyz32 = (const float *)G.xyz32;
  P.coef32 = (const float *)G.coef32;
  P.p32[0] = (float *)G.p32[0];
  P.p32[1] = (float *)G.p32[1];
  P.q32 = (float *)G.q32;
  P.t = (double *)G.t;
  P.part = (double *)G.part;
  P.tot = (double *)G.tot;
  P.bar = (unsigned *)G.bar;
  P.wg0 = G.wg0;
  P.nwg = G.nwg;
  P.iters = (int *)G.iters;
  P.status = (int *)G.status;
  P.nref = (int *)G.nref;
  P.rr = (double *)G.rr;
  P.bb = (double *)G.bb;
  return P;
}
#undef Q1_GLB

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Barrier of the nwg waves of one problem, optionally fused with the sum of two
// partial-sum slots (sa, sb; sa < 0 for none) over the waves; false when the
// spin limit was hit.  Two levels, so neither arrivals nor polling meet on one
// address and no wave reads all nwg partials: wave me belongs to sub-group
// me % kSub, whose counter and generation copy share a cache line of their
// own.  The last arrival of a sub-group sums its members' partials (in member
// order) into the sub-group's totals, resets the counter and arrives at the top
// counter; the last top arrival sums the sub-group totals (in sub-group order),
// writes the problem's totals, resets the top counter and writes the new
// generation into every copy, which the waves poll.  Every wave then reads the
// same totals, so all waves hold bit-identical scalars and take the same branch.
// Ordering: the counters, generation copies and polls are relaxed atomics,
// ordered by explicit fences (a release fence before each arrival, an acquire
// fence after it is known to be complete), so each wave writes back and
// invalidates its L2 once per barrier instead of once per poll.
// bar: [0] top count, [32 (1 + k)] sub-counter k, [32 (1 + k) + 1] its generation.
// tot: [kSub][2R] sub-group totals, then [2R] problem totals.
constexpr unsigned kSub = 8;
constexpr unsigned kBarWords = 32 * (kSub + 1);
template <int R>
__device__ __forceinline__ bool problem_sync(const BProb &P, unsigned me, unsigned nwg,
                                             int *error, int sa, int sb, double (&a)[R],
                                             double (&b)[R]) {
  const int lane = threadIdx.x;
  unsigned *bar = P.bar;
  double *sub_tot = P.tot, *all_tot = P.tot + kSub * 2 * R;
  const unsigned nsub = nwg < kSub ? nwg : kSub;  // sub-groups in use
  const unsigned sub = me % nsub;
  const unsigned members = (nwg - sub + nsub - 1) / nsub;
  unsigned *sc = bar + 32 * (1 + sub);
  unsigned gen = 0;
  int sub_last = 0;
  // the generation is read before the fence, which waits for the read to return
  // and so orders it before this wave's arrival
  if (lane == 0) gen = __hip_atomic_load(sc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this wave's writes, all XCDs
  if (lane == 0) {
    sub_last = __hip_atomic_fetch_add(sc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               members - 1;
  }
  gen = __shfl(gen, 0);
  sub_last = __shfl(sub_last, 0);
  int top_last = 0;
  if (sub_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (sa >= 0) {
      double va[R], vb[R];
#pragma unroll
      for (int c = 0; c < R; ++c) va[c] = vb[c] = 0.0;
      for (unsigned k = lane; k < members; k += kW) {
        const int64_t w = sub + int64_t(k) * nsub;
#pragma unroll
        for (int c = 0; c < R; ++c) {
          va[c] += P.part[(int64_t(sa) * R + c) * nwg + w];
          vb[c] += P.part[(int64_t(sb) * R + c) * nwg + w];
        }
      }
#pragma unroll
      for (int c = 0; c < R; ++c) {
        va[c] = wave_sum64(va[c]);
        vb[c] = wave_sum64(vb[c]);
      }
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
          sub_tot[sub * 2 * R + c] = va[c];
          sub_tot[sub * 2 * R + R + c] = vb[c];
        }
      }
    }
    // every member has arrived: the counter is reset before the release fence,
    // so the reset is complete before anyone can pass this barrier
    if (lane == 0) __hip_atomic_store(sc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) {
      top_last = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 nsub - 1;
    }
    top_last = __shfl(top_last, 0);
  }
  bool ok = true;
  if (top_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (sa >= 0 && lane < 2 * R) {
      double t = 0.0;
      for (unsigned k = 0; k < nsub; ++k) t += sub_tot[k * 2 * R + lane];
      all_tot[lane] = t;
    }
    if (lane == 0) __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // totals and reset before release
    if (lane == 0) {
      for (unsigned k = 0; k < nsub; ++k)
        __hip_atomic_store(bar + 32 * (1 + k) + 1, gen + 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (lane == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(sc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit ||
          __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
    }
  }
  ok = __shfl(ok ? 1 : 0, 0) != 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (ok && sa >= 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      a[c] = __hip_atomic_load(all_tot + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b[c] = __hip_atomic_load(all_tot + R + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return ok;
}

// plain barrier
template <int R>
__device__ __forceinline__ bool problem_barrier(const BProb &P, unsigned me, unsigned nwg,
                                                int *error) {
  double a[R], b[R];
  return problem_sync<R>(P, me, nwg, error, -1, -1, a, b);
}

// dst = A src over this wave's tiles (src, dst [nn][R] of type T; LDS accumulation
// in FP64), used by the FP64 refresh of the mixed form.  The R right-hand sides are the components of one element product, so the geometry
// is evaluated once per element; PAR: every tile of every problem is a
// parallelepiped tile (flagged at set-up), so only corners 0, 1, 2, 4 are read
// and the closed-form parallelepiped action is used.  Dirichlet corners read
// zero; Dirichlet and shared nodes of dst are set by the caller; right-hand
// sides marked skip are neither read nor written.
template <typename T, int R, bool PAR>
__device__ __forceinline__ void apply_phase(const BProb &P, int me, int nwg, int lane,
                                            double *acc, uint32_t *sId, const T *xyz,
                                            const T *coef_t, const T *src, T *dst,
                                            const bool (&skip)[R]) {
  for (int t = me; t < P.n_tiles; t += nwg) {
    const int n0 = P.node_ptr[t], nm = P.node_ptr[t + 1] - n0;
    const int s0 = P.tile_step[t], s1 = P.tile_step[t + 1];
    // the first step's corner words and coefficient are requested with the staging
    // loads, and each later step's one step ahead, so a step waits for one memory
    // latency (its gathers) instead of two
    uint4 pk_next = make_uint4(0xffffffffu, 0, 0, 0);
    T k_next = T(0);
    if (s0 < s1) {
      pk_next = P.lconn[int64_t(s0) * kW + lane];
      k_next = coef_t[int64_t(s0) * kW + lane];
    }
    // node ids staged kStage per lane per round, all loads of a round issued first
    for (int ib = lane; ib < nm; ib += kStage * kW) {
      uint32_t id[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) id[u] = ib + u * kW < nm ? P.nodes[n0 + ib + u * kW] : 0u;
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int i = ib + u * kW;
        if (i >= nm) continue;
        sId[i] = id[u];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c * P.max_nodes + i] = 0.0;
      }
    }
    __syncthreads();
    for (int s = s0; s < s1; ++s) {
      const int64_t slot = int64_t(s) * kW + lane;
      const uint4 pk = pk_next;
      const T k = k_next;
      if (s + 1 < s1) {
        pk_next = P.lconn[slot + kW];
        k_next = coef_t[slot + kW];
      }
      if (pk.x == 0xffffffffu) continue;
      const int lc[8] = {int(pk.x & 0xffff), int(pk.x >> 16), int(pk.y & 0xffff),
                         int(pk.y >> 16),    int(pk.z & 0xffff), int(pk.z >> 16),
                         int(pk.w & 0xffff), int(pk.w >> 16)};
      int64_t g[8];
      bool fx[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const uint32_t raw = sId[lc[a]];
        g[a] = raw & kIdMaskB;
        fx[a] = (raw & kFixedBitB) != 0;
      }
      T X[3][8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!PAR || a == 0 || a == 1 || a == 2 || a == 4)
#pragma unroll
          for (int d = 0; d < 3; ++d) X[d][a] = xyz[d * P.nn + g[a]];
      T u[R][8], v[R][8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < R; ++c) u[c][a] = (fx[a] || skip[c]) ? T(0) : src[g[a] * R + c];
      if constexpr (PAR)
        laplace_element_parallelepiped_n<T, R>(X, u, k, v);
      else
        laplace_element_n<T, R>(X, u, k, v);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (skip[c]) continue;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          __hip_atomic_fetch_add(&acc[c * P.max_nodes + lc[a]], double(v[c][a]),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    __syncthreads();
    for (int i = lane; i < nm; i += kW) {
      const uint32_t raw = sId[i];
      if (raw & kFixedBitB) continue;  // set by the caller
      const int64_t gg = raw & kIdMaskB;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (skip[c]) continue;
        const T vv = T(acc[c * P.max_nodes + i]);
        if (raw & kSharedBitB)
          unsafeAtomicAdd(&dst[gg * R + c], vv);
        else
          dst[gg * R + c] = vv;
      }
    }
    __syncthreads();
  }
}

// The direction update and q = A p in one pass over this wave's tiles.  For
// each tile node the new direction p = D^-1 r + beta p_old (p = D^-1 r on the
// first iteration) is computed into LDS, where the element loop reads it (zero
// on Dirichlet corners and for finished right-hand sides); the node's writer
// entry also stores it to pnew and, on a Dirichlet node, sets q = p there (its
// row of A p) and adds p^2 to mp.  A node held by several tiles is computed
// by each from the same values, so every copy agrees.  Reading p_old from one
// buffer and writing pnew to the other lets the update run without a barrier
// before the apply.  With the element energies p_e^T A_e p_e (energy), mp
// completes p^T A p.  T is the precision of p, q and the element arithmetic.
template <typename T, int R, bool PAR>
__device__ __forceinline__ void update_apply_phase(const BProb &P, int me, int nwg, int lane,
                                                   double *acc, uint32_t *sId, T *sP,
                                                   const T *xyz, const T *coef_t, const T *pold,
                                                   T *pnew, T *q, const bool (&done)[R],
                                                   const double (&beta)[R], bool first,
                                                   double (&energy)[R], double (&mp)[R]) {
  const int M = P.max_nodes;
  for (int t = me; t < P.n_tiles; t += nwg) {
    const int n0 = P.node_ptr[t], nm = P.node_ptr[t + 1] - n0;
    const int s0 = P.tile_step[t], s1 = P.tile_step[t + 1];
    uint4 pk_next = make_uint4(0xffffffffu, 0, 0, 0);
    T k_next = T(0);
    if (s0 < s1) {
      pk_next = P.lconn[int64_t(s0) * kW + lane];
      k_next = coef_t[int64_t(s0) * kW + lane];
    }
    for (int ib = lane; ib < nm; ib += kStage * kW) {
      uint32_t id[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u)
        id[u] = ib + u * kW < nm ? P.onodes[n0 + ib + u * kW] : 0u;
      double wv[kStage], rv[kStage][R], pv[kStage][R];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const bool in = ib + u * kW < nm;
        const int64_t g = id[u] & kIdMaskOwnB;
        wv[u] = in ? P.w[g] : 0.0;
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const bool ld = in && !done[c];
          rv[u][c] = ld ? P.r[g * R + c] : 0.0;
          pv[u][c] = (ld && !first) ? double(pold[g * R + c]) : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int i = ib + u * kW;
        if (i >= nm) continue;
        const uint32_t raw = id[u];
        const bool fixed = (raw & kFixedBitB) != 0, own = (raw & kOwnBitB) != 0;
        const int64_t g = raw & kIdMaskOwnB;
        sId[i] = raw;
#pragma unroll
        for (int c = 0; c < R; ++c) {
          acc[c * M + i] = 0.0;
          if (done[c]) {
            sP[c * M + i] = T(0);
            continue;
          }
          const T pn = T(wv[u] * rv[u][c] + beta[c] * pv[u][c]);
          sP[c * M + i] = fixed ? T(0) : pn;
          if (own) {
            pnew[g * R + c] = pn;
            if (fixed) {
              q[g * R + c] = pn;  // Dirichlet rows of A p: the entry itself
              mp[c] += double(pn) * double(pn);
            }
          }
        }
      }
    }
    __syncthreads();
    for (int s = s0; s < s1; ++s) {
      const int64_t slot = int64_t(s) * kW + lane;
      const uint4 pk = pk_next;
      const T k = k_next;
      if (s + 1 < s1) {
        pk_next = P.lconn[slot + kW];
        k_next = coef_t[slot + kW];
      }
      if (pk.x == 0xffffffffu) continue;
      const int lc[8] = {int(pk.x & 0xffff), int(pk.x >> 16), int(pk.y & 0xffff),
                         int(pk.y >> 16),    int(pk.z & 0xffff), int(pk.z >> 16),
                         int(pk.w & 0xffff), int(pk.w >> 16)};
      T X[3][8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!PAR || a == 0 || a == 1 || a == 2 || a == 4) {
          const int64_t g = sId[lc[a]] & kIdMaskOwnB;
#pragma unroll
          for (int d = 0; d < 3; ++d) X[d][a] = xyz[d * P.nn + g];
        }
      T u[R][8], v[R][8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < R; ++c) u[c][a] = sP[c * M + lc[a]];
      if constexpr (PAR)
        laplace_element_parallelepiped_n<T, R>(X, u, k, v);
      else
        laplace_element_n<T, R>(X, u, k, v);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (done[c]) continue;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          energy[c] += double(u[c][a]) * double(v[c][a]);
          __hip_atomic_fetch_add(&acc[c * M + lc[a]], double(v[c][a]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    __syncthreads();
    for (int i = lane; i < nm; i += kW) {
      const uint32_t raw = sId[i];
      if (raw & kFixedBitB) continue;  // set above by the writer entry
      const int64_t gg = raw & kIdMaskOwnB;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (done[c]) continue;
        const T vv = T(acc[c * M + i]);
        if (raw & kSharedBitB)
          unsafeAtomicAdd(&q[gg * R + c], vv);
        else
          q[gg * R + c] = vv;
      }
    }
    __syncthreads();
  }
}

template <int R, bool MIXED, bool PAR>
__global__ __launch_bounds__(kW) void k_batched_pcg(const BProb *__restrict__ probs, int nprob,
                                                    const int *__restrict__ wg_prob, double tol2,
                                                    int maxit, double delta2, int *error) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x;
  const BProb P = load_problem(probs + wg_prob[blockIdx.x]);
  const int me = int(blockIdx.x) - P.wg0;
  const int nwg = P.nwg;
  using TP = typename std::conditional<MIXED, float, double>::type;  // precision of p, q
  double *acc = reinterpret_cast<double *>(smem_raw);                  // [R][max_nodes]
  TP *sP = reinterpret_cast<TP *>(acc + R * P.max_nodes);              // [R][max_nodes]
  uint32_t *sId = reinterpret_cast<uint32_t *>(sP + R * P.max_nodes);  // [max_nodes]
  auto part = [&](int slot, int r) { return P.part + (int64_t(slot) * R + r) * nwg; };
  // node range of this wave for the vector phases
  const int64_t chunk = (P.nn + nwg - 1) / nwg;
  const int64_t i0 = min(P.nn, int64_t(me) * chunk), i1 = min(P.nn, i0 + chunk);
  const int64_t rchunk = (P.n_reset + nwg - 1) / nwg;
  const int64_t j0 = min(P.n_reset, int64_t(me) * rchunk), j1 = min(P.n_reset, j0 + rchunk);

  // ---- init: x = 0, r = b, both direction buffers 0 (nodes in no tile keep p = 0),
  // q = 0 on shared nodes; partials rho_0 = b^T D^-1 b, b.b
  {
    double v_rho[R], v_bb[R];
#pragma unroll
    for (int c = 0; c < R; ++c) v_rho[c] = v_bb[c] = 0.0;
    for (int64_t i = i0 + lane; i < i1; i += kW) {
      const double wi = P.w[i];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double bi = P.b[i * R + c];
        P.x[i * R + c] = 0.0;
        P.r[i * R + c] = bi;
        if constexpr (MIXED) {
          P.p32[0][i * R + c] = 0.0f;
          P.p32[1][i * R + c] = 0.0f;
        } else {
          P.p[0][i * R + c] = 0.0;
          P.p[1][i * R + c] = 0.0;
        }
        v_rho[c] += bi * (wi * bi);
        v_bb[c] += bi * bi;
      }
    }
    for (int64_t j = j0 + lane; j < j1; j += kW) {
      const int64_t g = P.reset[j];
      if (P.mask && P.mask[g]) continue;  // Dirichlet rows: set by the first update
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if constexpr (MIXED) {
          P.q32[g * R + c] = 0.0f;
          P.t[g * R + c] = 0.0;  // shared nodes of the refresh apply
        } else {
          P.q[g * R + c] = 0.0;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double a = wave_sum64(v_rho[c]), bq = wave_sum64(v_bb[c]);
      if (lane == 0) {
        part(kRho0, c)[me] = a;
        part(kBB, c)[me] = bq;
      }
    }
  }
  double rho[R], bb[R];
  if (!problem_sync<R>(P, unsigned(me), unsigned(nwg), error, kRho0, kBB, rho, bb)) return;
  bool done[R];
  int it_done[R], st[R], nref[R];
  double rr_last[R], rr_ref[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    done[c] = !(bb[c] > 0.0);
    it_done[c] = 0;
    st[c] = Q1_OK;
    rr_last[c] = rr_ref[c] = bb[c];
    nref[c] = 0;
  }
  bool all_done = true;
#pragma unroll
  for (int c = 0; c < R; ++c) all_done = all_done && done[c];
  double beta[R];
#pragma unroll
  for (int c = 0; c < R; ++c) beta[c] = 0.0;

  for (int it = 1; it <= maxit && !all_done; ++it) {
    // ---- P1: p = D^-1 r + beta p_old and q = A p over this wave's tiles, with the
    // partials of p^T A p (element energies, Dirichlet p^2).  The direction
    // buffers of this iteration and the previous one are selected, not indexed,
    // so that the problem record stays in registers.
    const bool odd = (it & 1) != 0;
    double *const p64 = odd ? P.p[1] : P.p[0];
    double *const p64_old = odd ? P.p[0] : P.p[1];
    float *const p32 = odd ? P.p32[1] : P.p32[0];
    float *const p32_old = odd ? P.p32[0] : P.p32[1];
    double energy[R], v_mp[R];
#pragma unroll
    for (int c = 0; c < R; ++c) energy[c] = v_mp[c] = 0.0;
    if constexpr (MIXED)
      update_apply_phase<float, R, PAR>(P, me, nwg, lane, acc, sId, sP, P.xyz32, P.coef32,
                                        p32_old, p32, P.q32, done, beta, it == 1,
                                        energy, v_mp);
    else
      update_apply_phase<double, R, PAR>(P, me, nwg, lane, acc, sId, sP, P.xyz, P.coef_t,
                                         p64_old, p64, P.q, done, beta, it == 1, energy,
                                         v_mp);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double e = wave_sum64(energy[c]), m = wave_sum64(v_mp[c]);
      if (lane == 0) {
        part(kEnergy, c)[me] = e;
        part(kMp2, c)[me] = m;
      }
    }
    double alpha[R], en[R], mp[R];
    if (!problem_sync<R>(P, unsigned(me), unsigned(nwg), error, kEnergy, kMp2, en, mp)) return;

    // ---- P2: alpha, x, r; partials rho', r.r
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double pq = en[c] + mp[c];
      alpha[c] = 0.0;
      if (!done[c]) {
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho[c])) {
          done[c] = true;
          st[c] = Q1_EBREAKDOWN;
          it_done[c] = it - 1;
        } else {
          alpha[c] = rho[c] / pq;
        }
      }
    }
    {
      double v_rho[R], v_rr[R];
#pragma unroll
      for (int c = 0; c < R; ++c) v_rho[c] = v_rr[c] = 0.0;
      for (int64_t ib = i0 + lane; ib < i1; ib += kU * kW) {
        double wv[kU], po[kU][R], qo[kU][R], xo[kU][R], ro[kU][R];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int64_t i = ib + u * kW;
          const bool in = i < i1;
          wv[u] = in ? P.w[i] : 0.0;
#pragma unroll
          for (int c = 0; c < R; ++c) {
            const int64_t o = i * R + c;
            const bool ld = in && !done[c];
            if constexpr (MIXED) {
              po[u][c] = ld ? double(p32[o]) : 0.0;
              qo[u][c] = ld ? double(P.q32[o]) : 0.0;
            } else {
              po[u][c] = ld ? p64[o] : 0.0;
              qo[u][c] = ld ? P.q[o] : 0.0;
            }
            xo[u][c] = ld ? P.x[o] : 0.0;
            ro[u][c] = ld ? P.r[o] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int64_t i = ib + u * kW;
          if (i >= i1) continue;
#pragma unroll
          for (int c = 0; c < R; ++c) {
            if (done[c]) continue;
            const int64_t o = i * R + c;
            P.x[o] = xo[u][c] + alpha[c] * po[u][c];
            const double rn = ro[u][c] - alpha[c] * qo[u][c];
            P.r[o] = rn;
            // q was last read here: zero it for the next P1, whose tiles store
            // their private nodes and add into shared ones (P3 then sets the
            // Dirichlet rows)
            if constexpr (MIXED)
              P.q32[o] = 0.0f;
            else
              P.q[o] = 0.0;
            v_rho[c] += rn * wv[u] * rn;
            v_rr[c] += rn * rn;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double a = wave_sum64(v_rho[c]), bq = wave_sum64(v_rr[c]);
        if (lane == 0) {
          part(kRho, c)[me] = a;
          part(kRR, c)[me] = bq;
        }
      }
    }
    double rho_n[R], rr_n[R];
    if (!problem_sync<R>(P, unsigned(me), unsigned(nwg), error, kRho, kRR, rho_n, rr_n)) return;

    // ---- convergence and beta (the direction update runs with the next apply)
    bool refresh[R];
    bool any_refresh = false;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      beta[c] = 0.0;
      refresh[c] = false;
      if (done[c]) continue;
      const double rho1 = rho_n[c];
      const double rr = rr_n[c];
      rr_last[c] = rr;
      if constexpr (MIXED) {
        // the recurrence only triggers a refresh; convergence is decided on b - A64 x
        if (!isfinite(rr)) {
          done[c] = true;
          st[c] = Q1_EBREAKDOWN;
          it_done[c] = it;
        } else if (rr <= fmax(delta2 * rr_ref[c], 0.5 * tol2 * bb[c]) || it >= maxit) {
          refresh[c] = true;
          any_refresh = true;
        } else {
          beta[c] = rho1 / rho[c];
          rho[c] = rho1;
        }
      } else {
        if (rr <= tol2 * bb[c] || !isfinite(rr) || it >= maxit) {
          done[c] = true;
          st[c] = rr <= tol2 * bb[c] ? Q1_OK : (!isfinite(rr) ? Q1_EBREAKDOWN : Q1_ENOCONV);
          it_done[c] = it;
        } else {
          beta[c] = rho1 / rho[c];
          rho[c] = rho1;
        }
      }
    }
    if constexpr (MIXED) {
      if (any_refresh) {
        // R1: t = A64 x for the refreshed right-hand sides (FP64 geometry and coefficients)
        bool skip[R];
#pragma unroll
        for (int c = 0; c < R; ++c) skip[c] = !refresh[c];
        apply_phase<double, R, PAR>(P, me, nwg, lane, acc, sId, P.xyz, P.coef_t, P.x, P.t, skip);
        if (!problem_barrier<R>(P, unsigned(me), unsigned(nwg), error)) return;
        // R2: r = b - A64 x (Dirichlet rows are the identity); partials rho', r.r
        double v_rho[R], v_rr[R];
#pragma unroll
        for (int c = 0; c < R; ++c) v_rho[c] = v_rr[c] = 0.0;
        for (int64_t i = i0 + lane; i < i1; i += kW) {
          const double wi = P.w[i];
          const bool fx = P.mask && P.mask[i];
#pragma unroll
          for (int c = 0; c < R; ++c) {
            if (!refresh[c]) continue;
            const int64_t o = i * R + c;
            const double rn = P.b[o] - (fx ? P.x[o] : P.t[o]);
            P.r[o] = rn;
            v_rho[c] += rn * wi * rn;
            v_rr[c] += rn * rn;
          }
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const double a = wave_sum64(v_rho[c]), bq = wave_sum64(v_rr[c]);
          if (lane == 0) {
            part(kRho, c)[me] = a;
            part(kRR, c)[me] = bq;
          }
        }
        if (!problem_sync<R>(P, unsigned(me), unsigned(nwg), error, kRho, kRR, rho_n, rr_n))
          return;
        // R3: decide on the true residual; otherwise continue from it with p kept
#pragma unroll
        for (int c = 0; c < R; ++c) {
          if (!refresh[c]) continue;
          const double rho1 = rho_n[c];
          const double rr = rr_n[c];
          rr_last[c] = rr;
          ++nref[c];
          if (rr <= tol2 * bb[c] || !isfinite(rr) || it >= maxit) {
            done[c] = true;
            st[c] = rr <= tol2 * bb[c] ? Q1_OK : (!isfinite(rr) ? Q1_EBREAKDOWN : Q1_ENOCONV);
            it_done[c] = it;
          } else {
            rr_ref[c] = rr;
            beta[c] = rho1 / rho[c];
            rho[c] = rho1;
          }
        }
        // shared nodes of t start the next refresh at zero (their values were read in R2)
        for (int64_t j = j0 + lane; j < j1; j += kW) {
          const int64_t g = P.reset[j];
          if (P.mask && P.mask[g]) continue;
#pragma unroll
          for (int c = 0; c < R; ++c)
            if (refresh[c]) P.t[g * R + c] = 0.0;
        }
      }
    }
    all_done = true;
#pragma unroll
    for (int c = 0; c < R; ++c) all_done = all_done && done[c];
    if (all_done) break;
  }
  if (me == 0 && lane == 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      P.iters[c] = it_done[c];
      P.status[c] = done[c] ? st[c] : Q1_ENOCONV;
      P.rr[c] = rr_last[c];
      P.bb[c] = bb[c];
      P.nref[c] = nref[c];
    }
  }
}

// interleave: dst[i*R + c] = src_c[i]; and back
__global__ void k_interleave(int64_t n, int R, int c, const double *__restrict__ src,
                             double *__restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i * R + c] = src[i];
}
__global__ void k_deinterleave(int64_t n, int R, int c, const double *__restrict__ src,
                               double *__restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i * R + c];
}
__global__ void k_invert(int64_t n, double *__restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;  // 0 on zero rows (unreferenced nodes)
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}

__global__ void k_fill_i32(int64_t n, int32_t *__restrict__ a, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// first[g] = the smallest entry index of node g over the tile node lists
__global__ void k_first_entry(int64_t nent, const uint32_t *__restrict__ nodes,
                              int32_t *__restrict__ first) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nent) atomicMin(&first[nodes[e] & kIdMaskB], int32_t(e));
}

// the node lists with the writer bit set on each node's first entry
__global__ void k_mark_writers(int64_t nent, const uint32_t *__restrict__ nodes,
                               const int32_t *__restrict__ first, uint32_t *__restrict__ onodes) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  const uint32_t raw = nodes[e];
  onodes[e] = raw | (first[raw & kIdMaskB] == int32_t(e) ? kOwnBitB : 0u);
}

template <int R, bool MIXED, bool PAR>
int run_batched(const std::vector<BProb> &hp, const std::vector<int> &wg_prob, double tol2,
                int maxit, double delta2, size_t lds, hipStream_t s, int *d_error) {
  BProb *dp = nullptr;
  int *dwg = nullptr;
  Q1_HIP(hipMalloc(&dp, hp.size() * sizeof(BProb)));
  Q1_HIP(hipMalloc(&dwg, wg_prob.size() * sizeof(int)));
  Q1_HIP(hipMemcpy(dp, hp.data(), hp.size() * sizeof(BProb), hipMemcpyHostToDevice));
  Q1_HIP(hipMemcpy(dwg, wg_prob.data(), wg_prob.size() * sizeof(int), hipMemcpyHostToDevice));
  int nprob = int(hp.size());
  void *args[] = {&dp, &nprob, &dwg, &tol2, &maxit, &delta2, &d_error};
  hipError_t e = hipLaunchCooperativeKernel(
      reinterpret_cast<const void *>(k_batched_pcg<R, MIXED, PAR>),
      dim3(unsigned(wg_prob.size())), dim3(kW), args, unsigned(lds), s);
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(dp);
  (void)hipFree(dwg);
  if (e != hipSuccess) return fail(Q1_EHIP, "cooperative launch failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(Q1_EHIP, "batched PCG: %s", hipGetErrorString(e2));
  return Q1_OK;
}

template <int R, bool MIXED, bool PAR>
int max_coresident(size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(k_batched_pcg<R, MIXED, PAR>), kW, lds) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

template <bool MIXED, bool PAR>
int coresident_for(int nrhs, size_t lds) {
  switch (nrhs) {
    case 1: return max_coresident<1, MIXED, PAR>(lds);
    case 2: return max_coresident<2, MIXED, PAR>(lds);
    case 3: return max_coresident<3, MIXED, PAR>(lds);
    default: return max_coresident<4, MIXED, PAR>(lds);
  }
}

template <bool MIXED, bool PAR>
int run_for(int nrhs, const std::vector<BProb> &hp, const std::vector<int> &wg_prob, double tol2,
            int maxit, double delta2, size_t lds, hipStream_t s, int *d_error) {
  switch (nrhs) {
    case 1: return run_batched<1, MIXED, PAR>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    case 2: return run_batched<2, MIXED, PAR>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    case 3: return run_batched<3, MIXED, PAR>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    default: return run_batched<4, MIXED, PAR>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
  }
}

// Shared host side of the FP64 and mixed-precision batched solvers.
int batched_impl(const char *name, bool mixed, int nprob, q1_op *const *ops, int nrhs,
                 const double *const *b_d, double *const *x_d, double rtol, double delta,
                 int maxit, q1_stats *st, hipStream_t s) {
  Q1_CHECK(nprob > 0 && ops && b_d && x_d, Q1_EINVAL, "%s: bad arguments", name);
  Q1_CHECK(nrhs >= 1 && nrhs <= kRmax, Q1_EINVAL, "%s: 1 <= nrhs <= %d", name, kRmax);
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "%s: bad tolerance or limit", name);
  Q1_CHECK(!mixed || (delta > 0 && delta < 1), Q1_EINVAL, "%s: need 0 < delta < 1", name);
  int64_t total_elems = 0;
  int max_nodes = 0;
  for (int p = 0; p < nprob; ++p) {
    const Op *o = reinterpret_cast<const Op *>(ops[p]);
    Q1_CHECK(o, Q1_EINVAL, "%s: NULL operator %d", name, p);
    Q1_CHECK(o->physics == Q1_LAPLACE && o->dtype == Q1_F64 && o->variant == Q1_V_LDS_TILE,
             Q1_EUNSUPPORTED, "%s: operator %d must be an FP64 scalar-Laplace LDS-tile operator",
             name, p);
    for (int c = 0; c < nrhs; ++c)
      Q1_CHECK(b_d[p * nrhs + c] && x_d[p * nrhs + c], Q1_EINVAL, "%s: NULL vector", name);
    total_elems += o->n_elems;
    max_nodes = std::max(max_nodes, o->tiles.max_nodes);
  }
  // LDS per wave: FP64 accumulators, the staged directions (FP32 in the mixed form)
  // and the node words
  const size_t lds = size_t(max_nodes) * (size_t(nrhs) * sizeof(double) +
                                          size_t(nrhs) * (mixed ? sizeof(float) : sizeof(double)) +
                                          sizeof(uint32_t));
  bool par = true;  // every tile of every problem a parallelepiped tile
  for (int p = 0; p < nprob; ++p) par = par && reinterpret_cast<const Op *>(ops[p])->tiles.all_affine;
  const int cap = mixed ? (par ? coresident_for<true, true>(nrhs, lds)
                               : coresident_for<true, false>(nrhs, lds))
                        : (par ? coresident_for<false, true>(nrhs, lds)
                               : coresident_for<false, false>(nrhs, lds));
  Q1_CHECK(cap >= nprob, Q1_EUNSUPPORTED,
           "%s: %d problems need one co-resident wave each, but only %d fit", name, nprob, cap);
  // waves per problem in proportion to its expected work, at least one each:
  // elements times iterations, and Jacobi-PCG iterations on an n^3 grid grow
  // like n, so the weight is n_elems^(4/3)
  std::vector<int> nwg(nprob, 1);
  int spare = cap - nprob;
  double wsum = 0.0;
  for (int p = 0; p < nprob; ++p)
    wsum += std::pow(double(reinterpret_cast<const Op *>(ops[p])->n_elems), 4.0 / 3.0);
  for (int p = 0; p < nprob; ++p) {
    const Op *o = reinterpret_cast<const Op *>(ops[p]);
    const double wp = std::pow(double(o->n_elems), 4.0 / 3.0);
    const int extra = int(double(spare) * wp / std::max(1.0, wsum));
    nwg[p] += std::min(extra, std::max(0, o->tiles.n_tiles - 1));
  }
  // device workspace per problem
  std::vector<void *> allocs;
  struct Guard {
    std::vector<void *> &a;
    ~Guard() {
      for (void *p : a) (void)hipFree(p);
    }
  } guard{allocs};
  auto dalloc = [&](void **ptr, size_t bytes) -> int {
    Q1_HIP(hipMalloc(ptr, std::max<size_t>(bytes, 8)));
    allocs.push_back(*ptr);
    return Q1_OK;
  };
  int *d_error = nullptr;
  int rc;
  if ((rc = dalloc(reinterpret_cast<void **>(&d_error), sizeof(int)))) return rc;
  Q1_HIP(hipMemsetAsync(d_error, 0, sizeof(int), s));
  std::vector<BProb> hp(nprob);
  std::vector<int> wg_prob;
  int *d_iters = nullptr, *d_status = nullptr, *d_nref = nullptr;
  double *d_rr = nullptr, *d_bb = nullptr;
  const size_t nres = size_t(nprob) * nrhs;
  if ((rc = dalloc(reinterpret_cast<void **>(&d_iters), nres * sizeof(int))) ||
      (rc = dalloc(reinterpret_cast<void **>(&d_status), nres * sizeof(int))) ||
      (rc = dalloc(reinterpret_cast<void **>(&d_nref), nres * sizeof(int))) ||
      (rc = dalloc(reinterpret_cast<void **>(&d_rr), nres * sizeof(double))) ||
      (rc = dalloc(reinterpret_cast<void **>(&d_bb), nres * sizeof(double))))
    return rc;
  auto grid = [](int64_t n) { return dim3(unsigned((n + 255) / 256)); };
  for (int p = 0; p < nprob; ++p) {
    Op &o = *reinterpret_cast<Op *>(ops[p]);
    const TileMap &tm = o.tiles;
    BProb &B = hp[p];
    B = BProb{};
    const int64_t n = o.n_nodes;
    B.nn = n;
    B.n_tiles = tm.n_tiles;
    B.max_nodes = max_nodes;
    B.node_ptr = tm.node_ptr;
    B.nodes = tm.nodes;
    B.tile_step = tm.tile_step;
    B.lconn = reinterpret_cast<const uint4 *>(tm.lconn);
    B.coef_t = static_cast<const double *>(tm.coef_t);
    B.xyz = static_cast<const double *>(o.xyz);
    B.reset = tm.reset;
    B.n_reset = tm.n_reset;
    B.mask = o.mask;
    Q1_CHECK(n < int64_t(kIdMaskOwnB), Q1_EUNSUPPORTED, "%s: operator %d has %lld nodes (at most %u)",
             name, p, (long long)n, kIdMaskOwnB);
    // the node lists with the writer bit on each node's first entry (first tile in order)
    {
      const int64_t nent = tm.n_entries;
      int32_t *first = nullptr;
      uint32_t *onodes = nullptr;
      if ((rc = dalloc(reinterpret_cast<void **>(&first), size_t(n) * sizeof(int32_t))) ||
          (rc = dalloc(reinterpret_cast<void **>(&onodes), size_t(nent) * sizeof(uint32_t))))
        return rc;
      hipLaunchKernelGGL(k_fill_i32, grid(n), dim3(256), 0, s, n, first, INT32_MAX);
      hipLaunchKernelGGL(k_first_entry, grid(nent), dim3(256), 0, s, nent, tm.nodes, first);
      hipLaunchKernelGGL(k_mark_writers, grid(nent), dim3(256), 0, s, nent, tm.nodes, first,
                         onodes);
      B.onodes = onodes;
    }
    const size_t nv = size_t(n) * nrhs;
    double *vec[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int v = 0; v < 6; ++v) {
      if (mixed && v >= 3) continue;  // p, q are FP32 in the mixed form
      if ((rc = dalloc(reinterpret_cast<void **>(&vec[v]), nv * sizeof(double)))) return rc;
    }
    B.b = vec[0]; B.x = vec[1]; B.r = vec[2]; B.q = vec[3]; B.p[0] = vec[4]; B.p[1] = vec[5];
    if (mixed) {
      // FP32 copies of the geometry and of the lane-ordered coefficients: the FP32 operator
      float *xyz32 = nullptr, *coef32 = nullptr;
      const int64_t ncoef = tm.n_steps * kW;
      if ((rc = dalloc(reinterpret_cast<void **>(&B.p32[0]), nv * sizeof(float))) ||
          (rc = dalloc(reinterpret_cast<void **>(&B.p32[1]), nv * sizeof(float))) ||
          (rc = dalloc(reinterpret_cast<void **>(&B.q32), nv * sizeof(float))) ||
          (rc = dalloc(reinterpret_cast<void **>(&B.t), nv * sizeof(double))) ||
          (rc = dalloc(reinterpret_cast<void **>(&xyz32), size_t(3 * n) * sizeof(float))) ||
          (rc = dalloc(reinterpret_cast<void **>(&coef32), size_t(ncoef) * sizeof(float))))
        return rc;
      hipLaunchKernelGGL(k_to_f32, grid(3 * n), dim3(256), 0, s, 3 * n, B.xyz, xyz32);
      hipLaunchKernelGGL(k_to_f32, grid(ncoef), dim3(256), 0, s, ncoef, B.coef_t, coef32);
      B.xyz32 = xyz32;
      B.coef32 = coef32;
    }
    double *w = nullptr;
    if ((rc = dalloc(reinterpret_cast<void **>(&w), size_t(n) * sizeof(double)))) return rc;
    if ((rc = launch_diag(o, w, s))) return rc;
    hipLaunchKernelGGL(k_invert, grid(n), dim3(256), 0, s, n, w);
    B.w = w;
    for (int c = 0; c < nrhs; ++c)
      hipLaunchKernelGGL(k_interleave, grid(n), dim3(256), 0, s, n, nrhs, c, b_d[p * nrhs + c],
                         B.b);
    if ((rc = dalloc(reinterpret_cast<void **>(&B.part), size_t(kSlots) * nrhs * nwg[p] *
                                                             sizeof(double))))
      return rc;
    if ((rc = dalloc(reinterpret_cast<void **>(&B.bar), kBarWords * sizeof(unsigned)))) return rc;
    if ((rc = dalloc(reinterpret_cast<void **>(&B.tot), (kSub + 1) * 2 * nrhs * sizeof(double))))
      return rc;
    Q1_HIP(hipMemsetAsync(B.bar, 0, kBarWords * sizeof(unsigned), s));
    B.wg0 = int(wg_prob.size());
    B.nwg = nwg[p];
    for (int k = 0; k < nwg[p]; ++k) wg_prob.push_back(p);
    B.iters = d_iters + p * nrhs;
    B.status = d_status + p * nrhs;
    B.nref = d_nref + p * nrhs;
    B.rr = d_rr + p * nrhs;
    B.bb = d_bb + p * nrhs;
  }
  Q1_HIP(hipGetLastError());
  Q1_HIP(hipStreamSynchronize(s));
  const auto t_setup = std::chrono::steady_clock::now();
  const double tol2 = rtol * rtol, delta2 = delta * delta;
  rc = mixed ? (par ? run_for<true, true>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s, d_error)
                    : run_for<true, false>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s, d_error))
             : (par ? run_for<false, true>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s, d_error)
                    : run_for<false, false>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s,
                                            d_error));
  if (rc) return rc;
  const auto t_solve = std::chrono::steady_clock::now();
  int h_error = 0;
  Q1_HIP(hipMemcpy(&h_error, d_error, sizeof(int), hipMemcpyDeviceToHost));
  Q1_CHECK(h_error == 0, Q1_EHIP, "%s: a problem barrier timed out", name);
  for (int p = 0; p < nprob; ++p)
    for (int c = 0; c < nrhs; ++c)
      hipLaunchKernelGGL(k_deinterleave, grid(hp[p].nn), dim3(256), 0, s, hp[p].nn, nrhs, c,
                         hp[p].x, x_d[p * nrhs + c]);
  Q1_HIP(hipGetLastError());
  std::vector<int> h_it(nres), h_st(nres), h_nref(nres);
  std::vector<double> h_rr(nres), h_bb(nres);
  Q1_HIP(hipMemcpy(h_it.data(), d_iters, nres * sizeof(int), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(h_st.data(), d_status, nres * sizeof(int), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(h_nref.data(), d_nref, nres * sizeof(int), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(h_rr.data(), d_rr, nres * sizeof(double), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(h_bb.data(), d_bb, nres * sizeof(double), hipMemcpyDeviceToHost));
  const double secs = std::chrono::duration<double>(t_solve - t_setup).count();
  int worst = Q1_OK;
  for (size_t k = 0; k < nres; ++k) {
    if (st) {
      st[k].iters = h_it[k];
      st[k].status = h_st[k];
      st[k].rel_res = h_bb[k] > 0 ? std::sqrt(h_rr[k] / h_bb[k]) : 0.0;
      st[k].true_rel_res = st[k].rel_res;
      st[k].seconds = secs;       // one launch for all solves
      st[k].fallback_at = -1;
      st[k].outer_iters = h_nref[k];
    }
    if (h_st[k] == Q1_EBREAKDOWN) worst = Q1_EBREAKDOWN;
    else if (h_st[k] == Q1_ENOCONV && worst == Q1_OK) worst = Q1_ENOCONV;
  }
  return worst;
}

}  // namespace
}  // namespace q1

using namespace q1;

extern "C" int q1_batched_pcg(int nprob, q1_op *const *ops, int nrhs,
                              const double *const *b_d, double *const *x_d, double rtol,
                              int maxit, q1_stats *st, void *stream) {
  return batched_impl("q1_batched_pcg", false, nprob, ops, nrhs, b_d, x_d, rtol, 0.0, maxit, st,
                      static_cast<hipStream_t>(stream));
}

extern "C" int q1_batched_mpcg(int nprob, q1_op *const *ops, int nrhs,
                               const double *const *b_d, double *const *x_d, double rtol,
                               double delta, int maxit, q1_stats *st, void *stream) {
  return batched_impl("q1_batched_mpcg", true, nprob, ops, nrhs, b_d, x_d, rtol, delta, maxit, st,
                      static_cast<hipStream_t>(stream));
}
