// Batched persistent Jacobi-PCG: many independent scalar-Laplace problems,
// each with up to four right-hand sides, solved by ONE cooperative launch.
//
// Each problem p owns a contiguous range of single-wavefront workgroups
// (sized in proportion to its element count).  The waves of a problem meet at
// a barrier built from two global counters; problems never wait for each
// other.  Vectors are stored interleaved [node][R] so that one gather of a
// node serves all R right-hand sides.  Per iteration (the CG operations of
// Table 4):
//   P1  q = A p through the operator's LDS tiles (as in q1_tile.hip), and the
//       partial sums of p^T A p as element energies sum_e p_e^T A_e p_e
//   P2  alpha = rho / p^T A p; x += alpha p; r -= alpha q; partials of
//       rho' = r^T D^{-1} r and r^T r
//   P3  convergence test; beta = rho'/rho; p = D^{-1} r + beta p; q = p on
//       Dirichlet nodes (their rows of A p) and q = 0 on nodes shared between
//       tiles, ready for the next P1; partials of sum p_c^2 over Dirichlet
//       nodes
// with one barrier after each phase.  In the mixed-precision form the search
// directions p, q and the applies of P1 are FP32 (the FP32 operator's
// coordinates and coefficients), while x, r and every dot product stay FP64;
// whenever the recurrence residual has fallen by delta since the last refresh
// (and before convergence is declared) the true residual r = b - A64 x is
// recomputed with an FP64 apply of x inside the same launch (three more
// barriers), and the recurrences continue from it with p kept.
// Every wave re-reduces the partials in
// the same order, so all waves of a problem hold bit-identical scalars and
// take the same branch.  Each barrier wait has a spin limit: past it the
// kernel records an error and every wave returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
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
constexpr unsigned kSpinLimit = 1u << 26;  // barrier polls before giving up

// partial-sum slots per problem: [slot][rhs][nwg]
enum { kEnergy = 0, kMp2 = 1, kRho = 2, kRR = 3, kBB = 4, kRho0 = 5, kSlots = 6 };

struct BProb {
  int64_t nn;
  int n_tiles, max_nodes;
  const int32_t *node_ptr;
  const uint32_t *nodes;
  const int32_t *tile_step;
  const uint4 *lconn;
  const double *coef_t;
  const double *xyz;
  const int32_t *reset;
  int64_t n_reset;
  const uint8_t *mask;
  double *b, *x, *r, *p, *q;  // [nn][R]
  const double *w;            // inverse diagonal [nn]
  // mixed precision: FP32 geometry, coefficients and directions; FP64 refresh output
  const float *xyz32, *coef32;
  float *p32, *q32;           // [nn][R]
  double *t;                  // [nn][R]
  double *part;               // [kSlots][R][nwg]
  unsigned *bar;              // [2]: arrival count, generation
  int wg0, nwg;
  int *iters, *status, *nref; // [R]
  double *rr, *bb;            // [R]
};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// sum of n partials in a fixed order, returned to every lane
__device__ __forceinline__ double reduce_partials(const double *part, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kW) s += __hip_atomic_load(part + i, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
  return wave_sum64(s);
}

// barrier of the nwg waves of one problem; false when the spin limit was hit
__device__ __forceinline__ bool problem_barrier(unsigned *bar, unsigned nwg, int *error) {
  bool ok = true;
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // writes visible to other XCDs
    const unsigned arrived =
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nwg - 1) {
      __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit || __hip_atomic_load(error, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  ok = __shfl(ok ? 1 : 0, 0) != 0;
  return ok;
}

// q = A src over this wave's tiles (src, dst [nn][R] of type T; LDS accumulation in
// FP64), and with ENERGY the element energies src_e^T A_e src_e.  Dirichlet
// corners read zero; Dirichlet and shared nodes of dst are set by the caller.
template <typename T, int R, bool ENERGY>
__device__ __forceinline__ void apply_phase(const BProb &P, int me, int nwg, int lane,
                                            double *acc, uint32_t *sId, const T *xyz,
                                            const T *coef_t, const T *src, T *dst,
                                            const bool (&done)[R], double (&energy)[R]) {
  for (int t = me; t < P.n_tiles; t += nwg) {
    const int n0 = P.node_ptr[t], nm = P.node_ptr[t + 1] - n0;
    for (int i = lane; i < nm; i += kW) {
      sId[i] = P.nodes[n0 + i];
#pragma unroll
      for (int c = 0; c < R; ++c) acc[c * P.max_nodes + i] = 0.0;
    }
    __syncthreads();
    for (int s = P.tile_step[t]; s < P.tile_step[t + 1]; ++s) {
      const int64_t slot = int64_t(s) * kW + lane;
      const uint4 pk = P.lconn[slot];
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
      T X0[3][8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) X0[d][a] = xyz[d * P.nn + g[a]];
      const T k = coef_t[slot];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (done[c]) continue;
        T X[3][8], u[8], v[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          X[0][a] = X0[0][a]; X[1][a] = X0[1][a]; X[2][a] = X0[2][a];
          u[a] = fx[a] ? T(0) : src[g[a] * R + c];
        }
        laplace_element<T>(X, u, k, v);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          if constexpr (ENERGY) energy[c] += double(u[a]) * double(v[a]);
          __hip_atomic_fetch_add(&acc[c * P.max_nodes + lc[a]], double(v[a]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
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
        if (done[c]) continue;
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

template <int R, bool MIXED>
__global__ __launch_bounds__(kW) void k_batched_pcg(const BProb *__restrict__ probs, int nprob,
                                                    const int *__restrict__ wg_prob, double tol2,
                                                    int maxit, double delta2, int *error) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x;
  const BProb P = probs[wg_prob[blockIdx.x]];
  const int me = int(blockIdx.x) - P.wg0;
  const int nwg = P.nwg;
  double *acc = reinterpret_cast<double *>(smem_raw);                        // [R][max_nodes]
  uint32_t *sId = reinterpret_cast<uint32_t *>(acc + R * P.max_nodes);       // [max_nodes]
  auto part = [&](int slot, int r) { return P.part + (int64_t(slot) * R + r) * nwg; };
  // node range of this wave for the vector phases
  const int64_t chunk = (P.nn + nwg - 1) / nwg;
  const int64_t i0 = min(P.nn, int64_t(me) * chunk), i1 = min(P.nn, i0 + chunk);
  const int64_t rchunk = (P.n_reset + nwg - 1) / nwg;
  const int64_t j0 = min(P.n_reset, int64_t(me) * rchunk), j1 = min(P.n_reset, j0 + rchunk);

  // ---- init: x = 0, r = b, p = w b, q reset; partials rho_0, b.b, Dirichlet p^2
  {
    double v_rho[R], v_bb[R], v_mp[R];
#pragma unroll
    for (int c = 0; c < R; ++c) v_rho[c] = v_bb[c] = v_mp[c] = 0.0;
    for (int64_t i = i0 + lane; i < i1; i += kW) {
      const double wi = P.w[i];
      const bool fx = P.mask && P.mask[i];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double bi = P.b[i * R + c];
        double zi = wi * bi;
        P.x[i * R + c] = 0.0;
        P.r[i * R + c] = bi;
        if constexpr (MIXED) {
          const float zf = float(zi);
          P.p32[i * R + c] = zf;
          v_rho[c] += bi * zi;
          zi = double(zf);
        } else {
          P.p[i * R + c] = zi;
          v_rho[c] += bi * zi;
        }
        v_bb[c] += bi * bi;
        if (fx) v_mp[c] += zi * zi;
      }
    }
    for (int64_t j = j0 + lane; j < j1; j += kW) {
      const int64_t g = P.reset[j];
      const bool fx = P.mask && P.mask[g];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double qg = fx ? P.w[g] * P.b[g * R + c] : 0.0;
        if constexpr (MIXED) {
          P.q32[g * R + c] = float(qg);
          if (!fx) P.t[g * R + c] = 0.0;  // shared nodes of the refresh apply
        } else {
          P.q[g * R + c] = qg;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double a = wave_sum64(v_rho[c]), bq = wave_sum64(v_bb[c]), m = wave_sum64(v_mp[c]);
      if (lane == 0) {
        part(kRho0, c)[me] = a;
        part(kBB, c)[me] = bq;
        part(kMp2, c)[me] = m;
      }
    }
  }
  if (!problem_barrier(P.bar, nwg, error)) return;
  double rho[R], bb[R];
  bool done[R];
  int it_done[R], st[R], nref[R];
  double rr_last[R], rr_ref[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    rho[c] = reduce_partials(part(kRho0, c), nwg);
    bb[c] = reduce_partials(part(kBB, c), nwg);
    done[c] = !(bb[c] > 0.0);
    it_done[c] = 0;
    st[c] = Q1_OK;
    rr_last[c] = rr_ref[c] = bb[c];
    nref[c] = 0;
  }
  bool all_done = true;
#pragma unroll
  for (int c = 0; c < R; ++c) all_done = all_done && done[c];

  for (int it = 1; it <= maxit && !all_done; ++it) {
    // ---- P1: q = A p over this wave's tiles, element energies p_e^T A_e p_e
    double energy[R];
#pragma unroll
    for (int c = 0; c < R; ++c) energy[c] = 0.0;
    if constexpr (MIXED)
      apply_phase<float, R, true>(P, me, nwg, lane, acc, sId, P.xyz32, P.coef32, P.p32, P.q32,
                                  done, energy);
    else
      apply_phase<double, R, true>(P, me, nwg, lane, acc, sId, P.xyz, P.coef_t, P.p, P.q, done,
                                   energy);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double e = wave_sum64(energy[c]);
      if (lane == 0) part(kEnergy, c)[me] = e;
    }
    if (!problem_barrier(P.bar, nwg, error)) return;

    // ---- P2: alpha, x, r; partials rho', r.r
    double alpha[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double pq = reduce_partials(part(kEnergy, c), nwg) + reduce_partials(part(kMp2, c), nwg);
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
      for (int64_t i = i0 + lane; i < i1; i += kW) {
        const double wi = P.w[i];
#pragma unroll
        for (int c = 0; c < R; ++c) {
          if (done[c]) continue;
          const int64_t o = i * R + c;
          double po, qo;
          if constexpr (MIXED) {
            po = double(P.p32[o]);
            qo = double(P.q32[o]);
          } else {
            po = P.p[o];
            qo = P.q[o];
          }
          P.x[o] += alpha[c] * po;
          const double rn = P.r[o] - alpha[c] * qo;
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
    }
    if (!problem_barrier(P.bar, nwg, error)) return;

    // ---- P3: convergence, beta, p; reset q on shared and Dirichlet nodes
    double beta[R];
    bool refresh[R];
    bool any_refresh = false;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      beta[c] = 0.0;
      refresh[c] = false;
      if (done[c]) continue;
      const double rho1 = reduce_partials(part(kRho, c), nwg);
      const double rr = reduce_partials(part(kRR, c), nwg);
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
        double unused[R];
#pragma unroll
        for (int c = 0; c < R; ++c) skip[c] = !refresh[c];
        apply_phase<double, R, false>(P, me, nwg, lane, acc, sId, P.xyz, P.coef_t, P.x, P.t,
                                      skip, unused);
        if (!problem_barrier(P.bar, nwg, error)) return;
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
        if (!problem_barrier(P.bar, nwg, error)) return;
        // R3: decide on the true residual; otherwise continue from it with p kept
#pragma unroll
        for (int c = 0; c < R; ++c) {
          if (!refresh[c]) continue;
          const double rho1 = reduce_partials(part(kRho, c), nwg);
          const double rr = reduce_partials(part(kRR, c), nwg);
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
    {
      double v_mp[R];
#pragma unroll
      for (int c = 0; c < R; ++c) v_mp[c] = 0.0;
      for (int64_t i = i0 + lane; i < i1; i += kW) {
        const double wi = P.w[i];
        const bool fx = P.mask && P.mask[i];
#pragma unroll
        for (int c = 0; c < R; ++c) {
          if (done[c]) continue;
          const int64_t o = i * R + c;
          if constexpr (MIXED) {
            const float pn = float(wi * P.r[o] + beta[c] * double(P.p32[o]));
            P.p32[o] = pn;
            if (fx) {
              P.q32[o] = pn;  // Dirichlet rows of A p: the entry itself
              v_mp[c] += double(pn) * double(pn);
            }
          } else {
            const double pn = wi * P.r[o] + beta[c] * P.p[o];
            P.p[o] = pn;
            if (fx) {
              P.q[o] = pn;  // Dirichlet rows of A p: the entry itself
              v_mp[c] += pn * pn;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double m = wave_sum64(v_mp[c]);
        if (lane == 0) part(kMp2, c)[me] = m;
      }
    }
    // shared nodes of q start the next P1 at zero (their values were last read in P2)
    for (int64_t j = j0 + lane; j < j1; j += kW) {
      const int64_t g = P.reset[j];
      if (P.mask && P.mask[g]) continue;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (done[c]) continue;
        if constexpr (MIXED)
          P.q32[g * R + c] = 0.0f;
        else
          P.q[g * R + c] = 0.0;
      }
    }
    if (!problem_barrier(P.bar, nwg, error)) return;
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
  if (i < n) d[i] = 1.0 / d[i];
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}

template <int R, bool MIXED>
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
      reinterpret_cast<const void *>(k_batched_pcg<R, MIXED>), dim3(unsigned(wg_prob.size())),
      dim3(kW), args, unsigned(lds), s);
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(dp);
  (void)hipFree(dwg);
  if (e != hipSuccess) return fail(Q1_EHIP, "cooperative launch failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(Q1_EHIP, "batched PCG: %s", hipGetErrorString(e2));
  return Q1_OK;
}

template <int R, bool MIXED>
int max_coresident(size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(k_batched_pcg<R, MIXED>), kW, lds) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

template <bool MIXED>
int coresident_for(int nrhs, size_t lds) {
  switch (nrhs) {
    case 1: return max_coresident<1, MIXED>(lds);
    case 2: return max_coresident<2, MIXED>(lds);
    case 3: return max_coresident<3, MIXED>(lds);
    default: return max_coresident<4, MIXED>(lds);
  }
}

template <bool MIXED>
int run_for(int nrhs, const std::vector<BProb> &hp, const std::vector<int> &wg_prob, double tol2,
            int maxit, double delta2, size_t lds, hipStream_t s, int *d_error) {
  switch (nrhs) {
    case 1: return run_batched<1, MIXED>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    case 2: return run_batched<2, MIXED>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    case 3: return run_batched<3, MIXED>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
    default: return run_batched<4, MIXED>(hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
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
  const size_t lds = size_t(max_nodes) * (size_t(nrhs) * sizeof(double) + sizeof(uint32_t));
  const int cap = mixed ? coresident_for<true>(nrhs, lds) : coresident_for<false>(nrhs, lds);
  Q1_CHECK(cap >= nprob, Q1_EUNSUPPORTED, "%s: %d problems need %d co-resident waves", name,
           nprob, nprob);
  // waves per problem in proportion to its elements, at least one each
  std::vector<int> nwg(nprob, 1);
  int spare = cap - nprob;
  for (int p = 0; p < nprob; ++p) {
    const Op *o = reinterpret_cast<const Op *>(ops[p]);
    const int extra = int(double(spare) * double(o->n_elems) / double(std::max<int64_t>(1, total_elems)));
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
    const size_t nv = size_t(n) * nrhs;
    double *vec[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int v = 0; v < 5; ++v) {
      if (mixed && v >= 3) continue;  // p, q are FP32 in the mixed form
      if ((rc = dalloc(reinterpret_cast<void **>(&vec[v]), nv * sizeof(double)))) return rc;
    }
    B.b = vec[0]; B.x = vec[1]; B.r = vec[2]; B.p = vec[3]; B.q = vec[4];
    if (mixed) {
      // FP32 copies of the geometry and of the lane-ordered coefficients: the FP32 operator
      float *xyz32 = nullptr, *coef32 = nullptr;
      const int64_t ncoef = tm.n_steps * kW;
      if ((rc = dalloc(reinterpret_cast<void **>(&B.p32), nv * sizeof(float))) ||
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
    if ((rc = dalloc(reinterpret_cast<void **>(&B.bar), 2 * sizeof(unsigned)))) return rc;
    Q1_HIP(hipMemsetAsync(B.bar, 0, 2 * sizeof(unsigned), s));
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
  rc = mixed ? run_for<true>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s, d_error)
             : run_for<false>(nrhs, hp, wg_prob, tol2, maxit, delta2, lds, s, d_error);
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
