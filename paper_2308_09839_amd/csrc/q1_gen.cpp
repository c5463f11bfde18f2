// Host generators of the synthetic workloads and the error/version plumbing.
//
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based generator:
// draw(seed, stream, i) = mix(key + i + golden), key = seed ^ stream*golden.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "q1_internal.hpp"

namespace q1 {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z += kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t key_of(uint64_t seed, uint64_t stream) { return seed ^ (stream * kGolden); }

inline double unif(uint64_t key, uint64_t i) {
  return static_cast<double>(mix64(key + i) >> 11) * 0x1.0p-53;
}

inline double gauss(uint64_t key, uint64_t i) {
  const double u1 = unif(key, 2 * i), u2 = unif(key, 2 * i + 1);
  return std::sqrt(-2.0 * std::log(1.0 - u1)) * std::cos(2.0 * M_PI * u2);
}

}  // namespace
}  // namespace q1

using namespace q1;

extern "C" {

const char *q1_last_error(void) { return g_err; }

int q1_version(void) { return 100; }

int q1_box_sizes(int nx, int ny, int nz, int64_t *n_nodes, int64_t *n_elems) {
  Q1_CHECK(nx > 0 && ny > 0 && nz > 0, Q1_EINVAL, "box sizes must be positive (%d %d %d)", nx,
           ny, nz);
  const int64_t nn = int64_t(nx + 1) * (ny + 1) * (nz + 1);
  Q1_CHECK(nn < (int64_t(1) << 31), Q1_EINVAL, "box has %lld nodes, int32 ids overflow",
           (long long)nn);
  if (n_nodes) *n_nodes = nn;
  if (n_elems) *n_elems = int64_t(nx) * ny * nz;
  return Q1_OK;
}

int q1_box_mesh(int nx, int ny, int nz, double h, double jitter_frac, uint64_t seed,
                double *xyz, int32_t *conn) {
  int64_t nn, ne;
  int rc = q1_box_sizes(nx, ny, nz, &nn, &ne);
  if (rc) return rc;
  Q1_CHECK(xyz && conn, Q1_EINVAL, "q1_box_mesh: NULL output");
  Q1_CHECK(h > 0 && jitter_frac >= 0 && jitter_frac < 0.5, Q1_EINVAL,
           "q1_box_mesh: need h > 0 and 0 <= jitter_frac < 0.5");
  const uint64_t key = key_of(seed, 0);
  const double amp = jitter_frac * h;
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        const int64_t id = i + int64_t(nx + 1) * (j + int64_t(ny + 1) * k);
        double p[3] = {double(i) * h, double(j) * h, double(k) * h};
        const bool interior = i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz;
        if (interior && jitter_frac != 0.0)
          for (int c = 0; c < 3; ++c) {
            const double u = unif(key, uint64_t(3 * id + c));
            p[c] = p[c] + (2.0 * u - 1.0) * amp;
          }
        for (int c = 0; c < 3; ++c) xyz[c * nn + id] = p[c];
      }
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        const int64_t e = ex + int64_t(nx) * (ey + int64_t(ny) * ez);
        for (int a = 0; a < 8; ++a) {
          const int di = a & 1, dj = (a >> 1) & 1, dk = (a >> 2) & 1;
          conn[a * ne + e] =
              int32_t((ex + di) + int64_t(nx + 1) * ((ey + dj) + int64_t(ny + 1) * (ez + dk)));
        }
      }
  return Q1_OK;
}

int q1_face_mask(int nx, int ny, int nz, int face, uint8_t *mask) {
  int64_t nn;
  int rc = q1_box_sizes(nx, ny, nz, &nn, nullptr);
  if (rc) return rc;
  Q1_CHECK(mask && face >= 0 && face < 6, Q1_EINVAL, "q1_face_mask: bad face or NULL mask");
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        const int64_t id = i + int64_t(nx + 1) * (j + int64_t(ny + 1) * k);
        const bool on[6] = {i == 0, i == nx, j == 0, j == ny, k == 0, k == nz};
        mask[id] = on[face] ? 1 : 0;
      }
  return Q1_OK;
}

int q1_field_lognormal(int64_t n, double mu, double sigma, uint64_t seed, uint64_t stream,
                       double *out) {
  Q1_CHECK(n >= 0 && (out || n == 0), Q1_EINVAL, "q1_field_lognormal: bad arguments");
  const uint64_t key = key_of(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = std::exp(mu + sigma * gauss(key, uint64_t(i)));
  return Q1_OK;
}

int q1_field_layered(int nx, int ny, int nz, int layer_cells, double s_layer, double s_cell,
                     uint64_t seed, double *k) {
  int64_t ne;
  int rc = q1_box_sizes(nx, ny, nz, nullptr, &ne);
  if (rc) return rc;
  Q1_CHECK(k && layer_cells > 0, Q1_EINVAL, "q1_field_layered: bad arguments");
  const uint64_t k1 = key_of(seed, 1), k2 = key_of(seed, 2);
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t ez = e / (int64_t(nx) * ny);
    const double lay = std::exp(s_layer * gauss(k1, uint64_t(ez / layer_cells)));
    k[e] = lay * std::exp(s_cell * gauss(k2, uint64_t(e)));
  }
  return Q1_OK;
}

int q1_field_elastic(int64_t n, uint64_t seed, double *E, double *nu) {
  Q1_CHECK(n >= 0 && ((E && nu) || n == 0), Q1_EINVAL, "q1_field_elastic: bad arguments");
  const uint64_t k1 = key_of(seed, 1), k2 = key_of(seed, 2);
  for (int64_t i = 0; i < n; ++i) {
    E[i] = std::exp(std::log(10.0) + 1.0 * gauss(k1, uint64_t(i)));
    nu[i] = 0.15 + 0.2 * unif(k2, uint64_t(i));
  }
  return Q1_OK;
}

int q1_lame_from_E_nu(int64_t n, const double *E, const double *nu, double *lam, double *mu) {
  Q1_CHECK(n >= 0 && ((E && nu && lam && mu) || n == 0), Q1_EINVAL,
           "q1_lame_from_E_nu: bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    Q1_CHECK(nu[i] > -1.0 && nu[i] < 0.5 && E[i] > 0.0, Q1_EINVAL,
             "q1_lame_from_E_nu: need E > 0 and -1 < nu < 0.5 (cell %lld)", (long long)i);
    lam[i] = E[i] * nu[i] / ((1.0 + nu[i]) * (1.0 - 2.0 * nu[i]));
    mu[i] = E[i] / (2.0 * (1.0 + nu[i]));
  }
  return Q1_OK;
}

int q1_vec_uniform(int64_t n, uint64_t seed, uint64_t stream, double lo, double hi,
                   double *out) {
  Q1_CHECK(n >= 0 && (out || n == 0), Q1_EINVAL, "q1_vec_uniform: bad arguments");
  const uint64_t key = key_of(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = lo + (hi - lo) * unif(key, uint64_t(i));
  return Q1_OK;
}

/* Section 4 byte model (Tables 1-3). */
int q1_model_bytes(int kind, int physics, int real_bytes, int coef_bytes, int64_t n_nodes,
                   int64_t n_elems, int cache, double *bytes) {
  Q1_CHECK(bytes && physics >= 1 && physics <= 3 && (real_bytes == 4 || real_bytes == 8) &&
               n_nodes >= 0 && n_elems >= 0 && coef_bytes >= 0 && (cache == 0 || cache == 1),
           Q1_EINVAL, "q1_model_bytes: bad arguments");
  const double dpn = physics == 1 ? 1.0 : 3.0, R = real_bytes;
  const double ndof = double(n_nodes) * dpn;
  // nodal data read once (perfect cache) or once per element corner (no cache)
  const double node_reads = cache == 0 ? double(n_nodes) : 8.0 * double(n_elems);
  switch (kind) {
    case 0: {  // SpMV: 12 B per non-zero (8 B value + 4 B column), 2 vectors
      const double nnz = ndof * 27.0 * dpn;
      *bytes = nnz * (R + 4.0) + 2.0 * ndof * R;
      return Q1_OK;
    }
    case 1: {  // matrix-free: node map, cell constant, coordinates, 3 vector streams
      *bytes = double(n_elems) * (32.0 + coef_bytes) + node_reads * 3.0 * R +
               node_reads * 3.0 * dpn * R;
      return Q1_OK;
    }
    case 2: {  // partial assembly: node map, cell constant, 8 qp x (6 | 21) reals, vectors
      // (the Laplace kinds store the symmetric 3x3 geometric factor, elasticity 21 reals)
      const double per_qp = physics == 3 ? 21.0 : 6.0;
      *bytes = double(n_elems) * (32.0 + coef_bytes) + double(n_elems) * 8.0 * per_qp * R +
               node_reads * 3.0 * dpn * R;
      return Q1_OK;
    }
    default:
      return fail(Q1_EINVAL, "q1_model_bytes: unknown kind %d", kind);
  }
}

}  // extern "C"
