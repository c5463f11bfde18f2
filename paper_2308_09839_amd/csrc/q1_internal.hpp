// Internal declarations of libq1mf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "q1mf.h"

namespace q1 {

// Thread-local error text behind q1_last_error().
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define Q1_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::q1::fail(Q1_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                          \
  } while (0)

#define Q1_CHECK(cond, code, ...)                          \
  do {                                                     \
    if (!(cond)) return ::q1::fail((code), __VA_ARGS__);   \
  } while (0)

// Per-tile data of the LDS-tiled apply (built once at operator creation).
struct TileMap {
  int n_tiles = 0;
  int max_nodes = 0;     // largest node count of a tile (LDS sizing)
  int tile_elems = 0;    // elements per tile (threads per workgroup)
  int32_t *node_ptr = nullptr;   // [n_tiles+1] offsets into nodes
  int32_t *nodes = nullptr;      // tile node lists (global node ids); sign bit set = shared node
  int32_t *elem = nullptr;       // [n_tiles*tile_elems] global element id or -1
  uint16_t *lconn = nullptr;     // [8][n_tiles*tile_elems] tile-local node index
  int64_t n_shared = 0;          // number of distinct shared nodes
  int32_t *shared = nullptr;     // [n_shared] shared global node ids (zeroed before apply)
  size_t bytes = 0;
};

struct Op {
  int physics = 1;  // DOF per node
  int dtype = Q1_F64;
  int variant = Q1_V_ATOMIC;
  int64_t n_nodes = 0, n_elems = 0;
  const void *xyz = nullptr;
  const int32_t *conn = nullptr;
  const void *coef = nullptr;
  const uint8_t *mask = nullptr;
  int device = 0;
  int num_cus = 256;
  TileMap tiles;
};

inline int xcd_count() { return 8; }

// launchers (defined in the .hip files)
int launch_apply(Op &op, const void *x, void *y, hipStream_t s);
int launch_diag(Op &op, void *d, hipStream_t s);
int build_tiles(Op &op, hipStream_t s);
void free_tiles(Op &op);

}  // namespace q1
