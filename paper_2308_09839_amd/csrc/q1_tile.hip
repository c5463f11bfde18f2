// LDS-tiled apply: set-up of the tile maps (placeholder until the tiled
// kernels land; creation with this variant reports it as unsupported).
#include "q1_internal.hpp"

namespace q1 {

int build_tiles(Op &op, hipStream_t) {
  (void)op;
  return fail(Q1_EUNSUPPORTED, "LDS-tile variant not built yet");
}

void free_tiles(Op &op) {
  TileMap &t = op.tiles;
  if (t.node_ptr) (void)hipFree(t.node_ptr);
  if (t.nodes) (void)hipFree(t.nodes);
  if (t.elem) (void)hipFree(t.elem);
  if (t.lconn) (void)hipFree(t.lconn);
  if (t.shared) (void)hipFree(t.shared);
  t = TileMap{};
}

}  // namespace q1
