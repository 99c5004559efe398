// Tile-shape selection (placeholder table; replaced by the measured tuner).
#include <stdlib.h>

#include "bls_plan.h"

namespace bls {

TileChoice choose_tiles(bls_plan *p, const std::vector<CurveShape> &shapes, bool weighted) {
  (void)p;
  (void)shapes;
  TileChoice tc = default_tiles(weighted);
  if (const char *s = getenv("BLS_LDS_BUDGET")) tc.lds_budget = atoi(s);
  if (const char *s = getenv("BLS_TILE_CAP")) tc.tile_cap = atoi(s);
  if (const char *s = getenv("BLS_OCCUPANCY")) tc.occupancy = atoi(s);
  return tc;
}

}  // namespace bls
