// Three-product (Gauss) instances of the complex split products, precision
// KP_BF16X3.
#include "mode_tile.h"
#include "mode_gauss.h"

namespace mm {
KernFn pick_gauss_bf16x3(int ld, int pro, int epi, int cls, int full) {
  return gauss_pick<KP_BF16X3>(ld, pro, epi, cls, full);
}
bool gauss_shape_bf16x3(int cls, TileShape* out) { return gauss_shape<KP_BF16X3>(cls, out); }
}  // namespace mm
