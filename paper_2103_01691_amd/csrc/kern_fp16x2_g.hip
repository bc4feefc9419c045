// Three-product (Gauss) instances of the complex split products, precision
// KP_FP16X2.
#include "mode_tile.h"
#include "mode_gauss.h"

namespace mm {
KernFn pick_gauss_fp16x2(int ld, int pro, int epi, int cls, int full) {
  return gauss_pick<KP_FP16X2>(ld, pro, epi, cls, full);
}
bool gauss_shape_fp16x2(int cls, TileShape* out) { return gauss_shape<KP_FP16X2>(cls, out); }
}  // namespace mm
