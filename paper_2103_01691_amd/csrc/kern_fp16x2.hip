// Kernel instances of the mu-mode product for precision KP_FP16X2.
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_fp16x2_ida(int cplx, int ld, int pro, int epi, int cls, int full);
KernFn pick_kernel_fp16x2(int cplx, int ld, int pro, int epi, int cls, int full, int ida) {
  if (is_gauss_class(cls)) return (cplx && !ida) ? pick_gauss_fp16x2(ld, pro, epi, cls, full) : nullptr;
  if (ida) return pick_kernel_fp16x2_ida(cplx, ld, pro, epi, cls, full);
  return pick_kernel<KP_FP16X2, false>(cplx, ld, pro, epi, cls, full);
}
bool batch_kind_fp16x2(int cplx, int ld, int cls) { return batch_kind<KP_FP16X2>(cplx, ld, cls); }
bool tile_shape_fp16x2(int cls, TileShape* out) {
  return is_gauss_class(cls) ? gauss_shape_fp16x2(cls, out) : shape_table<KP_FP16X2>(cls, out);
}
}  // namespace mm
