// Kernel instances of the mu-mode product for precision KP_BF16X3.
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_bf16x3_ida(int cplx, int ld, int pro, int epi, int cls, int full);
KernFn pick_kernel_bf16x3(int cplx, int ld, int pro, int epi, int cls, int full, int ida) {
  if (is_gauss_class(cls)) return (cplx && !ida) ? pick_gauss_bf16x3(ld, pro, epi, cls, full) : nullptr;
  if (ida) return pick_kernel_bf16x3_ida(cplx, ld, pro, epi, cls, full);
  return pick_kernel<KP_BF16X3, false>(cplx, ld, pro, epi, cls, full);
}
bool batch_kind_bf16x3(int cplx, int ld, int cls) { return batch_kind<KP_BF16X3>(cplx, ld, cls); }
bool tile_shape_bf16x3(int cls, TileShape* out) {
  return is_gauss_class(cls) ? gauss_shape_bf16x3(cls, out) : shape_table<KP_BF16X3>(cls, out);
}
BatchFn pick_batch_merged_bf16x3() { return pick_batch_merged<KP_BF16X3, false>(); }
}  // namespace mm
