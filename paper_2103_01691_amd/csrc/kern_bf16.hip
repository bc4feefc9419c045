// Kernel instances of the mu-mode product for precision KP_BF16.
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_bf16_ida(int cplx, int ld, int pro, int epi, int cls, int full);
KernFn pick_kernel_bf16(int cplx, int ld, int pro, int epi, int cls, int full, int ida) {
  if (ida) return pick_kernel_bf16_ida(cplx, ld, pro, epi, cls, full);
  return pick_kernel<KP_BF16, false>(cplx, ld, pro, epi, cls, full);
}
bool batch_kind_bf16(int cplx, int ld, int cls) { return batch_kind<KP_BF16>(cplx, ld, cls); }
bool tile_shape_bf16(int cls, TileShape* out) { return shape_table<KP_BF16>(cls, out); }
BatchFn pick_batch_merged_bf16() { return pick_batch_merged<KP_BF16, false>(); }
}  // namespace mm
