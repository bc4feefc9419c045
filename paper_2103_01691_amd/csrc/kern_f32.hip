// Kernel instances of the mu-mode product for precision KP_F32.
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_f32_ida(int cplx, int ld, int pro, int epi, int cls, int full);
KernFn pick_kernel_f32(int cplx, int ld, int pro, int epi, int cls, int full, int ida) {
  if (ida) return pick_kernel_f32_ida(cplx, ld, pro, epi, cls, full);
  return pick_kernel<KP_F32, false>(cplx, ld, pro, epi, cls, full);
}
bool batch_kind_f32(int cplx, int ld, int cls) { return batch_kind<KP_F32>(cplx, ld, cls); }
bool tile_shape_f32(int cls, TileShape* out) { return shape_table<KP_F32>(cls, out); }
BatchFn pick_batch_merged_f32() { return pick_batch_merged<KP_F32, false>(); }
}  // namespace mm
