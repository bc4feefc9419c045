// Kernel instances of the mu-mode product for precision KP_F64.
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_f64_ida(int cplx, int ld, int pro, int epi, int cls, int full);
KernFn pick_kernel_f64(int cplx, int ld, int pro, int epi, int cls, int full, int ida) {
  if (ida) return pick_kernel_f64_ida(cplx, ld, pro, epi, cls, full);
  return pick_kernel<KP_F64, false>(cplx, ld, pro, epi, cls, full);
}
bool batch_kind_f64(int cplx, int ld, int cls) { return batch_kind<KP_F64>(cplx, ld, cls); }
bool tile_shape_f64(int cls, TileShape* out) { return shape_table<KP_F64>(cls, out); }
BatchFn pick_batch_merged_f64() { return pick_batch_merged<KP_F64, false>(); }
}  // namespace mm
