// Kernel instances of the mu-mode product for precision KP_F64 with the
// identity add (operators prepared as L - I).
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_f64_ida(int cplx, int ld, int pro, int epi, int cls, int full) {
  return pick_kernel<KP_F64, true>(cplx, ld, pro, epi, cls, full);
}
BatchFn pick_batch_merged_f64_ida() { return pick_batch_merged<KP_F64, true>(); }
}  // namespace mm
