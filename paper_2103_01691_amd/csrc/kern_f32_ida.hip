// Kernel instances of the mu-mode product for precision KP_F32 with the
// identity add (operators prepared as L - I).
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_f32_ida(int cplx, int ld, int pro, int epi, int cls, int full) {
  return pick_kernel<KP_F32, true>(cplx, ld, pro, epi, cls, full);
}
BatchFn pick_batch_merged_f32_ida() { return pick_batch_merged<KP_F32, true>(); }
}  // namespace mm
