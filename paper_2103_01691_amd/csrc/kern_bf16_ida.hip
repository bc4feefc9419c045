// Kernel instances of the mu-mode product for precision KP_BF16 with the
// identity add (operators prepared as L - I).
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_bf16_ida(int cplx, int ld, int pro, int epi, int cls, int full) {
  return pick_kernel<KP_BF16, true>(cplx, ld, pro, epi, cls, full);
}
BatchFn pick_batch_merged_bf16_ida() { return pick_batch_merged<KP_BF16, true>(); }
}  // namespace mm
