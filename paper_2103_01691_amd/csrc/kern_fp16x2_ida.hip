// Kernel instances of the mu-mode product for precision KP_FP16X2 with the
// identity add (operators prepared as L - I).
#include "mode_tile.h"

namespace mm {
KernFn pick_kernel_fp16x2_ida(int cplx, int ld, int pro, int epi, int cls, int full) {
  return pick_kernel<KP_FP16X2, true>(cplx, ld, pro, epi, cls, full);
}
}  // namespace mm
