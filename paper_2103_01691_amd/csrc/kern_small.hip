// Whole-run kernel for small states: one workgroup applies nsteps of the
// integrator T <- T x_1 E_1 ... x_d E_d, every mode product of every step,
// in a single launch.  The state is small enough to stay in the L2 of the
// CU's XCD between products, and the per-launch cost (a few microseconds per
// kernel) no longer multiplies with 2 x nsteps products.  Each product runs
// the same tile code as the one-product kernels (mode_tile), tile after
// tile, with a workgroup barrier between tiles and products (all waves of
// the workgroup share the CU's caches, so the barrier orders the global
// writes of one product before the reads of the next).
#include "mode_tile.h"

namespace mm {
namespace {

template <int PR, int CLS>
constexpr int small_threads() {
  return 64 * Cfg<PR, CLS>::WM * Cfg<PR, CLS>::WN;
}

template <int PR, bool CPLX, int CLS, int THREADS>
__global__ __launch_bounds__(THREADS) void small_run_kernel(SmallRun r) {
  typedef Cfg<PR, CLS> C;
  typedef typename Tr<PR>::pc pc;
  constexpr int CHUNK = C::KCH * C::WN * C::WNF * Tr<PR>::NPB * 64 * Tr<PR>::KPL;
  __shared__ __attribute__((aligned(16))) pc lds[2 * CHUNK];
  for (int s = 0; s < r.nsteps; ++s) {
    for (int k = 0; k < r.d; ++k) {
      if (!r.m[k].A) continue;
      for (int tx = 0; tx < r.tiles[k]; ++tx) {
        switch (r.load[k]) {
          case KL_KCONTIG:
            mode_tile<PR, CPLX, KL_KCONTIG, C::WMF, C::WNF, C::WM, C::WN, C::KCH, false, false, 1>(r.m[k], tx, 0, lds);
            break;
          case KL_FCONTIG:
            mode_tile<PR, CPLX, KL_FCONTIG, C::WMF, C::WNF, C::WM, C::WN, C::KCH, false, false, 1>(r.m[k], tx, 0, lds);
            break;
          default:
            mode_tile<PR, CPLX, KL_GENERIC, C::WMF, C::WNF, C::WM, C::WN, C::KCH, false, false, 1>(r.m[k], tx, 0, lds);
            break;
        }
        __syncthreads();
      }
    }
  }
}

}  // namespace

hipError_t launch_small_run(int prec, int cplx, const SmallRun& r, int* threads_out, hipStream_t s) {
  constexpr int CLS = SMALL_RUN_CLASS;
  int threads = 0;
  if (prec == KP_F64) {
    threads = small_threads<KP_F64, CLS>();
    if (cplx) hipLaunchKernelGGL((small_run_kernel<KP_F64, true, CLS, small_threads<KP_F64, CLS>()>), dim3(1), dim3(threads), 0, s, r);
    else hipLaunchKernelGGL((small_run_kernel<KP_F64, false, CLS, small_threads<KP_F64, CLS>()>), dim3(1), dim3(threads), 0, s, r);
  } else if (prec == KP_F32) {
    threads = small_threads<KP_F32, CLS>();
    if (cplx) hipLaunchKernelGGL((small_run_kernel<KP_F32, true, CLS, small_threads<KP_F32, CLS>()>), dim3(1), dim3(threads), 0, s, r);
    else hipLaunchKernelGGL((small_run_kernel<KP_F32, false, CLS, small_threads<KP_F32, CLS>()>), dim3(1), dim3(threads), 0, s, r);
  } else {
    return hipErrorInvalidValue;
  }
  if (threads_out) *threads_out = threads;
  return hipGetLastError();
}

}  // namespace mm
