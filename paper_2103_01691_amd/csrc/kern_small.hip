// Whole-run kernel for small states: one workgroup applies nsteps of the
// integrator T <- T x_1 E_1 ... x_d E_d, every mode product of every step,
// in a single launch.  The state is small enough to stay in the L2 of the
// CU's XCD between products, and the per-launch cost (a few microseconds per
// kernel) no longer multiplies with 2 x nsteps products.  Each product runs
// the same tile code as the one-product kernels (mode_tile), tile after
// tile, with a workgroup barrier between tiles and products (all waves of
// the workgroup share the CU's caches, so the barrier orders the global
// writes of one product before the reads of the next).
#include <type_traits>

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

// Whole run of a small 2-D real FP64 integrator with the state and both
// operators resident in LDS for every step: U <- E1 U E2^T (mode-1 product
// E1 U, then mode-2 product U E2^T), nsteps times, in one workgroup, with
// one read of U and the operators from global memory at the start and one
// write of U at the end.  Modes up to 64 long, zero-padded to multiples of
// 16 (padded rows and columns stay zero: the operators' padding is zero).
// Leading dimension 65 in LDS spreads the 16 consecutive columns a
// fragment reads over distinct banks.  FP64 MFMA 16x16x4: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r holds
// D[l / 16 + 4 r][l % 16].  Sixteen waves (four per SIMD, so the LDS
// reads of some overlap the MFMAs of others) each own one of the (at most
// sixteen) 16 x 16 output tiles of a product; measured per step on the
// 64 x 64 heat problem: 9.4 us with four waves, 7.1 with eight, 5.1 with
// sixteen (the MFMA work alone is ~3.4 us on one CU).
constexpr int SL_N = 64;
constexpr int SL_LD = SL_N + 1;
constexpr int SL_WAVES = 16;                    // four per SIMD
constexpr int SL_TPW = 16 / SL_WAVES;           // output tiles per wave (at most)
constexpr int SL_THREADS = 64 * SL_WAVES;

__global__ __launch_bounds__(SL_THREADS) void small_lds_kernel(double* __restrict__ U, int n1, int n2,
                                                        const double* __restrict__ E1, const double* __restrict__ E2,
                                                        int nsteps) {
  __shared__ double sU[2][SL_N * SL_LD];
  __shared__ double sE[2][SL_N * SL_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int M1 = (n1 + 15) & ~15, M2 = (n2 + 15) & ~15;
  for (int e = tid; e < SL_N * SL_N; e += SL_THREADS) {
    const int i = e % SL_N, j = e / SL_N;
    sU[0][i + SL_LD * j] = (i < n1 && j < n2) ? U[i + (int64_t)n1 * j] : 0.0;
    sE[0][i + SL_LD * j] = (E1 && i < n1 && j < n1) ? E1[i + n1 * j] : 0.0;
    sE[1][i + SL_LD * j] = (E2 && i < n2 && j < n2) ? E2[i + n2 * j] : 0.0;
  }
  __syncthreads();
  const int ntc = M2 / 16;              // output tiles: (M1/16) x (M2/16)
  const int ntiles = (M1 / 16) * ntc;
  const int lr = lane % 16, lk = lane / 16;
  int cur = 0;
  // out[i, j] = sum_k A[i, k] B[k, j] with A at a[i + SL_LD k] and B at
  // b[k + SL_LD j] (mode 1: B = U) or b[j + SL_LD k] (mode 2: B = E2^T).
  // Per-lane offsets of the wave's tiles are formed once; tiles beyond the
  // product's count are skipped by a wave-uniform test.
  int aoff[SL_TPW], b1off[SL_TPW], b2off[SL_TPW], ooff[SL_TPW];
  bool on[SL_TPW];
#pragma unroll
  for (int t = 0; t < SL_TPW; ++t) {
    const int tile = wave + SL_WAVES * t;
    on[t] = tile < ntiles;
    const int tr = on[t] ? tile / ntc : 0, tc = on[t] ? tile % ntc : 0;
    aoff[t] = (tr * 16 + lr) + SL_LD * lk;
    b1off[t] = lk + SL_LD * (tc * 16 + lr);           // B[k][j] = U[k, j]
    b2off[t] = (tc * 16 + lr) + SL_LD * lk;           // B[k][j] = E2[j, k]
    ooff[t] = (tr * 16 + lk) + SL_LD * (tc * 16 + lr);
  }
  auto product = [&](const double* a, const double* b, auto mode2, int K, double* o) {
    constexpr bool M2B = decltype(mode2)::value;
    f64x4 acc[SL_TPW];
#pragma unroll
    for (int t = 0; t < SL_TPW; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k4 = 0; k4 < K / 4; ++k4) {
#pragma unroll
      for (int t = 0; t < SL_TPW; ++t) {
        if (on[t]) {
          const double av = a[aoff[t] + 4 * SL_LD * k4];
          const double bv = M2B ? b[b2off[t] + 4 * SL_LD * k4] : b[b1off[t] + 4 * k4];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < SL_TPW; ++t)
      if (on[t]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) o[ooff[t] + 4 * r] = acc[t][r];
      }
  };
  for (int s = 0; s < nsteps; ++s) {
    if (E1) {
      product(sE[0], sU[cur], std::integral_constant<bool, false>{}, M1, sU[cur ^ 1]);
      cur ^= 1;
      __syncthreads();
    }
    if (E2) {
      product(sU[cur], sE[1], std::integral_constant<bool, true>{}, M2, sU[cur ^ 1]);
      cur ^= 1;
      __syncthreads();
    }
  }
  for (int e = tid; e < n1 * n2; e += SL_THREADS) {
    const int i = e % n1, j = e / n1;
    U[i + (int64_t)n1 * j] = sU[cur][i + SL_LD * j];
  }
}

}  // namespace

hipError_t launch_small_lds(double* U, int n1, int n2, const double* E1, const double* E2, int nsteps,
                            hipStream_t s) {
  if (n1 < 1 || n2 < 1 || n1 > SL_N || n2 > SL_N || nsteps < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(small_lds_kernel, dim3(1), dim3(SL_THREADS), 0, s, U, n1, n2, E1, E2, nsteps);
  return hipGetLastError();
}

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
