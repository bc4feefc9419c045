// Operator preparation, FP64 reductions and the host-side planning and
// dispatch of the mu-mode product kernels (tables in kern_<prec>.hip).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>

#include "mode_tile.h"

namespace mm {
namespace {

// -------------------------------------------------------- preparation -----

// The stored pieces of one operator value x at out[base] (piece p at
// base + p * 64 * KPL).
template <int PR>
__device__ __forceinline__ void put_pieces(typename Tr<PR>::pc* __restrict__ out, int64_t base, double x,
                                           int a_exp) {
  constexpr int KPL = Tr<PR>::KPL, NPC = Tr<PR>::NPS;
  if constexpr (PR == KP_F64) {
    out[base] = x;
  } else if constexpr (PR == KP_F32) {
    out[base] = (float)x;
  } else if constexpr (PR == KP_FP16X2) {
    // stored pieces (h 2^11, l) of x 2^-a_exp = h + 2^-11 l; the residual
    // is exact in FP64.  h 2^11 multiplies both state pieces, l the high
    // one.
    const double xs = ldexp(x, -a_exp);
    const _Float16 h = (_Float16)(float)xs;
    const _Float16 l = (_Float16)(float)((xs - (double)h) * 2048.0);
    out[base] = (_Float16)((float)h * 2048.0f);
    out[base + (int64_t)64 * KPL] = l;
  } else {
    double r = x;
#pragma unroll
    for (int p = 0; p < NPC; ++p) {
      __bf16 h = (__bf16)(float)r;
      out[base + (int64_t)p * 64 * KPL] = h;
      r = r - (double)(float)h;
    }
  }
}

// One fragment slot s = (kb, mf, lane) of the prepared operator.
template <int PR>
__device__ __forceinline__ void prepare_slot(int64_t s, const double* __restrict__ master, int64_t rows,
                                             int64_t cols, int64_t ld, int cplx, const PhaseScale& ph,
                                             void* __restrict__ outv, int KBT, int MFT, int a_exp) {
  typedef Tr<PR> T;
  typedef typename T::pc pc;
  constexpr int MB = T::MB, KB = T::KB, KPL = T::KPL, NPC = T::NPS;
  const int64_t slots = (int64_t)KBT * MFT * 64;   // (kb, mf, lane)
  if (s >= slots) return;
  const int lane = (int)(s % 64);
  const int64_t t = s / 64;
  const int mf = (int)(t % MFT);
  const int kb = (int)(t / MFT);
  const int64_t Mr = cplx ? 2 * rows : rows;
  const int64_t Kr = cplx ? 2 * cols : cols;
  pc* out = (pc*)outv;
  // physical fragment row -> logical row of the real block operator; the
  // FP64 16x16 accumulator layout puts row lane/16 + 4r in register r, so
  // its complex rows are permuted to keep (re, im) pairs in one lane
  const int rho = lane % MB;
  const int row = (PR == KP_F64 && cplx) ? 2 * (mf * 8 + (rho % 4) + 4 * (rho / 8)) + ((rho / 4) % 2)
                                         : mf * MB + rho;
  for (int e = 0; e < KPL; ++e) {
    const int kap = kb * KB + KPL * (lane / MB) + e;
    double x = 0.0;
    if (row < Mr && kap < Kr) {
      if (cplx) {
        const int64_t i = row / 2, j = kap / 2;
        const int cr = row & 1, ck = kap & 1;
        double re = master[2 * (i + j * ld)], im = master[2 * (i + j * ld) + 1];
        // L'[i,j] = exp(-i rc rx2[i]) L[i,j] exp(-i cc cx2[j])
        double th = 0.0;
        if (ph.rx2) th += ph.rc * ph.rx2[i];
        if (ph.cx2) th += ph.cc * ph.cx2[j];
        if (th != 0.0) {
          double sn, cs;
          sincos(th, &sn, &cs);
          const double r2 = re * cs + im * sn;
          im = im * cs - re * sn;
          re = r2;
        }
        x = (cr == ck) ? re : (cr == 0 ? -im : im);
      } else {
        x = master[row + kap * ld];
      }
    }
    const int64_t base = (((int64_t)kb * MFT + mf) * NPC) * 64 * KPL + lane * KPL + e;
    put_pieces<PR>(out, base, x, a_exp);
  }
}

// Three-product (Gauss) preparation: slot ((jb * 3 + t) * MFT + mf, lane)
// holds 8 columns of complex row mf * 32 + lane % 32 of Re L (t = 0), Im L
// (t = 1) or Re L + Im L (t = 2), formed in FP64.
template <int PR>
__global__ void prepare_gauss_kernel(const double* __restrict__ master, int64_t rows, int64_t cols, int64_t ld,
                                     void* __restrict__ outv, int JBT, int MFT, int a_exp) {
  typedef typename Tr<PR>::pc pc;
  constexpr int NPC = Tr<PR>::NPS;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)JBT * 3 * MFT * 64) return;
  const int lane = (int)(s % 64);
  const int64_t t = s / 64;
  const int mf = (int)(t % MFT);
  const int64_t kbg = t / MFT;
  const int ty = (int)(kbg % 3);
  const int64_t jb = kbg / 3;
  const int64_t i = (int64_t)mf * 32 + lane % 32;
  pc* out = (pc*)outv;
  for (int e = 0; e < 8; ++e) {
    const int64_t j = jb * 16 + 8 * (lane / 32) + e;
    double x = 0.0;
    if (i < rows && j < cols) {
      const double re = master[2 * (i + j * ld)], im = master[2 * (i + j * ld) + 1];
      x = ty == 0 ? re : (ty == 1 ? im : re + im);
    }
    put_pieces<PR>(out, ((kbg * MFT + mf) * NPC) * 64 * 8 + lane * 8 + e, x, a_exp);
  }
}

template <int PR>
__global__ void prepare_kernel(const double* __restrict__ master, int64_t rows, int64_t cols,
                               int64_t ld, int cplx, PhaseScale ph, void* __restrict__ outv, int KBT,
                               int MFT, int a_exp) {
  prepare_slot<PR>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, master, rows, cols, ld, cplx, ph, outv, KBT,
                   MFT, a_exp);
}

// Several operators of one precision in one launch (blockIdx.y selects the
// operator): the per-step operators of a time-dependent splitting step.
template <int PR>
__global__ void prepare_multi_kernel(PrepJobs jobs) {
  const PrepJob& p = jobs.j[blockIdx.y];
  prepare_slot<PR>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, p.master, p.rows, p.cols, p.ld, p.cplx, p.ph,
                   p.out, p.KBT, p.MFT, p.a_exp);
}

// Per-step operators of the time-dependent harmonic-oscillator splitting
// (blockIdx.y = step * modes + entry).
template <int PR>
__global__ void prepare_steps_kernel(StepPrep p) {
  const int e = (int)(blockIdx.y % p.modes);
  const int st = (int)(blockIdx.y / p.modes);
  const StepPrepMode& m = p.m[e];
  const double t = p.t0 + st * p.tau;
  const double th = t + 0.5 * p.tau;
  PhaseScale ph;
  ph.rx2 = m.x2;
  ph.cx2 = m.x2;
  ph.cc = 0.5 * p.eps * (cos(t) - cos(th));           // first half step: columns
  ph.rc = 0.5 * p.eps * (cos(th) - cos(t + p.tau));   // second half step: rows
  prepare_slot<PR>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, m.master, m.n, m.n, m.n, 1, ph,
                   m.out + (size_t)st * m.stride, m.KBT, m.MFT, m.a_exp);
}

// ------------------------------------------------------------- norm2 ------

constexpr int NORM_BLOCKS = 1024;
constexpr int NORM_THREADS = 256;

template <typename S, int KIND>
__global__ __launch_bounds__(NORM_THREADS) void reduce_partial_kernel(const S* __restrict__ x,
                                                                      const S* __restrict__ y,
                                                                      int64_t count,
                                                                      double* __restrict__ partial) {
  __shared__ double red[NORM_THREADS];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * NORM_THREADS;
  int64_t start = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x;
  if constexpr (KIND == RED_SQ) {
    // 16-byte loads (the state is 16-byte aligned), then the scalar tail
    constexpr int VN = 16 / sizeof(S);
    typedef S vecS __attribute__((ext_vector_type(VN)));
    const int64_t countv = count / VN;
    const vecS* __restrict__ xv = (const vecS*)x;
    for (int64_t i = start; i < countv; i += stride) {
      const vecS v = xv[i];
#pragma unroll
      for (int e = 0; e < VN; ++e) acc += (double)v[e] * (double)v[e];
    }
    start += VN * countv;
  }
  for (int64_t i = start; i < count; i += stride) {
    if constexpr (KIND == RED_SQ) {
      const double v = (double)x[i];
      acc += v * v;
    } else if constexpr (KIND == RED_DOT_RE) {
      acc += (double)x[2 * i] * (double)y[2 * i] + (double)x[2 * i + 1] * (double)y[2 * i + 1];
    } else {
      const double a2 = (double)x[2 * i] * (double)x[2 * i] + (double)x[2 * i + 1] * (double)x[2 * i + 1];
      acc += a2 * a2;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NORM_THREADS) void norm_final_kernel(const double* __restrict__ partial,
                                                                  int nparts,
                                                                  double* __restrict__ result) {
  __shared__ double red[NORM_THREADS];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NORM_THREADS) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) result[0] = red[0];
}

// ------------------------------------------------------------ maxabs ------

// Bound of the state for the FP16X2 products: max |x_k| as float bits
// (non-negative floats order like their bit patterns; NaN bits order above
// every finite value).
__global__ __launch_bounds__(NORM_THREADS) void maxabs_partial_kernel(const float* __restrict__ x,
                                                                      int64_t count,
                                                                      uint32_t* __restrict__ partial) {
  __shared__ uint32_t red[NORM_THREADS];
  uint32_t m = 0;
  // 16-byte loads (the state is 16-byte aligned), four in flight per thread,
  // then the scalar tail
  const int64_t count4 = count / 4;
  const f32x4* __restrict__ x4 = (const f32x4*)x;
  const int64_t stride = (int64_t)gridDim.x * NORM_THREADS;
  int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x;
  for (; i + 3 * stride < count4; i += 4 * stride) {
    f32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = x4[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) m = max(m, __float_as_uint(fabsf(v[u][e])));
  }
  for (; i < count4; i += stride) {
    const f32x4 v = x4[i];
#pragma unroll
    for (int e = 0; e < 4; ++e) m = max(m, __float_as_uint(fabsf(v[e])));
  }
  for (int64_t t = 4 * count4 + (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; t < count; t += stride)
    m = max(m, __float_as_uint(fabsf(x[t])));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NORM_THREADS) void maxabs_final_kernel(const uint32_t* __restrict__ partial,
                                                                    int nparts, uint32_t* __restrict__ slots) {
  __shared__ uint32_t red[NORM_THREADS];
  uint32_t m = 0;
  for (int i = threadIdx.x; i < nparts; i += NORM_THREADS) m = max(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  // slot 0 gets the bound (word 0; its other words and slots 1, 2 cleared)
  for (int i = threadIdx.x; i < 3 * SMAX_WORDS; i += NORM_THREADS) slots[i] = i == 0 ? red[0] : 0u;
}

// ------------------------------------------------------ device expm ------
// Helpers of the device matrix exponential (complex FP64, column-major,
// interleaved (re, im), n x n, leading dimension n).

// X = f (A + g diag(d)) with complex f, g; d real (nullable)
__global__ void expm_generator_kernel(const double* __restrict__ A, int n, const double* __restrict__ d,
                                      double gr, double gi, double fr, double fi, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  double re = A[2 * e], im = A[2 * e + 1];
  if (d && i == j) {
    re += gr * d[i];
    im += gi * d[i];
  }
  X[2 * e] = fr * re - fi * im;
  X[2 * e + 1] = fr * im + fi * re;
}

// T = I + f W (f real); W == nullptr: T = I
__global__ void expm_horner_kernel(double* __restrict__ T, const double* __restrict__ W, int n, double f) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  const double one = i == j ? 1.0 : 0.0;
  T[2 * e] = one + (W ? f * W[2 * e] : 0.0);
  T[2 * e + 1] = W ? f * W[2 * e + 1] : 0.0;
}

// P = W + c0 I + c1 X + c2 X2 + c3 X3 (W nullable): one Paterson-Stockmeyer
// block of the Taylor polynomial
__global__ void expm_ps_kernel(double* __restrict__ P, const double* __restrict__ W, const double* __restrict__ X,
                               const double* __restrict__ X2, const double* __restrict__ X3, int n, double c0,
                               double c1, double c2, double c3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t k = 2 * e + c;
    double v = (W ? W[k] : 0.0) + c1 * X[k] + c2 * X2[k] + c3 * X3[k];
    if (c == 0 && i == j) v += c0;
    P[k] = v;
  }
}

// per-column sum of |A_ij| (1-norm = max over columns)
__global__ void expm_colsum_kernel(const double* __restrict__ A, int n, const double* __restrict__ d, double gr,
                                   double gi, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const int64_t e = (int64_t)j * n + i;
    double re = A[2 * e], im = A[2 * e + 1];
    if (d && i == j) {
      re += gr * d[i];
      im += gi * d[i];
    }
    s += sqrt(re * re + im * im);
  }
  out[j] = s;
}

// Collapsed exact harmonic-oscillator propagator in nodal Hermite space:
// out[i, l] = sum_k Psi[i, k] exp(-i tau (k + 1/2)) Phi[k, l] (complex FP64,
// column-major interleaved, m x m); Phi is K x m, Psi m x K, real, ld = rows.
// One thread per entry; the phase of coefficient k is that mode's exact
// flow under the oscillator (phi_k has energy k + 1/2).
__global__ void hermite_collapse_kernel(const double* __restrict__ Phi, const double* __restrict__ Psi, int m,
                                        int K, double tau, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e % m);
  const int l = (int)(e / m);
  double re = 0.0, im = 0.0;
  for (int k = 0; k < K; ++k) {
    double sn, cs;
    sincos(tau * (k + 0.5), &sn, &cs);
    const double v = Psi[i + (int64_t)k * m] * Phi[k + (int64_t)l * K];
    re += v * cs;
    im -= v * sn;
  }
  out[2 * e] = re;
  out[2 * e + 1] = im;
}

// Exact flow over time s of the nonlinear part of the Section 4.5 vortex
// problem in the symmetrised variable v = W^(1/2) u:
// v <- exp((i s / 2)(1 - W^-1 |v|^2)) v, W^-1 the product over the modes of
// the inverse dual-cell widths winv[k * 4096 + i_k].  |v| is constant along
// the flow.  One thread per entry (grid-stride); FP32 states take the angle
// and its sine / cosine in FP32 (the library's own reduction and series),
// FP64 states in FP64.
struct Dims6 {
  int64_t n[6];
};
template <typename T>
__global__ __launch_bounds__(256) void vortex_phase_kernel(T* __restrict__ v, int64_t count, int d, Dims6 dims,
                                                           const double* __restrict__ winv, double s) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    double wi = 1.0;
    for (int k = 0; k < d; ++k) {
      const int64_t i = r % dims.n[k];
      r /= dims.n[k];
      wi *= winv[(int64_t)k * 4096 + i];
    }
    T re = v[2 * e], im = v[2 * e + 1];
    const T th = (T)(0.5 * s) * ((T)1 - (T)wi * (re * re + im * im));
    T sn, cs;
    if constexpr (sizeof(T) == 8) sincos(th, &sn, &cs);
    else sincos_f32<false>(th, &sn, &cs);
    v[2 * e] = re * cs - im * sn;
    v[2 * e + 1] = im * cs + re * sn;
  }
}

// ---------------------------------------------------------- host side -----

KernFn pick_kernel_any(int prec, int cplx, int ld, int pro, int epi, int cls, int full = 0, int ida = 0) {
  switch (prec) {
    case KP_F64: return pick_kernel_f64(cplx, ld, pro, epi, cls, full, ida);
    case KP_F32: return pick_kernel_f32(cplx, ld, pro, epi, cls, full, ida);
    case KP_BF16X3: return pick_kernel_bf16x3(cplx, ld, pro, epi, cls, full, ida);
    case KP_FP16X2: return pick_kernel_fp16x2(cplx, ld, pro, epi, cls, full, ida);
    default: return pick_kernel_bf16(cplx, ld, pro, epi, cls, full, ida);
  }
}

bool batch_kind_any(int prec, int cplx, int ld, int cls) {
  switch (prec) {
    case KP_F64: return batch_kind_f64(cplx, ld, cls);
    case KP_F32: return batch_kind_f32(cplx, ld, cls);
    case KP_BF16X3: return batch_kind_bf16x3(cplx, ld, cls);
    case KP_FP16X2: return batch_kind_fp16x2(cplx, ld, cls);
    default: return batch_kind_bf16(cplx, ld, cls);
  }
}

}  // namespace

bool tile_shape(int prec, int cls, TileShape* out) {
  switch (prec) {
    case KP_F64: return tile_shape_f64(cls, out);
    case KP_F32: return tile_shape_f32(cls, out);
    case KP_BF16X3: return tile_shape_bf16x3(cls, out);
    case KP_FP16X2: return tile_shape_fp16x2(cls, out);
    default: return tile_shape_bf16(cls, out);
  }
}

FragGeom frag_geom(int prec) {
  switch (prec) {
    case KP_F64: return {16, 16, 4, 1, 1, 8, 32};
    case KP_F32: return {32, 32, 2, 1, 1, 32, 16};
    case KP_BF16X3: return {32, 32, 16, 8, 3, 4, 16};
    case KP_FP16X2: return {32, 32, 16, 8, 2, 4, 16};
    default: return {32, 32, 16, 8, 1, 4, 16};
  }
}

void op_blocks(int prec, int64_t Mr, int64_t Kr, int* KBT, int* MFT) {
  FragGeom g = frag_geom(prec);
  const int64_t kb = (Kr + g.KB - 1) / g.KB;
  const int64_t mf = (Mr + g.MB - 1) / g.MB;
  *KBT = (int)((kb + g.KPAD - 1) / g.KPAD * g.KPAD);
  *MFT = (int)((mf + g.MPAD - 1) / g.MPAD * g.MPAD);
}

size_t prepared_bytes(int prec, int KBT, int MFT) {
  FragGeom g = frag_geom(prec);
  size_t elems = (size_t)KBT * MFT * g.NPC * 64 * g.KPL;
  size_t es = prec == KP_F64 ? 8 : prec == KP_F32 ? 4 : 2;
  return elems * es;
}

int num_classes(int prec) {
  return (prec == KP_BF16X3 || prec == KP_FP16X2) ? 11 : (prec == KP_F64 ? 4 : 3);
}

void gauss_blocks(int64_t rows, int64_t cols, int* JBT, int* MFT) {
  *JBT = (int)(((cols + 15) / 16 + 3) / 4 * 4);
  *MFT = (int)(((rows + 31) / 32 + 7) / 8 * 8);
}

size_t gauss_prepared_bytes(int prec, int JBT, int MFT) {
  const int npc = prec == KP_BF16X3 ? 3 : 2;
  return (size_t)JBT * 3 * MFT * npc * 64 * 8 * 2;
}

hipError_t launch_prepare_gauss(int prec, const double* master, int64_t rows, int64_t cols, int64_t ld, void* out,
                                int JBT, int MFT, int a_exp, hipStream_t s) {
  const int64_t slots = (int64_t)JBT * 3 * MFT * 64;
  const dim3 grid((unsigned)((slots + 255) / 256));
  if (prec == KP_FP16X2)
    hipLaunchKernelGGL(prepare_gauss_kernel<KP_FP16X2>, grid, dim3(256), 0, s, master, rows, cols, ld, out, JBT, MFT,
                       a_exp);
  else if (prec == KP_BF16X3)
    hipLaunchKernelGGL(prepare_gauss_kernel<KP_BF16X3>, grid, dim3(256), 0, s, master, rows, cols, ld, out, JBT, MFT,
                       a_exp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

bool plan_mode(const ModeArgs& a, int prec, int cplx, bool want_pro, bool want_epi, bool fcontig_ok,
               bool kcontig_ok, ModePlan* plan, bool batch, int force_cls, bool gauss_ok) {
  FragGeom g = frag_geom(prec);
  // two interleaved real fibres (P == 2), 16-byte aligned runs of 8 rows
  const bool pair_ok = !kcontig_ok && !cplx && a.P == 2 && a.Kr % 8 == 0;
  const int load = kcontig_ok ? KL_KCONTIG : (pair_ok ? KL_PAIR : (fcontig_ok ? KL_FCONTIG : KL_GENERIC));
  const int pro = (want_pro && cplx) ? 1 : 0;
  const int epi = (want_epi && cplx) ? 1 : 0;
  TileShape t0;
  if (!tile_shape(prec, 0, &t0)) return false;
  int cls = 0;
  const int rw = t0.WMF * g.MB;                      // rows per wave
  const bool split = prec == KP_BF16X3 || prec == KP_FP16X2;
  TileShape tf;
  // three-product classes only where the caller has the operator's Gauss
  // preparation (complex operator and state, no batch, no identity split)
  if (is_gauss_class(force_cls) && !(gauss_ok && cplx && !batch && (load == KL_KCONTIG || load == KL_FCONTIG)))
    force_cls = -1;
  // the prepared operator's K-blocks must make whole LDS chunks of the class
  // (three-product classes: their own padding, a multiple of every chunk)
  int kbt = 0, mft = 0;
  op_blocks(prec, a.Mr, a.Kr, &kbt, &mft);
  if (force_cls >= 0 && tile_shape(prec, force_cls, &tf) && (is_gauss_class(force_cls) || kbt % tf.KCH == 0) &&
      (batch ? batch_kind_any(prec, cplx, load, force_cls)
             : pick_kernel_any(prec, cplx, load, pro, epi, force_cls) != nullptr)) {
    cls = force_cls;
  } else if (!batch && split && cplx && load != KL_GENERIC && a.Mr > 2 * rw) {
    cls = 4;   // 4 x 128 rows, 128 fibres, 2 K-blocks per chunk: fastest for 256-long complex modes
  } else if (!pro && !epi && load != KL_GENERIC) {
    if (a.Mr <= rw) cls = 2;
    else if (a.Mr <= 2 * rw) cls = 1;
  }
  TileShape t;
  if (!tile_shape(prec, cls, &t)) return false;
  plan->prec = prec;
  plan->cplx = cplx;
  plan->load = load;
  plan->pro = pro;
  plan->epi = epi;
  plan->cls = cls;
  plan->gauss = is_gauss_class(cls) ? 1 : 0;
  plan->nt = t.WN * t.WNF * g.NB;
  plan->threads = 64 * t.WM * t.WN;
  plan->mt_rows = t.WM * t.WMF * g.MB;
  plan->grid_x = (int)((a.F + plan->nt - 1) / plan->nt);
  const int mfr = (a.Mr + g.MB - 1) / g.MB;          // fragments holding real rows
  plan->grid_y = (mfr + t.WM * t.WMF - 1) / (t.WM * t.WMF);
  plan->covers_all_rows = plan->grid_y == 1;
  {
    const int64_t out_bytes = (int64_t)a.Mr * a.F * (prec == KP_F64 ? 8 : 4);
    plan->full = (a.F % plan->nt == 0 && a.Mr % plan->mt_rows == 0 && out_bytes < ((int64_t)1 << 32) &&
                  load != KL_GENERIC && (cls == 0 || cls >= 3))
                     ? 1
                     : 0;
  }
  if (batch) return plan->grid_x > 0 && batch_kind_any(prec, cplx, load, cls);
  return plan->grid_x > 0 && pick_kernel_any(prec, cplx, load, pro, epi, cls) != nullptr;
}

hipError_t launch_mode(const ModePlan& p, const ModeArgs& a, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  KernFn fn = pick_kernel_any(p.prec, p.cplx, p.load, p.pro, p.epi, p.cls, p.full, a.idadd ? 1 : 0);
  if (!fn) return hipErrorInvalidDeviceFunction;
  dim3 grid(p.grid_x, p.grid_y, 1);
  if (start || stop) {
    // events stamped by the kernel's own dispatch (no separate marker
    // packets between launches): the kernel's execution time
    hipExtLaunchKernelGGL(fn, grid, dim3(p.threads), 0, s, start, stop, 0, a);
  } else {
    hipLaunchKernelGGL(fn, grid, dim3(p.threads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_mode_batch_merged(int prec, int ida, const BatchItem* items, int count, hipStream_t s) {
  BatchFn fn = nullptr;
  switch (prec) {
    case KP_F64: fn = ida ? pick_batch_merged_f64_ida() : pick_batch_merged_f64(); break;
    case KP_F32: fn = ida ? pick_batch_merged_f32_ida() : pick_batch_merged_f32(); break;
    case KP_BF16X3: fn = ida ? pick_batch_merged_bf16x3_ida() : pick_batch_merged_bf16x3(); break;
    case KP_BF16: fn = ida ? pick_batch_merged_bf16_ida() : pick_batch_merged_bf16(); break;
    default: return hipErrorInvalidDeviceFunction;
  }
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fn, dim3(count), dim3(256), 0, s, items);
  return hipGetLastError();
}

hipError_t launch_prepare_multi(int prec, const PrepJobs& jobs, hipStream_t s) {
  if (jobs.n < 1 || jobs.n > MAX_PREP_JOBS) return hipErrorInvalidValue;
  int64_t slots = 0;
  for (int k = 0; k < jobs.n; ++k) slots = std::max(slots, (int64_t)jobs.j[k].KBT * jobs.j[k].MFT * 64);
  const int threads = 256;
  const dim3 grid((unsigned)((slots + threads - 1) / threads), (unsigned)jobs.n);
  switch (prec) {
    case KP_F64: hipLaunchKernelGGL(prepare_multi_kernel<KP_F64>, grid, dim3(threads), 0, s, jobs); break;
    case KP_F32: hipLaunchKernelGGL(prepare_multi_kernel<KP_F32>, grid, dim3(threads), 0, s, jobs); break;
    case KP_BF16X3: hipLaunchKernelGGL(prepare_multi_kernel<KP_BF16X3>, grid, dim3(threads), 0, s, jobs); break;
    case KP_FP16X2: hipLaunchKernelGGL(prepare_multi_kernel<KP_FP16X2>, grid, dim3(threads), 0, s, jobs); break;
    default: hipLaunchKernelGGL(prepare_multi_kernel<KP_BF16>, grid, dim3(threads), 0, s, jobs); break;
  }
  return hipGetLastError();
}

hipError_t launch_prepare_steps(int prec, const StepPrep& p, hipStream_t s) {
  if (p.modes < 1 || p.modes > MAX_STEP_MODES || p.steps < 1) return hipErrorInvalidValue;
  int64_t slots = 0;
  for (int k = 0; k < p.modes; ++k) slots = std::max(slots, (int64_t)p.m[k].KBT * p.m[k].MFT * 64);
  const dim3 grid((unsigned)((slots + 255) / 256), (unsigned)(p.modes * p.steps));
  switch (prec) {
    case KP_F64: hipLaunchKernelGGL(prepare_steps_kernel<KP_F64>, grid, dim3(256), 0, s, p); break;
    case KP_F32: hipLaunchKernelGGL(prepare_steps_kernel<KP_F32>, grid, dim3(256), 0, s, p); break;
    case KP_BF16X3: hipLaunchKernelGGL(prepare_steps_kernel<KP_BF16X3>, grid, dim3(256), 0, s, p); break;
    case KP_FP16X2: hipLaunchKernelGGL(prepare_steps_kernel<KP_FP16X2>, grid, dim3(256), 0, s, p); break;
    default: hipLaunchKernelGGL(prepare_steps_kernel<KP_BF16>, grid, dim3(256), 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_prepare(int prec, int cplx, const double* master, int64_t rows, int64_t cols,
                          int64_t ld, PhaseScale ph, void* out, int KBT, int MFT, hipStream_t s,
                          int a_exp) {
  const int64_t slots = (int64_t)KBT * MFT * 64;
  const int threads = 256;
  const int blocks = (int)((slots + threads - 1) / threads);
  switch (prec) {
    case KP_F64:
      hipLaunchKernelGGL(prepare_kernel<KP_F64>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, ph, out, KBT, MFT, a_exp);
      break;
    case KP_F32:
      hipLaunchKernelGGL(prepare_kernel<KP_F32>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, ph, out, KBT, MFT, a_exp);
      break;
    case KP_BF16X3:
      hipLaunchKernelGGL(prepare_kernel<KP_BF16X3>, dim3(blocks), dim3(threads), 0, s, master,
                         rows, cols, ld, cplx, ph, out, KBT, MFT, a_exp);
      break;
    case KP_FP16X2:
      hipLaunchKernelGGL(prepare_kernel<KP_FP16X2>, dim3(blocks), dim3(threads), 0, s, master,
                         rows, cols, ld, cplx, ph, out, KBT, MFT, a_exp);
      break;
    default:
      hipLaunchKernelGGL(prepare_kernel<KP_BF16>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, ph, out, KBT, MFT, a_exp);
      break;
  }
  return hipGetLastError();
}

int norm_partials() { return NORM_BLOCKS; }

hipError_t launch_expm_generator(const double* A, int n, const double* d, double gr, double gi, double fr, double fi,
                                 double* X, hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(expm_generator_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, n, d, gr, gi, fr,
                     fi, X);
  return hipGetLastError();
}

hipError_t launch_expm_horner(double* T, const double* W, int n, double f, hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(expm_horner_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, T, W, n, f);
  return hipGetLastError();
}

hipError_t launch_expm_ps(double* P, const double* W, const double* X, const double* X2, const double* X3, int n,
                          const double* c, hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(expm_ps_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, P, W, X, X2, X3, n, c[0],
                     c[1], c[2], c[3]);
  return hipGetLastError();
}

hipError_t launch_expm_colsum(const double* A, int n, const double* d, double gr, double gi, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(expm_colsum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, n, d, gr, gi, out);
  return hipGetLastError();
}

int fp16x2_op_exp(double amax) {
  if (!(amax > 0.0) || !std::isfinite(amax)) return 0;
  int e = 0;
  std::frexp(amax, &e);   // amax in [2^(e-1), 2^e)
  return e - 4;           // amax 2^-a_exp in [8, 16)
}

hipError_t launch_hermite_collapse(const double* Phi, const double* Psi, int m, int K, double tau, double* out,
                                  hipStream_t s) {
  const int64_t n = (int64_t)m * m;
  hipLaunchKernelGGL(hermite_collapse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Phi, Psi, m, K, tau,
                     out);
  return hipGetLastError();
}

hipError_t launch_vortex_phase(void* v, int is_f64, int d, const int64_t* dims, const double* winv, double s,
                               hipStream_t st) {
  Dims6 D;
  int64_t count = 1;
  for (int k = 0; k < 6; ++k) D.n[k] = k < d ? dims[k] : 1;
  for (int k = 0; k < d; ++k) count *= dims[k];
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
  if (is_f64)
    hipLaunchKernelGGL(vortex_phase_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (double*)v, count, d, D,
                       winv, s);
  else
    hipLaunchKernelGGL(vortex_phase_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (float*)v, count, d, D,
                       winv, s);
  return hipGetLastError();
}

hipError_t launch_maxabs(const float* x, int64_t count, uint32_t* partial, uint32_t* slots, hipStream_t s) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s, x, count, partial);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(NORM_THREADS), 0, s, partial, NORM_BLOCKS, slots);
  return hipGetLastError();
}

template <typename S>
void reduce_dispatch(int kind, const void* x, const void* y, int64_t count, double* partial, hipStream_t s) {
  const S* xs = (const S*)x;
  const S* ys = (const S*)y;
  switch (kind) {
    case RED_SQ:
      hipLaunchKernelGGL((reduce_partial_kernel<S, RED_SQ>), dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s, xs, ys,
                         count, partial);
      break;
    case RED_DOT_RE:
      hipLaunchKernelGGL((reduce_partial_kernel<S, RED_DOT_RE>), dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s, xs,
                         ys, count, partial);
      break;
    default:
      hipLaunchKernelGGL((reduce_partial_kernel<S, RED_ABS4>), dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s, xs,
                         ys, count, partial);
      break;
  }
}

hipError_t launch_reduce(int kind, const void* x, const void* y, int64_t count, int is_f64, double* partial,
                         double* result, hipStream_t s) {
  if (is_f64) reduce_dispatch<double>(kind, x, y, count, partial, s);
  else reduce_dispatch<float>(kind, x, y, count, partial, s);
  hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(NORM_THREADS), 0, s, partial, NORM_BLOCKS, result);
  return hipGetLastError();
}

}  // namespace mm
