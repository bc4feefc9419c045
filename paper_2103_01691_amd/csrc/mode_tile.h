// mu-mode product kernels for gfx950 (CDNA4).
//
// One launch computes S = U x_mu L (Definition 2.1 of the paper) for a
// tensor viewed as [P, n, Q]: P = n_1 ... n_{mu-1} (contiguous), n = n_mu,
// Q = n_{mu+1} ... n_d.  Every fibre (p, q) is multiplied by L, so the
// product is a GEMM  S[:, f] = L U[:, f]  over the F = P*Q fibres, done on
// the un-permuted array (the paper's Section 5 argues against an explicit
// permute pass).
//
// Real-GEMM view.  A complex operator acting on a complex state is the real
// operator  Lr[2i+c', 2j+c]  =  Re L_ij (c = c'),  -Im L_ij (c' = 0, c = 1),
// Im L_ij (c' = 1, c = 0)  acting on the real fibre vector kappa = 2j + c.
// So every case is a real GEMM  C (Mr x F) = Lr (Mr x Kr) B (Kr x F).
//
// Work split.  A workgroup owns NT consecutive fibres and, in the usual
// case, all Mr output rows, so each fibre is read from HBM once and written
// once, and a product may run in place.  Its WAVES waves split the rows;
// each wave holds a WMF x WNF grid of MFMA accumulators.  The fibre tile is
// staged through LDS (double buffered, one K-chunk at a time) in the exact
// per-lane order the MFMA B operand wants; the split into bfloat16 pieces
// happens once per element at staging.  The operator, prepared once in
// fragment order, is streamed by each wave straight from L2 with one
// 16-byte load per lane per fragment.
//
// Precisions (MFMA on gfx950):
//   KP_F64     v_mfma_f64_16x16x4_f64
//   KP_F32     v_mfma_f32_32x32x2_f32
//   KP_BF16X3  v_mfma_f32_32x32x16_bf16, operands split x = x0 + x1 + x2 into
//              RNE bfloat16 pieces; the six products x_a y_b with a + b <= 2
//              are accumulated in FP32.
//   KP_FP16X2  v_mfma_f32_32x32x16_f16, two-piece half-precision split with
//              the low piece scaled by 2^11 (x = h + 2^-11 l).  With the
//              operator kept as three pieces (h_A 2^11, h_A, l_A) one FP32
//              accumulator collects  2^11 [A B - (A - h_A)(B - h_B)]  in
//              three products; the epilogue scales it back.  Half precision
//              has a narrow exponent range, so the state is scaled by a
//              power of two from a running bound of max |component| that
//              every launch passes to the next (smax slots), and the
//              operator by a fixed power of two chosen at preparation.
//   KP_BF16    same MFMA as BF16X3, one piece each (comparison only).
//
// Fused Gross-Pitaevskii phase.  The exact nonlinear subflow
// psi <- exp(-i s beta |psi|^2) psi (Section 4.5: the nonlinear part is
// integrated exactly) is applied to the loaded fibres (prologue) and/or to
// the results (epilogue), so no separate pass over the state is needed.

#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mm_internal.h"

namespace mm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ traits -----

template <int PR> struct Tr;
template <> struct Tr<KP_F64> {
  typedef double st;     // state scalar
  typedef double pc;     // operator / staged piece scalar
  typedef double afrag;  // per-lane fragment
  typedef f64x4 acc;
  static constexpr int MB = 16, NB = 16, KB = 4, KPL = 1, NPA = 1, NPS = 1, NPB = 1, NACC = 4;
};
template <> struct Tr<KP_F32> {
  typedef float st;
  typedef float pc;
  typedef float afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 2, KPL = 1, NPA = 1, NPS = 1, NPB = 1, NACC = 16;
};
template <> struct Tr<KP_BF16X3> {
  typedef float st;
  typedef __bf16 pc;
  typedef bf16x8 afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 16, KPL = 8, NPA = 3, NPS = 3, NPB = 3, NACC = 16;
};
template <> struct Tr<KP_FP16X2> {
  typedef float st;
  typedef _Float16 pc;
  typedef f16x8 afrag;
  typedef f32x16 acc;
  // operator pieces (h 2^11, l) as stored; state pieces (h, r) with r the
  // unscaled residual
  static constexpr int MB = 32, NB = 32, KB = 16, KPL = 8, NPA = 2, NPS = 2, NPB = 2, NACC = 16;
};
template <> struct Tr<KP_BF16> {
  typedef float st;
  typedef __bf16 pc;
  typedef bf16x8 afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 16, KPL = 8, NPA = 1, NPS = 1, NPB = 1, NACC = 16;
};

__device__ __forceinline__ void mfma(f64x4& c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma(f32x16& c, float a, float b) {
  c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma(f32x16& c, bf16x8 a, bf16x8 b) {
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma(f32x16& c, f16x8 a, f16x8 b) {
  c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Piece pairs (a, b) of the split product: operator piece a times state
// piece b, in issue order.
template <int PR> struct Prods {
  static constexpr int N = 1;
  __device__ static constexpr int a(int) { return 0; }
  __device__ static constexpr int b(int) { return 0; }
};
template <> struct Prods<KP_BF16X3> {
  // (0,0) (0,1) (1,0) (0,2) (1,1) (2,0): piece orders a + b <= 2
  static constexpr int N = 6;
  __device__ static constexpr int a(int k) { return k == 2 ? 1 : k == 4 ? 1 : k == 5 ? 2 : 0; }
  __device__ static constexpr int b(int k) { return k == 1 ? 1 : k == 3 ? 2 : k == 4 ? 1 : 0; }
};
template <> struct Prods<KP_FP16X2> {
  // (h_A 2^11) h_B + (h_A 2^11) r_B + l_A h_B, every term at scale 2^11
  static constexpr int N = 3;
  __device__ static constexpr int a(int k) { return k == 2 ? 1 : 0; }
  __device__ static constexpr int b(int k) { return k == 1 ? 1 : 0; }
};

// Split a float into NPC round-to-nearest-even bfloat16 pieces.  Each
// residual is exact in FP32 (the piece is the value rounded to 8 bits).
template <int NPC>
__device__ __forceinline__ void split_bf16(float x, __bf16* p) {
  __bf16 h0 = (__bf16)x;
  p[0] = h0;
  if constexpr (NPC > 1) {
    float r1 = x - (float)h0;
    __bf16 h1 = (__bf16)r1;
    p[1] = h1;
    if constexpr (NPC > 2) {
      float r2 = r1 - (float)h1;
      p[2] = (__bf16)r2;
    }
  }
}

// Split x 2^-e into two RNE half-precision pieces h + r.  The residual
// x 2^-e - h is exact in FP32 (h is the value rounded to 11 bits).  The
// state exponent puts max |x| 2^-e in [2^14, 2^15), so r is a normal half
// (11 significant bits) wherever |x| is above 2^-17 of the maximum, and
// below that its absolute error (at most 2^-25) is under 2^-39 of the
// maximum; the operator's high piece is stored times 2^11, so the product
// with r lands at the scale of the other two terms.
// Two values at a time, so that both roundings use one packed conversion.
__device__ __forceinline__ void split_f16x2(float x0, float x1, int e, _Float16* p0, _Float16* p1) {
  typedef _Float16 h2v __attribute__((ext_vector_type(2)));
  typedef float f2v __attribute__((ext_vector_type(2)));
  const float a = ldexpf(x0, -e), b = ldexpf(x1, -e);
  const h2v h = __builtin_convertvector(f2v{a, b}, h2v);
  const h2v r = __builtin_convertvector(f2v{a - (float)h.x, b - (float)h.y}, h2v);
  p0[0] = h.x;
  p1[0] = h.y;
  p0[1] = r.x;
  p1[1] = r.y;
}

// Exponent e with max * 2^-e < 2^15 for the float whose bits are `bits`
// (a non-negative bound of the state); 0 for a zero bound.
__device__ __forceinline__ int fp16x2_state_exp(uint32_t bits) {
  const int be = (int)((bits >> 23) & 0xff);
  if (be == 0) return 0;
  return min(be - 127, 127) - 14;
}

// sin and cos of an FP32 argument: Cody-Waite reduction by pi/2 with a
// three-term split of pi/2 (each term the FP32 rounding of what remains of
// the FP64 value), then the Taylor series of sin (to x^9) and cos (to x^10)
// on |r| <= pi/4, whose truncation errors (< 2e-9, < 2e-10) are below FP32
// rounding.  Accurate to a few ulp for |x| up to ~1e5; needs no scratch.
// The two series alone, for |x| <= pi/4.
__device__ __forceinline__ void sincos_small_f32(float x, float* s, float* c) {
  const float r2 = x * x;
  *s = x * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
  *c = 1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
}

template <bool VOTE = true>
__device__ __forceinline__ void sincos_f32(float x, float* s, float* c) {
  if (VOTE && __all(fabsf(x) <= 0.78539816f)) {
    // every active lane already in [-pi/4, pi/4]: no reduction needed
    sincos_small_f32(x, s, c);
    return;
  }
  constexpr double PIO2 = 1.57079632679489661923;
  constexpr float P1 = (float)PIO2;
  constexpr float P2 = (float)(PIO2 - (double)P1);
  constexpr float P3 = (float)(PIO2 - (double)P1 - (double)P2);
  const float q = rintf(x * (float)(1.0 / PIO2));
  float r = fmaf(-q, P1, x);
  r = fmaf(-q, P2, r);
  r = fmaf(-q, P3, r);
  const float r2 = r * r;
  const float sp = r * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
  const float cp = 1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
  const int qi = ((int)q) & 3;
  const float ss = (qi & 1) ? cp : sp;
  const float cc = (qi & 1) ? sp : cp;
  *s = (qi & 2) ? -ss : ss;
  *c = ((qi + 1) & 2) ? -cc : cc;
}

// exp(-i s |z|^2) z.  VOTE: take the reduction-free path when every active
// lane allows it (a wave-uniform branch); without it the code is branch-free
// and can be interleaved with MFMA work by the scheduler.  SMALL: the caller
// guarantees |s| |z|^2 <= pi/4 (FP32 only), so no reduction is compiled.
template <typename T, bool VOTE = true, bool SMALL = false>
__device__ __forceinline__ void phase(T& re, T& im, T s) {
  T th = s * (re * re + im * im);
  T sn, cs;
  if constexpr (sizeof(T) == 8) {
    sincos(th, &sn, &cs);
  } else if constexpr (SMALL) {
    sincos_small_f32(th, &sn, &cs);
  } else {
    sincos_f32<VOTE>(th, &sn, &cs);
  }
  T r = re * cs + im * sn;
  T i = im * cs - re * sn;
  re = r;
  im = i;
}

// Swizzle of the lane slot inside a (K-block, N-fragment) LDS block for
// KPL = 8: spreads the 16-byte writes of one fibre's successive K-groups over
// different banks.  Readers apply the same map.
__device__ __forceinline__ int swz(int n, int kb, int g) { return n ^ ((kb * 2 + g) & 7); }

// Fibre f (global) -> element offset (in scalars) of its entry j = 0.
__device__ __forceinline__ int64_t fibre_base(int64_t f, int64_t P, int n, int comps) {
  int64_t q = f / P;
  int64_t p = f - q * P;
  return (p + P * (int64_t)n * q) * comps;
}

// ------------------------------------------------------------- kernel -----

// One workgroup tile: fibres [tile_x * NT, tile_x * NT + NT), M-fragments of
// row block tile_y.  WM x WN waves: wave (wm, wn) owns M-fragments
// [(tile_y*WM + wm)*WMF, +WMF) and N-fragments [wn*WNF, +WNF) of the tile.
template <int PR, bool CPLX, int LD, int WMF, int WNF, int WM, int WN, int KCH, bool PRO, bool EPI, int OCC,
          bool FULL = false, bool IDA = false>
__device__ __forceinline__ void mode_tile(const ModeArgs& a, int64_t tile_x, int tile_y,
                                          typename Tr<PR>::pc* __restrict__ lds) {
  typedef Tr<PR> T;
  typedef typename T::st st;
  typedef typename T::pc pc;
  typedef typename T::afrag afrag;
  typedef typename T::acc acc_t;
  constexpr int MB = T::MB, NB = T::NB, KB = T::KB, KPL = T::KPL, NPA = T::NPA, NPS = T::NPS, NPB = T::NPB;
  constexpr bool F16 = PR == KP_FP16X2;
  constexpr int THREADS = 64 * WM * WN;
  constexpr int NT = WN * WNF * NB;      // fibres per workgroup
  constexpr int NFR = WN * WNF;          // N-fragments per workgroup
  constexpr int CK = KCH * KB;           // real K values per chunk
  constexpr int BLK = 64 * KPL;          // scalars per (kb, nf, piece) block
  constexpr int CHUNK = KCH * NFR * NPB * BLK;
  constexpr int COMPS = CPLX ? 2 : 1;
  typedef Prods<PR> PP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const int64_t f0 = tile_x * NT;
  const int mf0 = (tile_y * WM + wm) * WMF;   // first M-fragment of this wave
  const int nf0 = wn * WNF;                   // first N-fragment of this wave

  const st* __restrict__ in = (const st*)a.in;
  const st s_pre = (st)a.s_pre;

  // FP16X2: state scale from the running bound; the first workgroup clears
  // the slot the previous launch read (it is complete: same stream)
  int s_exp = 0;
  // FP16X2 with a prologue phase: the running bound b of every component
  // bounds the phase angle by |s_pre| 2 b^2; when that is within pi/4 (with
  // a margin for rounding) the staging compiles its sincos without range
  // reduction (the main loop exists in both forms, chosen once here).
  bool ph_small = false;
  if constexpr (F16) {
    uint32_t bbits = 0;
#pragma unroll
    for (int w = 0; w < SMAX_WORDS; ++w) bbits = max(bbits, a.smax_in[w]);
    s_exp = fp16x2_state_exp(bbits);
    if (tile_x == 0 && tile_y == 0 && tid < SMAX_WORDS) a.smax_clr[tid] = 0u;
    const float bnd = __uint_as_float(bbits);
    ph_small = fabsf((float)a.s_pre) * 2.0f * bnd * bnd <= 0.78f;
  }

  // ---------------------------------------------------------------- staging
  // Tile of TK real K values x TF fibres handled by one thread at a time.
  constexpr int VL = 16 / sizeof(st);    // scalars per 16-byte vector
  constexpr int TK = (KPL == 8) ? 8 : (LD == KL_KCONTIG ? VL : (LD == KL_PAIR ? VL / 2 : (CPLX ? 2 : 1)));
  constexpr int TF = (LD == KL_FCONTIG) ? (KPL == 8 ? (CPLX ? VL / 2 : VL) : (CPLX ? VL / 2 : VL))
                                        : (LD == KL_PAIR ? 2 : 1);
  static_assert(LD != KL_PAIR || !CPLX, "paired fibres are real");
  constexpr int TILES_K = CK / TK;
  constexpr int TILES_F = NT / TF;
  constexpr int TILES = TILES_K * TILES_F;
  static_assert(TILES % THREADS == 0 || TILES < THREADS, "tiles must split evenly");
  constexpr int TPT = (TILES + THREADS - 1) / THREADS;   // tiles per thread
  constexpr int VPT = TK * TF;           // scalars per tile
  st stage[TPT][VPT];

  auto tile_coords = [&](int t, int& tk, int& tf) {
    if constexpr (LD == KL_KCONTIG || LD == KL_PAIR) {
      tk = t % TILES_K;
      tf = t / TILES_K;
    } else {
      tf = t % TILES_F;
      tk = t / TILES_F;
    }
  };

  // Per-tile source pointers of chunk 0 and fibre validity, computed once:
  // chunk c of a tile starts CSTRIDE * c scalars further on.
  constexpr bool FAST = LD != KL_GENERIC;
  const st* tsrc[TPT];
  bool tok[TPT];
  int tkl[TPT];   // first local real K of the tile within a chunk
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    int tk, tf;
    tile_coords(tid + u * THREADS, tk, tf);
    const int64_t fg = f0 + (int64_t)tf * TF;
    tok[u] = (TILES >= THREADS || tid < TILES) && fg < a.F;
    tkl[u] = tk * TK;
    if constexpr (LD == KL_KCONTIG) {
      tsrc[u] = in + (tok[u] ? fg * (int64_t)a.Kr + tk * TK : 0);
    } else if constexpr (LD == KL_PAIR) {
      // fibres fg, fg + 1 (fg even) are entries 0 and 1 of the pair fg / 2,
      // whose row j sits at 2 (j + n (fg / 2)) and 2 (j + n (fg / 2)) + 1
      tsrc[u] = in + (tok[u] ? (fg / 2) * (int64_t)(2 * a.Kr) + tk * TK * 2 : 0);
    } else if constexpr (LD == KL_FCONTIG) {
      tsrc[u] = in + (tok[u] ? fibre_base(fg, a.P, a.n, COMPS) + (int64_t)(tk * TK / COMPS) * a.P * COMPS : 0);
    } else {
      tsrc[u] = in;
    }
  }
  const int64_t cstride = (LD == KL_KCONTIG) ? (int64_t)CK : (LD == KL_PAIR ? (int64_t)2 * CK : (int64_t)CK * a.P);

  // Load chunk `c` (real K values [c*CK, c*CK + CK)) into registers.
  auto load_chunk = [&](int c) {
    const int klim = a.Kr - c * CK;   // local K values of this chunk that exist
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      if (TILES < THREADS && tid >= TILES) break;
      st* v = stage[u];
      if constexpr (LD == KL_KCONTIG) {
        // P == 1: fibre's K values are contiguous; TK of them, vectorised.
        if (tok[u] && tkl[u] < klim) {
          const st* src = tsrc[u] + c * cstride;
#pragma unroll
          for (int w = 0; w < TK / VL; ++w) {
            if constexpr (sizeof(st) == 4) {
              f32x4 x = *(const f32x4*)(src + w * VL);
#pragma unroll
              for (int e = 0; e < 4; ++e) v[w * VL + e] = x[e];
            } else {
              f64x2 x = *(const f64x2*)(src + w * VL);
              v[w * VL + 0] = x[0];
              v[w * VL + 1] = x[1];
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < VPT; ++e) v[e] = (st)0;
        }
      } else if constexpr (LD == KL_PAIR) {
        // TK rows of a fibre pair: 2 TK contiguous scalars, row-major over
        // (row, fibre of the pair), which is already the v[row * TF + fibre]
        // order of the staging tile.
        if (tok[u] && tkl[u] < klim) {
          const st* src = tsrc[u] + c * cstride;
#pragma unroll
          for (int w = 0; w < 2 * TK / VL; ++w) {
            if constexpr (sizeof(st) == 4) {
              f32x4 x = *(const f32x4*)(src + w * VL);
#pragma unroll
              for (int e = 0; e < 4; ++e) v[w * VL + e] = x[e];
            } else {
              f64x2 x = *(const f64x2*)(src + w * VL);
              v[w * VL + 0] = x[0];
              v[w * VL + 1] = x[1];
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < VPT; ++e) v[e] = (st)0;
        }
      } else if constexpr (LD == KL_FCONTIG) {
        // Fibres contiguous: one 16-byte vector holds TF fibres at one row j.
        constexpr int ROWS = CPLX ? TK / 2 : TK;
        const st* src0 = tsrc[u] + c * cstride;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          st xv[VL];
          if (tok[u] && tkl[u] + r * COMPS < klim) {
            const st* src = src0 + (int64_t)r * a.P * COMPS;
            if constexpr (sizeof(st) == 4) {
              f32x4 x = *(const f32x4*)src;
#pragma unroll
              for (int e = 0; e < 4; ++e) xv[e] = x[e];
            } else {
              f64x2 x = *(const f64x2*)src;
              xv[0] = x[0];
              xv[1] = x[1];
            }
          } else {
#pragma unroll
            for (int e = 0; e < VL; ++e) xv[e] = (st)0;
          }
          // scatter into v[kappa_local * TF + fibre_local]
#pragma unroll
          for (int e = 0; e < VL; ++e) {
            const int fi = CPLX ? e / 2 : e;
            const int kl = CPLX ? 2 * r + (e & 1) : r;
            v[kl * TF + fi] = xv[e];
          }
        }
      } else {
        // Generic gather: one fibre, TK real K values, scalar / pair loads.
        int tk, tf;
        tile_coords(tid + u * THREADS, tk, tf);
        const int k0 = c * CK + tk * TK;
        const int64_t fg = f0 + (int64_t)tf * TF;
        const bool fok = fg < a.F;
        const int64_t base = fok ? fibre_base(fg, a.P, a.n, COMPS) : 0;
#pragma unroll
        for (int e = 0; e < TK; e += COMPS) {
          const int kk = k0 + e;
          const int j = CPLX ? kk / 2 : kk;
          if (fok && kk < a.Kr) {
            const st* src = in + base + (int64_t)j * a.P * COMPS;
            v[e] = src[0];
            if constexpr (CPLX) v[e + 1] = src[1];
          } else {
            v[e] = (st)0;
            if constexpr (CPLX) v[e + 1] = (st)0;
          }
        }
      }
    }
  };

  // Write the staged registers of tile u into LDS buffer `buf`, split into
  // pieces.
  auto store_tile = [&](int u, int buf, auto small) {
    constexpr bool SMALL = decltype(small)::value;
    pc* L = lds + buf * CHUNK;
    {
      if (TILES < THREADS && tid >= TILES) return;
      int tk, tf;
      tile_coords(tid + u * THREADS, tk, tf);
      const int kl0 = tk * TK;
      const int fl0 = tf * TF;
      st* v = stage[u];
      if constexpr (PRO && CPLX) {
        // prologue phase, applied as the tile is staged (not when it is
        // fetched, so the wave does not wait for the fetch early); entries
        // (kappa even, odd) of one fibre are (re, im) of one value
#pragma unroll
        for (int fi = 0; fi < TF; ++fi)
#pragma unroll
          for (int kl = 0; kl < TK; kl += 2) phase<st, false, SMALL>(v[kl * TF + fi], v[(kl + 1) * TF + fi], s_pre);
      }
      if constexpr (KPL == 8) {
        // each fibre of the tile gets 8 consecutive K values = one lane slot
        const int kb = kl0 / KB;
        const int g = (kl0 % KB) / 8;
#pragma unroll
        for (int fi = 0; fi < TF; ++fi) {
          const int fl = fl0 + fi;
          const int nf = fl / NB, nn = fl % NB;
          pc pieces[8][NPB];
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            const float x0 = (float)v[e * TF + fi], x1 = (float)v[(e + 1) * TF + fi];
            if constexpr (F16) {
              split_f16x2(x0, x1, s_exp, pieces[e], pieces[e + 1]);
            } else {
              split_bf16<NPB>(x0, pieces[e]);
              split_bf16<NPB>(x1, pieces[e + 1]);
            }
          }
#pragma unroll
          for (int p = 0; p < NPB; ++p) {
            afrag w;
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = pieces[e][p];
            const int off = ((kb * NFR + nf) * NPB + p) * BLK + (g * NB + swz(nn, kb, g)) * 8;
            *(afrag*)(L + off) = w;
          }
        }
      } else {
        // KPL == 1: one scalar per (kappa, fibre); consecutive fibres are
        // consecutive lanes.
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
          const int kl = kl0 + kk;
          const int kb = kl / KB, g = kl % KB;
#pragma unroll
          for (int fi = 0; fi < TF; ++fi) {
            const int fl = fl0 + fi;
            const int nf = fl / NB, nn = fl % NB;
            const int off = (kb * NFR + nf) * BLK + g * NB + nn;
            L[off] = (pc)v[kk * TF + fi];
          }
        }
      }
    }
  };

  // -------------------------------------------------------------- compute
  acc_t acc[WMF][WNF];
#pragma unroll
  for (int i = 0; i < WMF; ++i)
#pragma unroll
    for (int j = 0; j < WNF; ++j)
#pragma unroll
      for (int r = 0; r < T::NACC; ++r) acc[i][j][r] = 0;

  const afrag* __restrict__ Aop = (const afrag*)a.A;
  // the prepared operator is padded to a whole number of chunks (K) and of
  // 512-row tiles (M), so the inner loop needs no bounds checks
  const int nchunks = a.KBT / KCH;

  // Operator fragments of one K-block for this wave (from L2).  The wave's
  // fragments of one K-block are contiguous: WMF * NPS blocks of 64 lanes.
  const afrag* __restrict__ Aw = Aop + (int64_t)mf0 * NPS * 64 + lane;
  const int64_t a_kstride = (int64_t)a.MFT * NPS * 64;
  auto load_a = [&](int kbg, afrag (&dst)[WMF][NPA]) {
    const afrag* src = Aw + kbg * a_kstride;
#pragma unroll
    for (int p = 0; p < NPA; ++p)
#pragma unroll
      for (int i = 0; i < WMF; ++i) dst[i][p] = src[(i * NPS + p) * 64];
  };

  auto store_chunk = [&](int buf, auto small) {
#pragma unroll
    for (int u = 0; u < TPT; ++u) store_tile(u, buf, small);
  };
  // tiles [u0, u1) of the staged chunk
  auto store_part = [&](int buf, int u0, int u1, auto small) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (u >= u0 && u < u1) store_tile(u, buf, small);
  };
  typedef std::integral_constant<bool, false> ph_full_t;
  typedef std::integral_constant<bool, true> ph_small_t;
  constexpr bool PH2 = F16 && PRO && CPLX && OCC == 1;   // two forms of the main loop

  // B fragments of one K-block (local index kk of the LDS chunk) for this wave.
  // Piece-major order: the first products of a K-block need piece 0 of
  // every fragment, so those reads are issued (and complete) first.
  auto read_b = [&](const pc* L, int kk, afrag (&dst)[WNF][NPB]) {
#pragma unroll
    for (int p = 0; p < NPB; ++p)
#pragma unroll
      for (int j = 0; j < WNF; ++j) {
        const pc* blk = L + ((kk * NFR + nf0 + j) * NPB + p) * BLK;
        if constexpr (KPL == 8) {
          const int g = lane / NB, nn = lane % NB;
          dst[j][p] = *(const afrag*)(blk + (g * NB + swz(nn, kk, g)) * 8);
        } else {
          dst[j][p] = blk[lane];
        }
      }
  };

  // All MFMAs of one K-block: the piece products (outer), then the wave's
  // WMF x WNF fragments, so that consecutive MFMAs use different
  // accumulators.
  auto mfma_kblock = [&](const afrag (&af)[WMF][NPA], const afrag (&bf)[WNF][NPB]) {
#pragma unroll
    for (int k = 0; k < PP::N; ++k)
#pragma unroll
      for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) mfma(acc[i][j], af[i][PP::a(k)], bf[j][PP::b(k)]);
  };

  load_chunk(0);
  if (PH2 && ph_small) store_chunk(0, ph_small_t{});
  else store_chunk(0, ph_full_t{});
  __syncthreads();

  // Software pipeline over K-blocks.  While the MFMAs of K-block kb run, the
  // operator fragments of kb+1 (from L2) and its B fragments (from LDS,
  // within a chunk) are loaded into the other halves of register double
  // buffers.  The fibre tile of the next chunk is fetched from HBM at the
  // start of the current chunk, right after the operator loads of the
  // chunk's second K-block (vector-memory counters retire in order, so no
  // wait for an operator fragment of a later K-block has to wait for that
  // slower fetch), then split and written to the idle LDS buffer after the
  // chunk's MFMAs.
  static_assert(KCH % 2 == 0, "K-blocks per chunk must be even (register double buffer)");
  auto main_loop = [&](auto small) {
    afrag a_buf[2][WMF][NPA];
    afrag b_buf[2][WNF][NPB];
    load_a(0, a_buf[0]);
    read_b(lds, 0, b_buf[0]);
    const int kb_last = a.KBT - 1;
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      const pc* L = lds + buf * CHUNK;
#pragma unroll
      for (int kk = 0; kk < KCH; ++kk) {
        const int cur = kk & 1, nxt = cur ^ 1;
        const int kbg = c * KCH + kk;
        load_a(min(kbg + 1, kb_last), a_buf[nxt]);
        if (kk == 0 && more) load_chunk(c + 1);
        if (kk + 1 < KCH) read_b(L, kk + 1, b_buf[nxt]);
        if constexpr (KPL != 8) __builtin_amdgcn_sched_barrier(0);
        mfma_kblock(a_buf[cur], b_buf[cur]);
        // split and LDS writes of the next chunk, free to interleave with the
        // MFMAs of the last K-block, or (FP16X2) of the last two when there
        // are four or more (the fetch has landed by then: the operator loads
        // issued after it are waited for at the start of K-block KCH-2).  On
        // the last chunk this rewrites the idle buffer with stale data nobody
        // reads.  FP16X2 spreads the split evenly over the MFMAs (measured
        // faster); the three-piece BF16 split is left to the scheduler
        // (measured faster there).
        constexpr bool ST2 = F16 && KCH >= 4 && TPT >= 2;
        const bool st_here = (kk + 1 == KCH) || (ST2 && kk + 2 == KCH);
        if constexpr (ST2) {
          if (kk + 2 == KCH) store_part(buf ^ 1, 0, TPT / 2, small);
          if (kk + 1 == KCH) store_part(buf ^ 1, TPT / 2, TPT, small);
        } else {
          if (kk + 1 == KCH) store_chunk(buf ^ 1, small);
        }
        if constexpr (KPL == 8) {
          // split kernels (many MFMAs per K-block): issue the next K-block's
          // operator loads and LDS reads one at a time between this
          // K-block's MFMAs, so their issue cycles hide under MFMA execution
#pragma unroll
          for (int g = 0; g < WMF * NPS + (kk == 0 ? TPT * 4 : 0); ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          }
#pragma unroll
          for (int g = 0; g < WNF * NPB; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
          if (!st_here) {
            __builtin_amdgcn_sched_group_barrier(0x008, 64, 0);
          } else if constexpr (F16) {
            // staging K-blocks: a few VALU instructions of the split after
            // each MFMA, so that the matrix unit never waits behind a long
            // VALU run (a pipeline of its own, sync id 1)
            constexpr int REST = PP::N * WMF * WNF - WMF * NPS - WNF * NPB;
            constexpr int PER = (PRO ? 24 : 8) / (ST2 ? 2 : 1);
#pragma unroll
            for (int g = 0; g < REST; ++g) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
              __builtin_amdgcn_sched_group_barrier(0x002, PER, 1);
            }
          }
        }
        if (kk + 1 < KCH) __builtin_amdgcn_sched_barrier(0);
      }
      __syncthreads();
      read_b(lds + (buf ^ 1) * CHUNK, 0, b_buf[0]);
    }
  };
  if constexpr (OCC == 1) {
    if constexpr (PH2) {
      if (ph_small) main_loop(ph_small_t{});
      else main_loop(ph_full_t{});
    } else {
      main_loop(ph_full_t{});
    }
  } else {
    // Two workgroups share each CU (register budget of two waves per SIMD):
    // single register buffers, the other workgroup's MFMAs cover the waits.
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      const pc* L = lds + buf * CHUNK;
#pragma unroll
      for (int kk = 0; kk < KCH; ++kk) {
        const int kbg = c * KCH + kk;
        afrag af[WMF][NPA];
        afrag bf[WNF][NPB];
        load_a(kbg, af);
        if (kk == KCH - 1 && more) load_chunk(c + 1);
        read_b(L, kk, bf);
        mfma_kblock(af, bf);
      }
      if (more) {
        store_chunk(buf ^ 1, ph_full_t{});
        __syncthreads();
      }
    }
  }

  // ------------------------------------------------------------- epilogue
  // FP16X2: the accumulators hold 2^11 * 2^-(s_exp + a_exp) * result
  const int o_exp = s_exp + a.a_exp - 11;
  float vmax = 0.0f;   // FP16X2: max |component| stored by this lane
  // Contiguous fibres (mu = 1): each lane of an MFMA fragment holds one
  // fibre, so direct stores would write 8 bytes per lane at fibre stride.
  // When the tile is full and the LDS can hold a wave's fragments of one
  // M-fragment row, stage them there (swizzled 16-byte blocks, [fibre][32
  // real rows]) and write every fibre's 32 rows as one 128-byte run (eight
  // lanes x 16 bytes).
  constexpr bool T_EPI = FULL && LD == KL_KCONTIG && MB == 32 && sizeof(st) == 4 &&
                         (size_t)2 * CHUNK * sizeof(pc) >= (size_t)WM * WN * WNF * 32 * 32 * 4;
  if constexpr (T_EPI) {
    typedef float f32x4v __attribute__((ext_vector_type(4)));
    __syncthreads();   // every wave is done with the main loop's LDS
    float* reg = (float*)lds + (size_t)wave * WNF * 32 * 32;
    st* __restrict__ out = (st*)a.out;
    const st s_post = (st)a.s_post;
    // identity part: the input entries of a row block are loaded together,
    // one block ahead of its stores, so their latency is paid once per block
    // and no load waits behind the stores before it (one counter, in order)
    constexpr int NSB = WNF * 32 / 8;
    f32x4v xin[IDA ? 2 : 1][IDA ? NSB : 1];
    auto load_in = [&](int i, f32x4v (&dst)[IDA ? NSB : 1]) {
#pragma unroll
      for (int sblk = 0; sblk < NSB; ++sblk) {
        const int f = 8 * sblk + lane / 8;
        const int64_t fg = f0 + (int64_t)nf0 * NB + f;
        dst[sblk] = *(const f32x4v*)((const st*)a.in + fg * a.Mr + (mf0 + i) * 32 + 4 * (lane % 8));
      }
    };
    if constexpr (IDA) load_in(0, xin[0]);
#pragma unroll
    for (int i = 0; i < WMF; ++i) {
      const int mf = mf0 + i;
      if constexpr (IDA) {
        if (i + 1 < WMF) load_in(i + 1, xin[(i + 1) & 1]);
      }
#pragma unroll
      for (int j = 0; j < WNF; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = j * 32 + (lane % 32);
          const int b = 2 * q + lane / 32;   // rows 8q + 4(lane/32) .. +3
          f32x4v v;
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = (float)acc[i][j][4 * q + r];
          *(f32x4v*)(reg + f * 32 + ((b ^ (f & 7)) * 4)) = v;
        }
#pragma unroll
      for (int sblk = 0; sblk < WNF * 32 / 8; ++sblk) {
        const int f = 8 * sblk + lane / 8;
        const int b = lane % 8;              // rows 4b .. 4b+3 of the fragment
        f32x4v v = *(const f32x4v*)(reg + f * 32 + ((b ^ (f & 7)) * 4));
        st w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          w[r] = v[r];
          if constexpr (F16) w[r] = ldexpf(w[r], o_exp);
        }
        const int64_t fg = f0 + (int64_t)nf0 * NB + f;
        if constexpr (IDA) {
          // identity part: the input entries at the same position (square
          // operator: same layout), read by the lane that overwrites them
          const f32x4v x = xin[i & 1][sblk];
          st y[4] = {x[0], x[1], x[2], x[3]};
          if constexpr (PRO && CPLX) {
            phase<st>(y[0], y[1], s_pre);
            phase<st>(y[2], y[3], s_pre);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) w[r] += y[r];
        }
        if constexpr (CPLX && EPI) {
          phase<st>(w[0], w[1], s_post);
          phase<st>(w[2], w[3], s_post);
        }
        if constexpr (F16) vmax = fmaxf(vmax, fmaxf(fmaxf(fabsf(w[0]), fabsf(w[1])), fmaxf(fabsf(w[2]), fabsf(w[3]))));
        *(f32x4v*)(out + fg * a.Mr + mf * 32 + 4 * b) = f32x4v{w[0], w[1], w[2], w[3]};
      }
    }
  } else if constexpr (FULL) {
    // Every row and fibre of the tile exists and every byte offset of the
    // output fits in 32 bits (checked by the planner): a store address is
    // a wave-uniform base (row) plus a per-fragment lane offset (fibre).
    st* __restrict__ out = (st*)a.out;
    const st s_post = (st)a.s_post;
    const int64_t ostride = (LD == KL_KCONTIG) ? COMPS : a.P * COMPS;   // between entries i, i+1
    //  32x32 fragments: register 4q+r holds row 8q + 4(lane/32) + r.
    //  16x16 FP64 fragments: register r holds row lane/16 + 4r (complex rows
    //  permuted at preparation: (0,1) and (2,3) are entries mf*8 + lane/16
    //  and that + 4).
    const int lp = (MB == 32) ? (CPLX ? 2 : 4) * (lane / 32) : lane / 16;
    uint32_t voff[WNF];
#pragma unroll
    for (int j = 0; j < WNF; ++j) {
      const uint32_t fg = (uint32_t)(f0 + (nf0 + j) * NB + (lane % NB));
      uint32_t ob;
      if constexpr (LD == KL_KCONTIG) {
        ob = fg * (uint32_t)(a.m * COMPS);
      } else {
        const uint32_t q = fg / (uint32_t)a.P;
        const uint32_t p = fg - q * (uint32_t)a.P;
        ob = (p + (uint32_t)a.P * (uint32_t)a.m * q) * COMPS;
      }
      voff[j] = (ob + (uint32_t)lp * (uint32_t)ostride) * (uint32_t)sizeof(st);
    }
    // every output byte offset fits in 32 bits (checked by the planner): a
    // uniform base plus one 32-bit per-lane offset per store
    const uint32_t obytes = (uint32_t)ostride * (uint32_t)sizeof(st);
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef typename std::conditional<sizeof(st) == 4, f32x2, f64x2>::type st2;
    constexpr int GROUPS = T::NACC / 4;
    // identity part: the input entries of a row block are loaded together
    // at the start of the block (complex: (re, im) pairs; real: scalars), so
    // their latency is paid once per block; one block ahead would need a
    // second buffer, which spills here
    constexpr int NIN = IDA ? WNF * GROUPS * (CPLX ? 2 : 4) : 1;
    typedef typename std::conditional<CPLX, st2, st>::type inT;
    inT yin[1][NIN];
    auto load_in = [&](int i, inT (&dst)[NIN]) {
      const int mf = mf0 + i;
#pragma unroll
      for (int j = 0; j < WNF; ++j)
#pragma unroll
        for (int gq = 0; gq < GROUPS; ++gq) {
          if constexpr (CPLX) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int u = (MB == 32) ? mf * 16 + 4 * gq + h : mf * 8 + 4 * h;
              dst[(j * GROUPS + gq) * 2 + h] = *(const st2*)((const char*)a.in + ((uint32_t)u * obytes + voff[j]));
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int u = (MB == 32) ? mf * 32 + 8 * gq + r : mf * 16 + 4 * r;
              dst[(j * GROUPS + gq) * 4 + r] = *(const st*)((const char*)a.in + ((uint32_t)u * obytes + voff[j]));
            }
          }
        }
    };
#pragma unroll
    for (int i = 0; i < WMF; ++i) {
      const int mf = mf0 + i;
      if constexpr (IDA) load_in(i, yin[0]);
#pragma unroll
      for (int j = 0; j < WNF; ++j) {
#pragma unroll
        for (int gq = 0; gq < GROUPS; ++gq) {
          st v4[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            v4[r] = (st)acc[i][j][gq * 4 + r];
            if constexpr (F16) v4[r] = ldexpf(v4[r], o_exp);
          }
          if constexpr (CPLX) {
            if constexpr (IDA) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const st2 x = yin[0][(j * GROUPS + gq) * 2 + h];
                st y0 = x[0], y1 = x[1];
                if constexpr (PRO) phase<st>(y0, y1, s_pre);
                v4[2 * h] += y0;
                v4[2 * h + 1] += y1;
              }
            }
            if constexpr (EPI) {
              phase<st>(v4[0], v4[1], s_post);
              phase<st>(v4[2], v4[3], s_post);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int u = (MB == 32) ? mf * 16 + 4 * gq + h : mf * 8 + 4 * h;
              if constexpr (F16) vmax = fmaxf(fmaxf(vmax, fabsf(v4[2 * h])), fabsf(v4[2 * h + 1]));
              *(st2*)((char*)out + ((uint32_t)u * obytes + voff[j])) = st2{v4[2 * h], v4[2 * h + 1]};
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int u = (MB == 32) ? mf * 32 + 8 * gq + r : mf * 16 + 4 * r;
              if constexpr (IDA) v4[r] += yin[0][(j * GROUPS + gq) * 4 + r];
              if constexpr (F16) vmax = fmaxf(vmax, fabsf(v4[r]));
              *(st*)((char*)out + ((uint32_t)u * obytes + voff[j])) = v4[r];
            }
          }
        }
      }
    }
  } else {
    st* __restrict__ out = (st*)a.out;
    const st s_post = (st)a.s_post;
    // output offset of this lane's fibre in each N-fragment (once per fragment)
    int64_t obases[WNF];
    bool fvalid[WNF];
  #pragma unroll
    for (int j = 0; j < WNF; ++j) {
      const int64_t fg = f0 + (nf0 + j) * NB + (lane % NB);
      fvalid[j] = fg < a.F;
      if constexpr (LD == KL_KCONTIG) {
        obases[j] = fg * (int64_t)a.m * COMPS;
      } else if (a.F <= 0x7fffffff) {
        const uint32_t q = (uint32_t)fg / (uint32_t)a.P;
        const uint32_t p = (uint32_t)fg - q * (uint32_t)a.P;
        obases[j] = ((int64_t)p + a.P * (int64_t)a.m * q) * COMPS;
      } else {
        obases[j] = fibre_base(fg, a.P, a.m, COMPS);
      }
    }
    const int64_t ostride = (LD == KL_KCONTIG) ? COMPS : a.P * COMPS;   // between entries i, i+1
  #pragma unroll
    for (int i = 0; i < WMF; ++i) {
      const int mf = mf0 + i;
  #pragma unroll
      for (int j = 0; j < WNF; ++j) {
        if (!fvalid[j]) continue;
        const int64_t obase = obases[j];
        // Rows of this lane, in groups of four accumulator registers.
        //  32x32 fragments: register 4q+r holds row 8q + 4(lane/32) + r.
        //  16x16 FP64 fragments: register r holds row lane/16 + 4r; for complex
        //  operators the prepared rows are permuted so that registers (0,1)
        //  and (2,3) are (re, im) of entries mf*8 + lane/16 and that + 4.
        constexpr int GROUPS = T::NACC / 4;
  #pragma unroll
        for (int gq = 0; gq < GROUPS; ++gq) {
          st v4[4];
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            v4[r] = (st)acc[i][j][gq * 4 + r];
            if constexpr (F16) v4[r] = ldexpf(v4[r], o_exp);
          }
          if constexpr (CPLX) {
            int e0, e1;   // entries held as (v4[0], v4[1]) and (v4[2], v4[3])
            if constexpr (MB == 32) {
              e0 = (mf * 32 + 8 * gq + 4 * (lane / 32)) / 2;
              e1 = e0 + 1;
            } else {
              e0 = mf * 8 + lane / 16;
              e1 = e0 + 4;
            }
            if constexpr (IDA) {
  #pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int ie = h ? e1 : e0;
                if (ie < a.m) {
                  const st* src = (const st*)a.in + obase + (int64_t)ie * ostride;
                  st y0 = src[0], y1 = src[1];
                  if constexpr (PRO) phase<st>(y0, y1, s_pre);
                  v4[2 * h] += y0;
                  v4[2 * h + 1] += y1;
                }
              }
            }
            if constexpr (EPI) {
              phase<st>(v4[0], v4[1], s_post);
              phase<st>(v4[2], v4[3], s_post);
            }
  #pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int ie = h ? e1 : e0;
              if (ie < a.m) {
                if constexpr (F16) vmax = fmaxf(vmax, fmaxf(fabsf(v4[2 * h]), fabsf(v4[2 * h + 1])));
                st* dst = out + obase + (int64_t)ie * ostride;
                if constexpr (sizeof(st) == 4) {
                  typedef float f32x2 __attribute__((ext_vector_type(2)));
                  *(f32x2*)dst = f32x2{v4[2 * h], v4[2 * h + 1]};
                } else {
                  *(f64x2*)dst = f64x2{v4[2 * h], v4[2 * h + 1]};
                }
              }
            }
          } else {
  #pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ie = (MB == 32) ? mf * 32 + 8 * gq + 4 * (lane / 32) + r : mf * 16 + lane / 16 + 4 * r;
              if (ie < a.m) {
                if constexpr (IDA) v4[r] += ((const st*)a.in)[obase + (int64_t)ie * ostride];
                if constexpr (F16) vmax = fmaxf(vmax, fabsf(v4[r]));
                out[obase + (int64_t)ie * ostride] = v4[r];
              }
            }
          }
        }
      }
    }
  }
  if constexpr (F16) {
    // wave maximum, the waves' maxima meet in LDS, then one atomic per
    // workgroup into one word of the next launch's slot (non-negative floats
    // order like their bit patterns).  Atomics on one word serialise, and
    // the workgroups of a round finish together: one per workgroup rather
    // than one per wave, spread over SMAX_WORDS words, keeps that queue
    // short (one atomic per wave on a single word cost ~10 % per launch).
    // Every thread of the workgroup reaches this point.
    uint32_t mb = __float_as_uint(vmax);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mb = max(mb, (uint32_t)__shfl_xor((int)mb, o));
    __syncthreads();   // every wave is done with the LDS buffers
    uint32_t* wmx = (uint32_t*)lds;
    if (lane == 0) wmx[wave] = mb;
    __syncthreads();
    if (tid == 0) {
      uint32_t m = 0;
#pragma unroll
      for (int w = 0; w < WM * WN; ++w) m = max(m, wmx[w]);
      atomicMax(a.smax_out + (int)(tile_x % SMAX_WORDS), m);
    }
  }
}

template <int PR, bool CPLX, int LD, int WMF, int WNF, int WM, int WN, int KCH, bool PRO, bool EPI, int OCC,
          bool FULL, bool IDA>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
void mode_kernel(ModeArgs a) {
  typedef typename Tr<PR>::pc pc;
  constexpr int CHUNK = KCH * WN * WNF * Tr<PR>::NPB * 64 * Tr<PR>::KPL;
  __shared__ __attribute__((aligned(16))) pc lds[2 * CHUNK];
  mode_tile<PR, CPLX, LD, WMF, WNF, WM, WN, KCH, PRO, EPI, OCC, FULL, IDA>(a, blockIdx.x, blockIdx.y, lds);
}

// ------------------------------------------------------------ configs -----

// Tile shapes: class 0 is the default (WM waves stacked along M cover up to
// 512 real rows), classes 1 and 2 regroup the same waves 2 x 2 and 1 x 4 for
// operators with at most 256 / 128 real rows, classes 3 and 4 are alternative
// shapes of the split complex kernels (4 x 128 rows, 128 fibres, with 4 or 2
// K-blocks per LDS chunk), classes 5 and 6 split shapes with 64 fibres sized
// for two workgroups per CU (OCC = 2), class 7 a small split tile (4 x 64
// rows, 32 fibres, two workgroups per CU) for modes of at most 128 complex
// entries, where larger tiles leave too few workgroups to cover latency;
// class 10 the same tile with the whole K range of a 128-entry complex mode
// in one LDS chunk (FP16X2; BF16X3: half of it), so a tile waits for one HBM
// round trip instead of one per chunk.  (Classes 8 and 9 are the
// three-product kernels of mode_gauss.h.)
template <int PR, int CLS> struct Cfg;
template <> struct Cfg<KP_F64, 0> { static constexpr int WMF = 8, WNF = 2, WM = 4, WN = 1, KCH = 8; static constexpr int OCC = 1; };
template <> struct Cfg<KP_F64, 1> { static constexpr int WMF = 8, WNF = 1, WM = 2, WN = 2, KCH = 8; static constexpr int OCC = 1; };
template <> struct Cfg<KP_F64, 2> { static constexpr int WMF = 8, WNF = 1, WM = 1, WN = 4, KCH = 8; static constexpr int OCC = 1; };
// FP64 class 3: one wave, 32 real rows x 16 fibres, four waves per SIMD, for
// products with few fibres (the 2-D matrix products of the device
// exponential: a 256 x 256 complex product has 256 fibres, 8 workgroups of
// class 0 but 256 of this class); it splits the rows over workgroups, so its
// products run out of place
template <> struct Cfg<KP_F64, 3> { static constexpr int WMF = 2, WNF = 1, WM = 1, WN = 1, KCH = 8; static constexpr int OCC = 4; };
template <> struct Cfg<KP_F32, 0> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 32; static constexpr int OCC = 1; };
template <> struct Cfg<KP_F32, 1> { static constexpr int WMF = 4, WNF = 1, WM = 2, WN = 2, KCH = 32; static constexpr int OCC = 1; };
template <> struct Cfg<KP_F32, 2> { static constexpr int WMF = 4, WNF = 1, WM = 1, WN = 4, KCH = 32; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 0> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 1> { static constexpr int WMF = 4, WNF = 1, WM = 2, WN = 2, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 2> { static constexpr int WMF = 4, WNF = 1, WM = 1, WN = 4, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 3> { static constexpr int WMF = 4, WNF = 4, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 4> { static constexpr int WMF = 4, WNF = 4, WM = 4, WN = 1, KCH = 2; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16X3, 5> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 2; };
template <> struct Cfg<KP_BF16X3, 6> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 2; static constexpr int OCC = 2; };
template <> struct Cfg<KP_BF16X3, 7> { static constexpr int WMF = 2, WNF = 1, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 2; };
template <> struct Cfg<KP_BF16X3, 10> { static constexpr int WMF = 2, WNF = 1, WM = 4, WN = 1, KCH = 8; static constexpr int OCC = 2; };
template <> struct Cfg<KP_FP16X2, 0> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_FP16X2, 1> { static constexpr int WMF = 4, WNF = 1, WM = 2, WN = 2, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_FP16X2, 2> { static constexpr int WMF = 4, WNF = 1, WM = 1, WN = 4, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_FP16X2, 3> { static constexpr int WMF = 4, WNF = 4, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_FP16X2, 4> { static constexpr int WMF = 4, WNF = 4, WM = 4, WN = 1, KCH = 2; static constexpr int OCC = 1; };
template <> struct Cfg<KP_FP16X2, 5> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 2; };
template <> struct Cfg<KP_FP16X2, 6> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 2; static constexpr int OCC = 2; };
template <> struct Cfg<KP_FP16X2, 7> { static constexpr int WMF = 2, WNF = 1, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 2; };
template <> struct Cfg<KP_FP16X2, 10> { static constexpr int WMF = 2, WNF = 1, WM = 4, WN = 1, KCH = 16; static constexpr int OCC = 2; };
template <> struct Cfg<KP_BF16, 0> { static constexpr int WMF = 4, WNF = 2, WM = 4, WN = 1, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16, 1> { static constexpr int WMF = 4, WNF = 1, WM = 2, WN = 2, KCH = 4; static constexpr int OCC = 1; };
template <> struct Cfg<KP_BF16, 2> { static constexpr int WMF = 4, WNF = 1, WM = 1, WN = 4, KCH = 4; static constexpr int OCC = 1; };

template <int PR> struct NumCls { static constexpr int N = 3; };
template <> struct NumCls<KP_BF16X3> { static constexpr int N = 11; };
template <> struct NumCls<KP_FP16X2> { static constexpr int N = 11; };

template <int PR, int CLS> TileShape shape_of() {
  typedef Cfg<PR, CLS> C;
  return TileShape{C::WMF, C::WNF, C::WM, C::WN, C::KCH, C::OCC};
}

template <int PR, bool CPLX, int LD, bool PRO, bool EPI, int CLS, bool FULL = false, bool IDA = false>
KernFn kfn() {
  typedef Cfg<PR, CLS> C;
  return &mode_kernel<PR, CPLX, LD, C::WMF, C::WNF, C::WM, C::WN, C::KCH, PRO, EPI, C::OCC, FULL, IDA>;
}

// Full-tile variant when the planner allows it.
template <int PR, bool CPLX, int LD, bool PRO, bool EPI, int CLS, bool IDA>
KernFn kfx(int full) {
  return full ? kfn<PR, CPLX, LD, PRO, EPI, CLS, true, IDA>() : kfn<PR, CPLX, LD, PRO, EPI, CLS, false, IDA>();
}

// Kernel table of one precision.  Instances that exist: every (complex,
// load, prologue, epilogue) in class 0; classes 1, 2 without phases and not
// for the generic gather; classes >= 3 only for complex split kernels with
// contiguous or strided fibres.  Classes 0 and >= 3 also have a full-tile
// variant (full != 0: no per-store bounds checks, 32-bit output offsets) for
// contiguous and strided fibres.
// IDA: the instances with the identity add (a separate compile unit per
// precision and IDA keeps the builds parallel).
template <int PR, bool IDA>
KernFn pick_kernel(int cplx, int ld, int pro, int epi, int cls, int full) {
  if (ld == KL_PAIR) {
    // real operator on paired fibres: classes 0..2, no phases
    if (cplx || pro || epi) return nullptr;
    switch (cls) {
      case 0: return kfx<PR, false, KL_PAIR, false, false, 0, IDA>(full);
      case 1: return kfn<PR, false, KL_PAIR, false, false, 1, false, IDA>();
      case 2: return kfn<PR, false, KL_PAIR, false, false, 2, false, IDA>();
      default: return nullptr;
    }
  }
#define MM_PH(C_, L_, K_)                                                     \
  do {                                                                        \
    if (pro && epi) return kfx<PR, C_, L_, true, true, K_, IDA>(full);       \
    if (pro) return kfx<PR, C_, L_, true, false, K_, IDA>(full);             \
    if (epi) return kfx<PR, C_, L_, false, true, K_, IDA>(full);             \
    return kfx<PR, C_, L_, false, false, K_, IDA>(full);                     \
  } while (0)
  if constexpr (PR == KP_F64) {
    if (cls == 3) {
      if (pro || epi || (ld != KL_KCONTIG && ld != KL_FCONTIG)) return nullptr;
      if (cplx)
        return ld == KL_KCONTIG ? kfx<PR, true, KL_KCONTIG, false, false, 3, IDA>(full)
                                : kfx<PR, true, KL_FCONTIG, false, false, 3, IDA>(full);
      return ld == KL_KCONTIG ? kfx<PR, false, KL_KCONTIG, false, false, 3, IDA>(full)
                              : kfx<PR, false, KL_FCONTIG, false, false, 3, IDA>(full);
    }
  }
  if (cls == 1 || cls == 2) {
    if (pro || epi || ld == KL_GENERIC) return nullptr;
    if (cls == 1) {
      if (cplx) return ld == KL_KCONTIG ? kfn<PR, true, KL_KCONTIG, false, false, 1, false, IDA>() : kfn<PR, true, KL_FCONTIG, false, false, 1, false, IDA>();
      return ld == KL_KCONTIG ? kfn<PR, false, KL_KCONTIG, false, false, 1, false, IDA>() : kfn<PR, false, KL_FCONTIG, false, false, 1, false, IDA>();
    }
    if (cplx) return ld == KL_KCONTIG ? kfn<PR, true, KL_KCONTIG, false, false, 2, false, IDA>() : kfn<PR, true, KL_FCONTIG, false, false, 2, false, IDA>();
    return ld == KL_KCONTIG ? kfn<PR, false, KL_KCONTIG, false, false, 2, false, IDA>() : kfn<PR, false, KL_FCONTIG, false, false, 2, false, IDA>();
  }
  if constexpr (NumCls<PR>::N > 3) {
    if (cls >= 3) {
      if (!cplx || ld == KL_GENERIC) return nullptr;
      switch (cls) {
        case 3: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 3); else MM_PH(true, KL_FCONTIG, 3);
        case 4: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 4); else MM_PH(true, KL_FCONTIG, 4);
        case 5: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 5); else MM_PH(true, KL_FCONTIG, 5);
        case 6: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 6); else MM_PH(true, KL_FCONTIG, 6);
        case 7: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 7); else MM_PH(true, KL_FCONTIG, 7);
        case 10: if (ld == KL_KCONTIG) MM_PH(true, KL_KCONTIG, 10); else MM_PH(true, KL_FCONTIG, 10);
        default: return nullptr;
      }
    }
  }
  if (cls != 0) return nullptr;
  if (cplx) {
    switch (ld) {
      case KL_KCONTIG: MM_PH(true, KL_KCONTIG, 0);
      case KL_FCONTIG: MM_PH(true, KL_FCONTIG, 0);
      default: full = 0; MM_PH(true, KL_GENERIC, 0);
    }
  }
  switch (ld) {
    case KL_KCONTIG: return kfx<PR, false, KL_KCONTIG, false, false, 0, IDA>(full);
    case KL_FCONTIG: return kfx<PR, false, KL_FCONTIG, false, false, 0, IDA>(full);
    default: return kfn<PR, false, KL_GENERIC, false, false, 0, false, IDA>();
  }
#undef MM_PH
}

// Whether the merged batched kernel of a precision has the tile code of a
// work item kind (FP16X2 needs a state bound per instance: no batched
// kernels).
template <int PR>
bool batch_kind(int cplx, int ld, int cls) {
  (void)cplx;
  if constexpr (PR == KP_FP16X2) return false;
  return (ld == KL_KCONTIG || ld == KL_FCONTIG) && cls >= 0 && cls <= 2;
}

template <int PR>
bool shape_table(int cls, TileShape* out) {
  switch (cls) {
    case 0: *out = shape_of<PR, 0>(); return true;
    case 1: *out = shape_of<PR, 1>(); return true;
    case 2: *out = shape_of<PR, 2>(); return true;
    default: break;
  }
  if constexpr (PR == KP_F64) {
    if (cls == 3) {
      *out = shape_of<PR, 3>();
      return true;
    }
  }
  if constexpr (NumCls<PR>::N > 3) {
    switch (cls) {
      case 3: *out = shape_of<PR, 3>(); return true;
      case 4: *out = shape_of<PR, 4>(); return true;
      case 5: *out = shape_of<PR, 5>(); return true;
      case 6: *out = shape_of<PR, 6>(); return true;
      case 7: *out = shape_of<PR, 7>(); return true;
      case 10: *out = shape_of<PR, 10>(); return true;
      default: break;
    }
  }
  return false;
}

// Merged batched kernel of one precision: a work item's kind selects the
// tile code (complex, load path, tile class 0..2), so items of every kind
// share one launch.  All classes 0..2 use 4 waves.
template <int PR, int CLS>
constexpr int lds_scalars() {
  typedef Cfg<PR, CLS> C;
  return 2 * C::KCH * C::WN * C::WNF * Tr<PR>::NPB * 64 * Tr<PR>::KPL;
}

template <int PR>
constexpr int merged_lds_scalars() {
  constexpr int a = lds_scalars<PR, 0>(), b = lds_scalars<PR, 1>(), c = lds_scalars<PR, 2>();
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <int PR, bool IDA>
__global__ __launch_bounds__(256) void mode_batch_merged_kernel(const BatchItem* __restrict__ items) {
  typedef typename Tr<PR>::pc pc;
  __shared__ __attribute__((aligned(16))) pc lds[merged_lds_scalars<PR>()];
  const BatchItem& it = items[blockIdx.x];
  const ModeArgs a = it.a;
#define MM_MK(C_, L_, K_)                                                                                  \
  case (C_ ? 100 : 0) + L_ * 10 + K_: {                                                                    \
    typedef Cfg<PR, K_> CF;                                                                                \
    static_assert(CF::WM * CF::WN == 4, "merged batch classes use 4 waves");                               \
    mode_tile<PR, C_, L_, CF::WMF, CF::WNF, CF::WM, CF::WN, CF::KCH, false, false, 1, false, IDA>(a, it.tile_x, it.tile_y, lds); \
    break;                                                                                                 \
  }
  switch (it.kind) {
    MM_MK(true, KL_KCONTIG, 0)
    MM_MK(true, KL_KCONTIG, 1)
    MM_MK(true, KL_KCONTIG, 2)
    MM_MK(true, KL_FCONTIG, 0)
    MM_MK(true, KL_FCONTIG, 1)
    MM_MK(true, KL_FCONTIG, 2)
    MM_MK(false, KL_KCONTIG, 0)
    MM_MK(false, KL_KCONTIG, 1)
    MM_MK(false, KL_KCONTIG, 2)
    MM_MK(false, KL_FCONTIG, 0)
    MM_MK(false, KL_FCONTIG, 1)
    MM_MK(false, KL_FCONTIG, 2)
    default: break;
  }
#undef MM_MK
}

// IDA: work items whose operators carry the identity split (a launch of
// their own, so the plain merged kernel keeps its register allocation).
template <int PR, bool IDA>
BatchFn pick_batch_merged() {
  return &mode_batch_merged_kernel<PR, IDA>;
}

}  // namespace mm
