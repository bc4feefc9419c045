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
//   KP_BF16    same MFMA, one piece each (comparison only).
//
// Fused Gross-Pitaevskii phase.  The exact nonlinear subflow
// psi <- exp(-i s beta |psi|^2) psi (Section 4.5: the nonlinear part is
// integrated exactly) is applied to the loaded fibres (prologue) and/or to
// the results (epilogue), so no separate pass over the state is needed.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstdlib>

#include "mm_internal.h"

namespace mm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
  static constexpr int MB = 16, NB = 16, KB = 4, KPL = 1, NPC = 1, NACC = 4;
};
template <> struct Tr<KP_F32> {
  typedef float st;
  typedef float pc;
  typedef float afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 2, KPL = 1, NPC = 1, NACC = 16;
};
template <> struct Tr<KP_BF16X3> {
  typedef float st;
  typedef __bf16 pc;
  typedef bf16x8 afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 16, KPL = 8, NPC = 3, NACC = 16;
};
template <> struct Tr<KP_BF16> {
  typedef float st;
  typedef __bf16 pc;
  typedef bf16x8 afrag;
  typedef f32x16 acc;
  static constexpr int MB = 32, NB = 32, KB = 16, KPL = 8, NPC = 1, NACC = 16;
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

// Piece pairs (a, b) of the split product, a + b <= NPC - 1.
template <int NPC> struct Prods;
template <> struct Prods<1> {
  static constexpr int N = 1;
  __device__ static constexpr int a(int) { return 0; }
  __device__ static constexpr int b(int) { return 0; }
};
template <> struct Prods<3> {
  static constexpr int N = 6;
  // (0,0) (0,1) (1,0) (0,2) (1,1) (2,0)
  __device__ static constexpr int a(int k) { return k == 2 ? 1 : k == 4 ? 1 : k == 5 ? 2 : 0; }
  __device__ static constexpr int b(int k) { return k == 1 ? 1 : k == 3 ? 2 : k == 4 ? 1 : 0; }
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

// exp(-i s |z|^2) z
template <typename T>
__device__ __forceinline__ void phase(T& re, T& im, T s) {
  T th = s * (re * re + im * im);
  T sn, cs;
  if constexpr (sizeof(T) == 8) {
    sincos(th, &sn, &cs);
  } else {
    sincosf(th, &sn, &cs);
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

template <int PR, bool CPLX, int LD, int WMF, int WNF, int WAVES, int KCH, bool PRO, bool EPI>
__global__ __launch_bounds__(64 * WAVES) void mode_kernel(ModeArgs a) {
  typedef Tr<PR> T;
  typedef typename T::st st;
  typedef typename T::pc pc;
  typedef typename T::afrag afrag;
  typedef typename T::acc acc_t;
  constexpr int MB = T::MB, NB = T::NB, KB = T::KB, KPL = T::KPL, NPC = T::NPC;
  constexpr int THREADS = 64 * WAVES;
  constexpr int NT = WNF * NB;           // fibres per workgroup
  constexpr int NFR = WNF;               // N-fragments per workgroup
  constexpr int CK = KCH * KB;           // real K values per chunk
  constexpr int BLK = 64 * KPL;          // scalars per (kb, nf, piece) block
  constexpr int CHUNK = KCH * NFR * NPC * BLK;
  constexpr int COMPS = CPLX ? 2 : 1;
  typedef Prods<NPC> PP;

  __shared__ __attribute__((aligned(16))) pc lds[2 * CHUNK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t f0 = (int64_t)blockIdx.x * NT;
  const int mf0 = (blockIdx.y * WAVES + wave) * WMF;   // first M-fragment of this wave

  const st* __restrict__ in = (const st*)a.in;
  const st s_pre = (st)a.s_pre;

  // ---------------------------------------------------------------- staging
  // Tile of TK real K values x TF fibres handled by one thread at a time.
  constexpr int VL = 16 / sizeof(st);    // scalars per 16-byte vector
  constexpr int TK = (KPL == 8) ? 8 : (LD == KL_KCONTIG ? VL : (CPLX ? 2 : 1));
  constexpr int TF = (LD == KL_FCONTIG) ? (KPL == 8 ? (CPLX ? VL / 2 : VL) : (CPLX ? VL / 2 : VL)) : 1;
  constexpr int TILES_K = CK / TK;
  constexpr int TILES_F = NT / TF;
  constexpr int TILES = TILES_K * TILES_F;
  static_assert(TILES % THREADS == 0 || TILES < THREADS, "tiles must split evenly");
  constexpr int TPT = (TILES + THREADS - 1) / THREADS;   // tiles per thread
  constexpr int VPT = TK * TF;           // scalars per tile
  st stage[TPT][VPT];

  auto tile_coords = [&](int t, int& tk, int& tf) {
    if constexpr (LD == KL_KCONTIG) {
      tk = t % TILES_K;
      tf = t / TILES_K;
    } else {
      tf = t % TILES_F;
      tk = t / TILES_F;
    }
  };

  // Load chunk `c` (real K values [c*CK, c*CK + CK)) into registers.
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      if (TILES < THREADS && tid >= TILES) break;
      int tk, tf;
      tile_coords(tid + u * THREADS, tk, tf);
      const int k0 = c * CK + tk * TK;       // first real K of the tile
      const int64_t fl = (int64_t)tf * TF;   // first local fibre
      const int64_t fg = f0 + fl;
      st* v = stage[u];
      if constexpr (LD == KL_KCONTIG) {
        // P == 1: fibre fg's K values are contiguous; TK of them, vectorised.
        if (fg < a.F && k0 < a.Kr) {
          const st* src = in + fg * (int64_t)a.Kr + k0;
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
      } else if constexpr (LD == KL_FCONTIG) {
        // Fibres contiguous: one 16-byte vector holds TF fibres at one row j.
        constexpr int ROWS = CPLX ? TK / 2 : TK;
        const int64_t base = (fg < a.F) ? fibre_base(fg, a.P, a.n, COMPS) : 0;
        const int j0 = CPLX ? k0 / 2 : k0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          const int j = j0 + r;
          st xv[VL];
          if (fg < a.F && j < a.n) {
            const st* src = in + base + (int64_t)j * a.P * COMPS;
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
      if constexpr (PRO && CPLX) {
        // entries (kappa even, odd) of one fibre are (re, im) of one value
#pragma unroll
        for (int fi = 0; fi < TF; ++fi)
#pragma unroll
          for (int kl = 0; kl < TK; kl += 2) phase<st>(v[kl * TF + fi], v[(kl + 1) * TF + fi], s_pre);
      }
    }
  };

  // Write the staged registers into LDS buffer `buf`, split into pieces.
  auto store_chunk = [&](int buf) {
    pc* L = lds + buf * CHUNK;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      if (TILES < THREADS && tid >= TILES) break;
      int tk, tf;
      tile_coords(tid + u * THREADS, tk, tf);
      const int kl0 = tk * TK;
      const int fl0 = tf * TF;
      const st* v = stage[u];
      if constexpr (KPL == 8) {
        // each fibre of the tile gets 8 consecutive K values = one lane slot
        const int kb = kl0 / KB;
        const int g = (kl0 % KB) / 8;
#pragma unroll
        for (int fi = 0; fi < TF; ++fi) {
          const int fl = fl0 + fi;
          const int nf = fl / NB, nn = fl % NB;
          __bf16 pieces[8][NPC];
#pragma unroll
          for (int e = 0; e < 8; ++e) split_bf16<NPC>((float)v[e * TF + fi], pieces[e]);
#pragma unroll
          for (int p = 0; p < NPC; ++p) {
            bf16x8 w;
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = pieces[e][p];
            const int off = ((kb * NFR + nf) * NPC + p) * BLK + (g * NB + swz(nn, kb, g)) * 8;
            *(bf16x8*)(L + off) = w;
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
  const int nchunks = (a.KBT + KCH - 1) / KCH;

  load_chunk(0);
  store_chunk(0);
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load_chunk(c + 1);   // global loads in flight during the MFMAs
    const pc* L = lds + buf * CHUNK;
#pragma unroll
    for (int kk = 0; kk < KCH; ++kk) {
      const int kbg = c * KCH + kk;           // global K-block
      if (kbg < a.KBT) {
        afrag af[WMF][NPC];
#pragma unroll
        for (int i = 0; i < WMF; ++i)
#pragma unroll
          for (int p = 0; p < NPC; ++p) {
            const int mf = mf0 + i;
            af[i][p] = (mf < a.MFT) ? Aop[(((int64_t)kbg * a.MFT + mf) * NPC + p) * 64 + lane]
                                    : afrag{};
          }
        afrag bfr[WNF][NPC];
#pragma unroll
        for (int j = 0; j < WNF; ++j)
#pragma unroll
          for (int p = 0; p < NPC; ++p) {
            const pc* blk = L + ((kk * NFR + j) * NPC + p) * BLK;
            if constexpr (KPL == 8) {
              const int g = lane / NB, nn = lane % NB;
              bfr[j][p] = *(const afrag*)(blk + (g * NB + swz(nn, kk, g)) * 8);
            } else {
              bfr[j][p] = blk[lane];
            }
          }
#pragma unroll
        for (int k = 0; k < PP::N; ++k)
#pragma unroll
          for (int i = 0; i < WMF; ++i)
#pragma unroll
            for (int j = 0; j < WNF; ++j) mfma(acc[i][j], af[i][PP::a(k)], bfr[j][PP::b(k)]);
      }
    }
    if (c + 1 < nchunks) {
      store_chunk(buf ^ 1);
      __syncthreads();
    }
  }

  // ------------------------------------------------------------- epilogue
  st* __restrict__ out = (st*)a.out;
  const st s_post = (st)a.s_post;
#pragma unroll
  for (int i = 0; i < WMF; ++i) {
    const int mf = mf0 + i;
    if (mf >= a.MFT) continue;
#pragma unroll
    for (int j = 0; j < WNF; ++j) {
      const int64_t fg = f0 + j * NB + (lane % NB);
      if (fg >= a.F) continue;
      const int64_t obase = (LD == KL_KCONTIG) ? fg * (int64_t)a.m * COMPS : fibre_base(fg, a.P, a.m, COMPS);
      const int64_t ostride = (LD == KL_KCONTIG) ? COMPS : a.P * COMPS;   // between entries i, i+1
      // rows of this lane: groups of 4 consecutive rows
      constexpr int GROUPS = T::NACC / 4;
#pragma unroll
      for (int gq = 0; gq < GROUPS; ++gq) {
        int row0;
        if constexpr (MB == 32) row0 = mf * 32 + 8 * gq + 4 * (lane / 32);
        else row0 = mf * 16 + 4 * (lane / 16);
        st v4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v4[r] = (st)acc[i][j][gq * 4 + r];
        if constexpr (CPLX) {
          // rows row0..row0+3 = (re, im) of entries i0 = row0/2 and i0 + 1
          const int i0 = row0 / 2;
          if constexpr (EPI) {
            phase<st>(v4[0], v4[1], s_post);
            phase<st>(v4[2], v4[3], s_post);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int ie = i0 + h;
            if (ie < a.m) {
              st* dst = out + obase + (int64_t)ie * ostride;
              if constexpr (sizeof(st) == 4) {
                *(float2*)dst = make_float2(v4[2 * h], v4[2 * h + 1]);
              } else {
                *(f64x2*)dst = f64x2{v4[2 * h], v4[2 * h + 1]};
              }
            }
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ie = row0 + r;
            if (ie < a.m) out[obase + (int64_t)ie * ostride] = v4[r];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ configs -----

// Tile shapes per precision: WMF x WNF fragments per wave, WAVES waves
// stacked along M, KCH K-blocks per LDS chunk.
template <int PR, int V = 0> struct Cfg;
template <> struct Cfg<KP_F64, 0> { static constexpr int WMF = 8, WNF = 2, WAVES = 4, KCH = 8; };
template <> struct Cfg<KP_F32, 0> { static constexpr int WMF = 4, WNF = 2, WAVES = 4, KCH = 32; };
template <> struct Cfg<KP_BF16X3, 0> { static constexpr int WMF = 4, WNF = 2, WAVES = 4, KCH = 4; };
template <> struct Cfg<KP_BF16, 0> { static constexpr int WMF = 4, WNF = 2, WAVES = 4, KCH = 4; };
// alternative tile shapes of the split complex kernels (selected at run time)
template <> struct Cfg<KP_BF16X3, 1> { static constexpr int WMF = 4, WNF = 4, WAVES = 4, KCH = 4; };
template <> struct Cfg<KP_BF16X3, 2> { static constexpr int WMF = 4, WNF = 4, WAVES = 4, KCH = 2; };
template <> struct Cfg<KP_BF16X3, 3> { static constexpr int WMF = 2, WNF = 2, WAVES = 8, KCH = 4; };
constexpr int SPLIT_VARIANTS = 4;

typedef void (*KernFn)(ModeArgs);

template <int PR, bool CPLX, int LD, bool PRO, bool EPI, int V>
KernFn pick5() {
  typedef Cfg<PR, V> C;
  return &mode_kernel<PR, CPLX, LD, C::WMF, C::WNF, C::WAVES, C::KCH, PRO, EPI>;
}

template <int PR, bool CPLX, int LD, bool PRO, bool EPI>
KernFn pick4(int v) {
  if constexpr (PR == KP_BF16X3 && CPLX && LD != KL_GENERIC) {
    switch (v) {
      case 1: return pick5<PR, CPLX, LD, PRO, EPI, 1>();
      case 2: return pick5<PR, CPLX, LD, PRO, EPI, 2>();
      case 3: return pick5<PR, CPLX, LD, PRO, EPI, 3>();
      default: break;
    }
  }
  return pick5<PR, CPLX, LD, PRO, EPI, 0>();
}

template <int PR, bool CPLX, int LD>
KernFn pick3(int pro, int epi, int v) {
  if constexpr (CPLX) {
    if (pro && epi) return pick4<PR, CPLX, LD, true, true>(v);
    if (pro) return pick4<PR, CPLX, LD, true, false>(v);
    if (epi) return pick4<PR, CPLX, LD, false, true>(v);
  }
  return pick4<PR, CPLX, LD, false, false>(v);
}

template <int PR, bool CPLX>
KernFn pick2(int ld, int pro, int epi, int v) {
  switch (ld) {
    case KL_KCONTIG: return pick3<PR, CPLX, KL_KCONTIG>(pro, epi, v);
    case KL_FCONTIG: return pick3<PR, CPLX, KL_FCONTIG>(pro, epi, v);
    default: return pick3<PR, CPLX, KL_GENERIC>(pro, epi, v);
  }
}

template <int PR>
KernFn pick1(int cplx, int ld, int pro, int epi, int v) {
  return cplx ? pick2<PR, true>(ld, pro, epi, v) : pick2<PR, false>(ld, pro, epi, v);
}

KernFn pick(int prec, int cplx, int ld, int pro, int epi, int v) {
  switch (prec) {
    case KP_F64: return pick1<KP_F64>(cplx, ld, pro, epi, 0);
    case KP_F32: return pick1<KP_F32>(cplx, ld, pro, epi, 0);
    case KP_BF16X3: return pick1<KP_BF16X3>(cplx, ld, pro, epi, v);
    default: return pick1<KP_BF16>(cplx, ld, pro, epi, 0);
  }
}

template <int PR, int V> void cfg_of(int& wmf, int& wnf, int& waves) {
  wmf = Cfg<PR, V>::WMF;
  wnf = Cfg<PR, V>::WNF;
  waves = Cfg<PR, V>::WAVES;
}

// -------------------------------------------------------- preparation -----

template <int PR>
__global__ void prepare_kernel(const double* __restrict__ master, int64_t rows, int64_t cols,
                               int64_t ld, int cplx, const double* __restrict__ rowph,
                               const double* __restrict__ colph, void* __restrict__ outv, int KBT,
                               int MFT) {
  typedef Tr<PR> T;
  typedef typename T::pc pc;
  constexpr int MB = T::MB, KB = T::KB, KPL = T::KPL, NPC = T::NPC;
  const int64_t slots = (int64_t)KBT * MFT * 64;   // (kb, mf, lane)
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= slots) return;
  const int lane = (int)(s % 64);
  const int64_t t = s / 64;
  const int mf = (int)(t % MFT);
  const int kb = (int)(t / MFT);
  const int64_t Mr = cplx ? 2 * rows : rows;
  const int64_t Kr = cplx ? 2 * cols : cols;
  pc* out = (pc*)outv;
  const int row = mf * MB + (lane % MB);
  for (int e = 0; e < KPL; ++e) {
    const int kap = kb * KB + KPL * (lane / MB) + e;
    double x = 0.0;
    if (row < Mr && kap < Kr) {
      if (cplx) {
        const int64_t i = row / 2, j = kap / 2;
        const int cr = row & 1, ck = kap & 1;
        double re = master[2 * (i + j * ld)], im = master[2 * (i + j * ld) + 1];
        if (rowph) {
          const double pr = rowph[2 * i], pi = rowph[2 * i + 1];
          const double r2 = re * pr - im * pi;
          im = re * pi + im * pr;
          re = r2;
        }
        if (colph) {
          const double qr = colph[2 * j], qi = colph[2 * j + 1];
          const double r2 = re * qr - im * qi;
          im = re * qi + im * qr;
          re = r2;
        }
        x = (cr == ck) ? re : (cr == 0 ? -im : im);
      } else {
        x = master[row + kap * ld];
      }
    }
    const int64_t base = (((int64_t)kb * MFT + mf) * NPC) * 64 * KPL + lane * KPL + e;
    if constexpr (PR == KP_F64) {
      out[base] = x;
    } else if constexpr (PR == KP_F32) {
      out[base] = (float)x;
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
}

// ------------------------------------------------------------- norm2 ------

constexpr int NORM_BLOCKS = 1024;
constexpr int NORM_THREADS = 256;

template <typename S>
__global__ __launch_bounds__(NORM_THREADS) void norm_partial_kernel(const S* __restrict__ x,
                                                                    int64_t count,
                                                                    double* __restrict__ partial) {
  __shared__ double red[NORM_THREADS];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * NORM_THREADS) {
    const double v = (double)x[i];
    acc += v * v;
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

}  // namespace

// ---------------------------------------------------------- host side -----

// Tile variant of the split complex kernels: MUMODE_SPLIT_TILE=0..3
// (read once; default 0).
int split_variant() {
  static int v = [] {
    const char* e = std::getenv("MUMODE_SPLIT_TILE");
    int x = e ? std::atoi(e) : 0;
    return (x >= 0 && x < SPLIT_VARIANTS) ? x : 0;
  }();
  return v;
}

FragGeom frag_geom(int prec) {
  switch (prec) {
    case KP_F64: return {16, 16, 4, 1, 1};
    case KP_F32: return {32, 32, 2, 1, 1};
    case KP_BF16X3: return {32, 32, 16, 8, 3};
    default: return {32, 32, 16, 8, 1};
  }
}

size_t prepared_bytes(int prec, int KBT, int MFT) {
  FragGeom g = frag_geom(prec);
  size_t elems = (size_t)KBT * MFT * g.NPC * 64 * g.KPL;
  size_t es = prec == KP_F64 ? 8 : prec == KP_F32 ? 4 : 2;
  return elems * es;
}

bool plan_mode(const ModeArgs& a, int prec, int cplx, bool want_pro, bool want_epi, bool fcontig_ok,
               bool kcontig_ok, ModePlan* plan) {
  int wmf = 0, wnf = 0, waves = 0;
  const int load = kcontig_ok ? KL_KCONTIG : (fcontig_ok ? KL_FCONTIG : KL_GENERIC);
  int v = 0;
  if (prec == KP_BF16X3 && cplx && load != KL_GENERIC) v = split_variant();
  switch (prec) {
    case KP_F64: cfg_of<KP_F64, 0>(wmf, wnf, waves); break;
    case KP_F32: cfg_of<KP_F32, 0>(wmf, wnf, waves); break;
    case KP_BF16X3:
      switch (v) {
        case 1: cfg_of<KP_BF16X3, 1>(wmf, wnf, waves); break;
        case 2: cfg_of<KP_BF16X3, 2>(wmf, wnf, waves); break;
        case 3: cfg_of<KP_BF16X3, 3>(wmf, wnf, waves); break;
        default: cfg_of<KP_BF16X3, 0>(wmf, wnf, waves); break;
      }
      break;
    default: cfg_of<KP_BF16, 0>(wmf, wnf, waves); break;
  }
  plan->variant = v;
  FragGeom g = frag_geom(prec);
  const int nt = wnf * g.NB;
  plan->prec = prec;
  plan->cplx = cplx;
  plan->pro = (want_pro && cplx) ? 1 : 0;
  plan->epi = (want_epi && cplx) ? 1 : 0;
  plan->load = load;
  plan->threads = 64 * waves;
  plan->mt_rows = waves * wmf * g.MB;
  plan->grid_x = (int)((a.F + nt - 1) / nt);
  plan->grid_y = (a.MFT + waves * wmf - 1) / (waves * wmf);
  plan->covers_all_rows = plan->grid_y == 1;
  return plan->grid_x > 0 && (int64_t)plan->grid_x * nt >= a.F;
}

hipError_t launch_mode(const ModePlan& p, const ModeArgs& a, hipStream_t s) {
  KernFn fn = pick(p.prec, p.cplx, p.load, p.pro, p.epi, p.variant);
  dim3 grid(p.grid_x, p.grid_y, 1);
  hipLaunchKernelGGL(fn, grid, dim3(p.threads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prepare(int prec, int cplx, const double* master, int64_t rows, int64_t cols,
                          int64_t ld, const double* rowph, const double* colph, void* out, int KBT,
                          int MFT, hipStream_t s) {
  const int64_t slots = (int64_t)KBT * MFT * 64;
  const int threads = 256;
  const int blocks = (int)((slots + threads - 1) / threads);
  switch (prec) {
    case KP_F64:
      hipLaunchKernelGGL(prepare_kernel<KP_F64>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, rowph, colph, out, KBT, MFT);
      break;
    case KP_F32:
      hipLaunchKernelGGL(prepare_kernel<KP_F32>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, rowph, colph, out, KBT, MFT);
      break;
    case KP_BF16X3:
      hipLaunchKernelGGL(prepare_kernel<KP_BF16X3>, dim3(blocks), dim3(threads), 0, s, master,
                         rows, cols, ld, cplx, rowph, colph, out, KBT, MFT);
      break;
    default:
      hipLaunchKernelGGL(prepare_kernel<KP_BF16>, dim3(blocks), dim3(threads), 0, s, master, rows,
                         cols, ld, cplx, rowph, colph, out, KBT, MFT);
      break;
  }
  return hipGetLastError();
}

int norm_partials() { return NORM_BLOCKS; }

hipError_t launch_norm2(const void* x, int64_t count, int is_f64, double* partial, double* result,
                        hipStream_t s) {
  if (is_f64)
    hipLaunchKernelGGL(norm_partial_kernel<double>, dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s,
                       (const double*)x, count, partial);
  else
    hipLaunchKernelGGL(norm_partial_kernel<float>, dim3(NORM_BLOCKS), dim3(NORM_THREADS), 0, s,
                       (const float*)x, count, partial);
  hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(NORM_THREADS), 0, s, partial, NORM_BLOCKS,
                     result);
  return hipGetLastError();
}

}  // namespace mm
