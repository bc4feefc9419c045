// Complex mu-mode products in split precision with three real products.
//
// For a complex operator L = A + iB acting on complex fibres x + iy, the
// result is  Re = A x - B y,  Im = A y + B x.  The kernels of mode_tile.h
// form it as one real GEMM with the 2 x 2 real block operator: four real
// products per complex multiply-add.  Gauss's form needs three,
//     T1 = A x,   T2 = B y,   T3 = (A + B)(x + y),
//     Re = T1 - T2,   Im = T3 - T1 - T2,
// so a quarter of the MFMA work goes (every split piece product of it).
// A + B is formed in FP64 when the operator is prepared and split like any
// other operator; x + y is formed in FP32 as the fibre tile is staged and
// split with x and y.  Error: besides the split rounding of the three
// products (each at the level of the four-product form), Im carries the
// FP32 rounding of x + y (2^-24 of |x + y|, below the split's own
// representation error) and the cancellation in T3 - T1 - T2, whose terms
// are at most about twice |Im|'s natural scale |A||y| + |B||x| when the
// operator is near a unitary one.  FP16X2 gives both sums one more bit of
// headroom: the state exponent is one above the four-product form's, and the
// operator scale is chosen from max(|A|, |B|, |A + B|).
//
// Layouts.  The prepared operator holds, per complex K-block jb (16 complex
// columns) and type t (0: A, 1: B, 2: A + B), the 32-row fragments of the
// complex rows in MFMA A-operand order:  slot ((jb * 3 + t) * MFT + mf,
// piece, lane) of 8 values, lane = row % 32 + 32 * (column half).  The LDS
// chunk holds KCJ complex K-blocks of the fibre tile as 3 * KCJ MFMA K-blocks
// (kk = kbj * 3 + t), each an x, y or x + y block of every N-fragment and
// piece.  A wave owns WMG complex-row fragments per type and WNF fibre
// fragments: 3 * WMG * WNF accumulators, and each MFMA K-block feeds only the
// accumulators of its own type.
//
// Pipeline.  The operator fragments of a whole chunk sit in a register ring
// (one slot per K-block); slot kk is refilled with the next chunk's fragment
// right after its MFMAs.  The next chunk of the fibre tile is fetched from
// HBM at the start of each chunk, before those refills, so no operator load
// that the current chunk waits for queues behind the slower fetch (the
// vector-memory counter retires in order); the fetch has a whole chunk of
// MFMA work to land before it is split into the idle LDS buffer.
#pragma once

namespace mm {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Tile classes of the three-product kernels (numbered after the four-product
// classes of the same precision).  WM waves x WMG complex-row fragments of
// 32 rows, WNF fibre fragments of 32 fibres, KCJ complex K-blocks per chunk.
template <int PR, int CLS> struct GCfg;
template <> struct GCfg<KP_FP16X2, 8> { static constexpr int WMG = 2, WNF = 2, WM = 4, KCJ = 4; };
template <> struct GCfg<KP_FP16X2, 9> { static constexpr int WMG = 2, WNF = 2, WM = 4, KCJ = 2; };
template <> struct GCfg<KP_BF16X3, 8> { static constexpr int WMG = 2, WNF = 2, WM = 4, KCJ = 2; };
template <> struct GCfg<KP_BF16X3, 9> { static constexpr int WMG = 2, WNF = 2, WM = 4, KCJ = 1; };

template <int PR, int LD, int WMG, int WNF, int WM, int KCJ, bool PRO, bool EPI, bool FULL>
__device__ __forceinline__ void gauss_tile(const ModeArgs& a, int64_t tile_x, int tile_y,
                                           typename Tr<PR>::pc* __restrict__ lds) {
  typedef Tr<PR> T;
  typedef float st;
  typedef typename T::pc pc;
  typedef typename T::afrag afrag;
  typedef Prods<PR> PP;
  constexpr int NPA = T::NPA, NPS = T::NPS, NPB = T::NPB;
  constexpr bool F16 = PR == KP_FP16X2;
  constexpr int THREADS = 64 * WM;
  constexpr int NT = WNF * 32;             // fibres per workgroup
  constexpr int NKB = 3 * KCJ;             // MFMA K-blocks per chunk
  constexpr int CJ = 16 * KCJ;             // complex K entries per chunk
  constexpr int BLK = 512;                 // pieces per (K-block, N-fragment, piece) block
  constexpr int CHUNK = NKB * WNF * NPB * BLK;
  static_assert(LD == KL_KCONTIG || LD == KL_FCONTIG, "contiguous or strided fibres");
  static_assert(PR == KP_FP16X2 || PR == KP_BF16X3, "split precisions");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t f0 = tile_x * NT;
  const int mf0 = (tile_y * WM + wave) * WMG;
  const st* __restrict__ in = (const st*)a.in;
  const st s_pre = (st)a.s_pre;

  // FP16X2: state exponent one above the four-product form's (x + y needs
  // the extra bit); the first workgroup clears the slot the previous launch
  // read.  ph_small: the prologue phase angle is bounded by pi/4.
  int s_exp = 0;
  bool ph_small = false;
  if constexpr (F16) {
    uint32_t bbits = 0;
#pragma unroll
    for (int w = 0; w < SMAX_WORDS; ++w) bbits = max(bbits, a.smax_in[w]);
    s_exp = fp16x2_state_exp(bbits) + 1;
    if (tile_x == 0 && tile_y == 0 && tid < SMAX_WORDS) a.smax_clr[tid] = 0u;
    const float bnd = __uint_as_float(bbits);
    ph_small = fabsf((float)a.s_pre) * 2.0f * bnd * bnd <= 0.78f;
  }

  // ---------------------------------------------------------------- staging
  // A staging tile is 8 complex entries (16 floats) of TF fibres: one lane
  // slot (8 K values) of each of the x, y and x + y blocks.
  constexpr int TF = (LD == KL_FCONTIG) ? 2 : 1;
  constexpr int TILES_K = CJ / 8;
  constexpr int TILES_F = NT / TF;
  constexpr int TILES = TILES_K * TILES_F;
  static_assert(TILES % THREADS == 0 || TILES < THREADS, "tiles must split evenly");
  constexpr int TPT = (TILES + THREADS - 1) / THREADS;
  constexpr int VPT = 16 * TF;
  st stage[TPT][VPT];   // v[kl * TF + fi]: real K value kl = 2 j + c of fibre fi

  auto tile_coords = [&](int t, int& tk, int& tf) {
    if constexpr (LD == KL_KCONTIG) {
      tk = t % TILES_K;
      tf = t / TILES_K;
    } else {
      tf = t % TILES_F;
      tk = t / TILES_F;
    }
  };
  // source of each staging tile in chunk 0
  const st* tsrc[TPT];
  bool tok[TPT];
  int tj[TPT];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    int tk, tf;
    tile_coords(tid + u * THREADS, tk, tf);
    const int64_t fg = f0 + (int64_t)tf * TF;
    tok[u] = (TILES >= THREADS || tid < TILES) && (FULL || fg < a.F);
    tj[u] = tk * 8;
    if constexpr (LD == KL_KCONTIG) {
      tsrc[u] = in + (tok[u] ? fg * (int64_t)a.Kr + tk * 16 : 0);
    } else {
      // fibres fg, fg + 1 (fg even, P a multiple of 4) share a 16-byte vector
      tsrc[u] = in + (tok[u] ? fibre_base(fg, a.P, a.n, 2) + (int64_t)(tk * 8) * a.P * 2 : 0);
    }
  }
  const int64_t rstride = (int64_t)a.P * 2;   // floats between rows j, j + 1 (strided fibres)
  const int64_t cstride = (LD == KL_KCONTIG) ? (int64_t)2 * CJ : (int64_t)CJ * rstride;

  auto load_chunk = [&](int c) {
    const int jlim = a.n - c * CJ;   // n is a multiple of 8: a tile is all in or all out
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      if (TILES < THREADS && tid >= TILES) break;
      st* v = stage[u];
      const bool ok = tok[u] && tj[u] < jlim;
      const st* src = tsrc[u] + c * cstride;
      if constexpr (LD == KL_KCONTIG) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          f32x4 x = {0.f, 0.f, 0.f, 0.f};
          if (ok) x = *(const f32x4*)(src + 4 * w);
#pragma unroll
          for (int e = 0; e < 4; ++e) v[4 * w + e] = x[e];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          f32x4 x = {0.f, 0.f, 0.f, 0.f};
          if (ok) x = *(const f32x4*)(src + r * rstride);
          // (re, im) of fibre 0, then of fibre 1, at row r
          v[(2 * r) * 2 + 0] = x[0];
          v[(2 * r + 1) * 2 + 0] = x[1];
          v[(2 * r) * 2 + 1] = x[2];
          v[(2 * r + 1) * 2 + 1] = x[3];
        }
      }
    }
  };

  // Prologue phase, x + y, the split into pieces and the LDS writes of
  // staging tile u into buffer `buf`.
  auto store_tile = [&](int u, int buf, auto small) {
    constexpr bool SMALL = decltype(small)::value;
    if (TILES < THREADS && tid >= TILES) return;
    pc* L = lds + buf * CHUNK;
    int tk, tf;
    tile_coords(tid + u * THREADS, tk, tf);
    st* v = stage[u];
    if constexpr (PRO) {
#pragma unroll
      for (int fi = 0; fi < TF; ++fi)
#pragma unroll
        for (int e = 0; e < 8; ++e) phase<st, false, SMALL>(v[(2 * e) * TF + fi], v[(2 * e + 1) * TF + fi], s_pre);
    }
    const int kbj = tk / 2, g = tk % 2;   // 8 entries: one half of a 16-entry K-block
#pragma unroll
    for (int fi = 0; fi < TF; ++fi) {
      const int fl = tf * TF + fi;
      const int nf = fl / 32, nn = fl % 32;
      pc pieces[3][8][NPB];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const float x0 = v[(2 * e) * TF + fi], y0 = v[(2 * e + 1) * TF + fi];
        const float x1 = v[(2 * e + 2) * TF + fi], y1 = v[(2 * e + 3) * TF + fi];
        const float z0 = x0 + y0, z1 = x1 + y1;
        if constexpr (F16) {
          split_f16x2(x0, x1, s_exp, pieces[0][e], pieces[0][e + 1]);
          split_f16x2(y0, y1, s_exp, pieces[1][e], pieces[1][e + 1]);
          split_f16x2(z0, z1, s_exp, pieces[2][e], pieces[2][e + 1]);
        } else {
          split_bf16<NPB>(x0, pieces[0][e]);
          split_bf16<NPB>(x1, pieces[0][e + 1]);
          split_bf16<NPB>(y0, pieces[1][e]);
          split_bf16<NPB>(y1, pieces[1][e + 1]);
          split_bf16<NPB>(z0, pieces[2][e]);
          split_bf16<NPB>(z1, pieces[2][e + 1]);
        }
      }
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int p = 0; p < NPB; ++p) {
          afrag w;
#pragma unroll
          for (int e = 0; e < 8; ++e) w[e] = pieces[t][e][p];
          const int kk = kbj * 3 + t;
          *(afrag*)(L + ((kk * WNF + nf) * NPB + p) * BLK + (g * 32 + swz(nn, kk, g)) * 8) = w;
        }
    }
  };

  // B fragments of LDS K-block kk for this wave, piece-major.
  auto read_b = [&](const pc* L, int kk, afrag (&dst)[WNF][NPB]) {
    const int g = lane / 32, nn = lane % 32;
#pragma unroll
    for (int p = 0; p < NPB; ++p)
#pragma unroll
      for (int j = 0; j < WNF; ++j)
        dst[j][p] = *(const afrag*)(L + ((kk * WNF + j) * NPB + p) * BLK + (g * 32 + swz(nn, kk, g)) * 8);
  };

  // Operator fragments of global MFMA K-block kbg (= jb * 3 + t) for this wave.
  const afrag* __restrict__ Aw = (const afrag*)a.A + (int64_t)mf0 * NPS * 64 + lane;
  const int64_t a_kstride = (int64_t)a.MFT * NPS * 64;
  auto load_a = [&](int kbg, afrag (&dst)[WMG][NPA]) {
    const afrag* src = Aw + kbg * a_kstride;
#pragma unroll
    for (int p = 0; p < NPA; ++p)
#pragma unroll
      for (int i = 0; i < WMG; ++i) dst[i][p] = src[(i * NPS + p) * 64];
  };

  f32x16 acc[3][WMG][WNF];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int i = 0; i < WMG; ++i)
#pragma unroll
      for (int j = 0; j < WNF; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][i][j][r] = 0.0f;

  auto mfma_kb = [&](auto tc, const afrag (&af)[WMG][NPA], const afrag (&bf)[WNF][NPB]) {
    constexpr int t = decltype(tc)::value;
#pragma unroll
    for (int k = 0; k < PP::N; ++k)
#pragma unroll
      for (int i = 0; i < WMG; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) mfma(acc[t][i][j], af[i][PP::a(k)], bf[j][PP::b(k)]);
  };

  typedef std::integral_constant<bool, false> ph_full_t;
  typedef std::integral_constant<bool, true> ph_small_t;
  constexpr bool PH2 = F16 && PRO;   // two forms of the main loop
  const int nchunks = a.KBT / KCJ;   // the prepared operator is padded to whole chunks

  // Epilogue of one tile (fibres from f0, complex-row fragments from mf0):
  // Re = T1 - T2, Im = T3 - (T1 + T2).  FP16X2: the accumulators hold
  // 2^11 * 2^-(s_exp + a_exp) * T_t.  Register 4q + r of a fragment holds
  // complex row 8q + 4 (lane / 32) + r.
  const int o_exp = s_exp + a.a_exp - 11;
  float vmax = 0.0f;
  st* __restrict__ out = (st*)a.out;
  const st s_post = (st)a.s_post;
  const int64_t ostride = (LD == KL_KCONTIG) ? 2 : rstride;   // floats between entries i, i + 1
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  auto epilogue = [&]() {
#pragma unroll
    for (int j = 0; j < WNF; ++j) {
      const int64_t fg = f0 + j * 32 + (lane % 32);
      const bool fok = FULL || fg < a.F;
      int64_t ob;
      if constexpr (LD == KL_KCONTIG) {
        ob = fg * 2 * (int64_t)a.m;
      } else {
        const int64_t q = fg / a.P;
        ob = (fg - q * a.P + a.P * (int64_t)a.m * q) * 2;
      }
#pragma unroll
      for (int i = 0; i < WMG; ++i) {
        const int mf = mf0 + i;
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
          float re[4], im[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float t1 = acc[0][i][j][4 * qd + r], t2 = acc[1][i][j][4 * qd + r];
            const float t3 = acc[2][i][j][4 * qd + r];
            re[r] = t1 - t2;
            im[r] = t3 - (t1 + t2);
            if constexpr (F16) {
              re[r] = ldexpf(re[r], o_exp);
              im[r] = ldexpf(im[r], o_exp);
            }
            if constexpr (EPI) phase<st>(re[r], im[r], s_post);
            if constexpr (F16) vmax = fmaxf(vmax, fmaxf(fabsf(re[r]), fabsf(im[r])));
          }
          const int e0 = mf * 32 + 8 * qd + 4 * (lane / 32);
          if constexpr (LD == KL_KCONTIG) {
            if (FULL || (fok && e0 + 3 < a.m)) {
              *(f32x4*)(out + ob + 2 * e0) = f32x4{re[0], im[0], re[1], im[1]};
              *(f32x4*)(out + ob + 2 * e0 + 4) = f32x4{re[2], im[2], re[3], im[3]};
            } else if (fok) {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (e0 + r < a.m) *(f32x2*)(out + ob + 2 * (e0 + r)) = f32x2{re[r], im[r]};
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (FULL || (fok && e0 + r < a.m)) *(f32x2*)(out + ob + (e0 + r) * ostride) = f32x2{re[r], im[r]};
          }
        }
      }
    }
  };

  auto main_loop = [&](auto small) {
    afrag ring[NKB][WMG][NPA];
    afrag b_buf[2][WNF][NPB];
    load_chunk(0);
    static_for<0, NKB>([&](auto kc) { load_a(decltype(kc)::value, ring[decltype(kc)::value]); });
#pragma unroll
    for (int u = 0; u < TPT; ++u) store_tile(u, 0, small);
    __syncthreads();
    read_b(lds, 0, b_buf[0]);
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const pc* L = lds + buf * CHUNK;
      // chunk fetched during this one: the next, or (last chunk) this one
      // again.  The fetch and the ring refills are issued on every path, so
      // the wait counts stay exact and a wait for one ring slot never drains
      // the refills issued after it.
      const int fc = min(c + 1, nchunks - 1);
      static_for<0, NKB>([&](auto kc) {
        constexpr int kk = decltype(kc)::value;
        constexpr int cur = kk & 1, nxt = cur ^ 1;
        if constexpr (kk == 0) load_chunk(fc);
        if constexpr (kk + 1 < NKB) read_b(L, kk + 1, b_buf[nxt]);
        mfma_kb(std::integral_constant<int, kk % 3>{}, ring[kk], b_buf[cur]);
        load_a(fc * NKB + kk, ring[kk]);
        // split and LDS writes of the fetched chunk over the last K-blocks
        // (on the last chunk this rewrites the idle buffer with stale data
        // nobody reads)
        constexpr int u0 = kk - (NKB - TPT);
        if constexpr (u0 >= 0) store_tile(u0, buf ^ 1, small);
        // the next K-block's LDS reads (and the chunk fetch) one at a time
        // between the first MFMAs, then (staging K-blocks) a few split
        // instructions after each MFMA; the ring refills can only follow the
        // MFMAs that read the slot, so they go last
        constexpr int NMF = PP::N * WMG * WNF;
        constexpr int NDS0 = (kk + 1 < NKB) ? WNF * NPB : 0;
        constexpr int NDS = NDS0 < NMF ? NDS0 : NMF;
        constexpr int NFE0 = kk == 0 ? TPT * (LD == KL_KCONTIG ? 4 : 8) : 0;
        constexpr int NFE = NFE0 < NMF - NDS ? NFE0 : NMF - NDS;
        static_for<0, NDS>([&](auto) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        });
        static_for<0, NFE>([&](auto) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        });
        if constexpr (u0 >= 0) {
          static_for<0, NMF - NDS - NFE>([&](auto) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, PRO ? 12 : 6, 0);
          });
        }
        if constexpr (kk + 1 < NKB) __builtin_amdgcn_sched_barrier(0);
      });
      __syncthreads();
      read_b(lds + (buf ^ 1) * CHUNK, 0, b_buf[0]);
    }
    epilogue();
  };
  if constexpr (PH2) {
    if (ph_small) main_loop(ph_small_t{});
    else main_loop(ph_full_t{});
  } else {
    main_loop(ph_full_t{});
  }

  if constexpr (F16) {
    // the running bound of the results: wave maximum, the waves meet in LDS,
    // one atomic per workgroup (non-negative floats order like their bits)
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
      for (int w = 0; w < WM; ++w) m = max(m, wmx[w]);
      atomicMax(a.smax_out + (int)(tile_x % SMAX_WORDS), m);
    }
  }
}

template <int PR, int LD, int WMG, int WNF, int WM, int KCJ, bool PRO, bool EPI, bool FULL>
__global__ __launch_bounds__(64 * WM) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gauss_kernel(ModeArgs a) {
  constexpr int CHUNK = 3 * KCJ * WNF * Tr<PR>::NPB * 512;
  __shared__ __attribute__((aligned(16))) typename Tr<PR>::pc lds[2 * CHUNK];
  gauss_tile<PR, LD, WMG, WNF, WM, KCJ, PRO, EPI, FULL>(a, blockIdx.x, blockIdx.y, lds);
}

template <int PR, int CLS, int LD, bool PRO, bool EPI>
KernFn gfn(int full) {
  typedef GCfg<PR, CLS> C;
  return full ? &gauss_kernel<PR, LD, C::WMG, C::WNF, C::WM, C::KCJ, PRO, EPI, true>
              : &gauss_kernel<PR, LD, C::WMG, C::WNF, C::WM, C::KCJ, PRO, EPI, false>;
}

template <int PR, int CLS>
KernFn gauss_pick_cls(int ld, int pro, int epi, int full) {
#define MM_G(L_)                                                      \
  do {                                                                \
    if (pro && epi) return gfn<PR, CLS, L_, true, true>(full);        \
    if (pro) return gfn<PR, CLS, L_, true, false>(full);              \
    if (epi) return gfn<PR, CLS, L_, false, true>(full);              \
    return gfn<PR, CLS, L_, false, false>(full);                      \
  } while (0)
  if (ld == KL_KCONTIG) MM_G(KL_KCONTIG);
  if (ld == KL_FCONTIG) MM_G(KL_FCONTIG);
#undef MM_G
  return nullptr;
}

// Three-product kernel of class cls (8 or 9) of a split precision, complex
// operator and state, contiguous or strided fibres; nullptr otherwise.
template <int PR>
KernFn gauss_pick(int ld, int pro, int epi, int cls, int full) {
  switch (cls) {
    case 8: return gauss_pick_cls<PR, 8>(ld, pro, epi, full);
    case 9: return gauss_pick_cls<PR, 9>(ld, pro, epi, full);
    default: return nullptr;
  }
}

template <int PR>
bool gauss_shape(int cls, TileShape* out) {
  // in the four-product terms of the planner: WMF real-row fragments of 32
  // rows per wave (2 WMG), KCH real K-blocks per chunk (2 KCJ)
  switch (cls) {
    case 8: *out = TileShape{2 * GCfg<PR, 8>::WMG, GCfg<PR, 8>::WNF, GCfg<PR, 8>::WM, 1, 2 * GCfg<PR, 8>::KCJ, 1}; return true;
    case 9: *out = TileShape{2 * GCfg<PR, 9>::WMG, GCfg<PR, 9>::WNF, GCfg<PR, 9>::WM, 1, 2 * GCfg<PR, 9>::KCJ, 1}; return true;
    default: return false;
  }
}

}  // namespace mm
