// Internal interface between the host runtime (mumode_runtime.cpp) and the
// HIP kernels (mode_kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

enum KPrec { KP_F64 = 0, KP_F32 = 1, KP_BF16X3 = 2, KP_BF16 = 3 };
enum KLoad { KL_KCONTIG = 0, KL_FCONTIG = 1, KL_GENERIC = 2 };

// Geometry of the MFMA fragment a precision uses: M rows and K values per
// fragment, K values each lane holds, operator pieces per value.
struct FragGeom {
  int MB, NB, KB, KPL, NPC;
};
FragGeom frag_geom(int prec);
int split_variant();

// Arguments of one mu-mode product launch (real-GEMM view, see
// mode_kernels.hip).  Complex tensors: P, Q, n, m count complex entries.
struct ModeArgs {
  const void* in;
  void* out;
  const void* A;       // operator in fragment order (mm_prepare_operator)
  int64_t P, Q, F;     // fibres: F = P*Q, entry (p, j, q) at p + P*(j + n*q)
  int n, m;            // mode length of input / output
  int Kr, Mr;          // real-GEMM K and M (2n, 2m when complex)
  int KBT, MFT;        // K-blocks and M-fragments of the prepared operator
  double s_pre;        // prologue phase: psi *= exp(-i s_pre |psi|^2) (0: off)
  double s_post;       // epilogue phase, same form
};

// Per-launch plan chosen by the runtime.
struct ModePlan {
  int prec, cplx, load, pro, epi;
  int variant;         // tile shape variant (split complex kernels)
  int grid_x, grid_y, threads;
  int mt_rows;         // real rows covered by one workgroup (multiple of MB)
  bool covers_all_rows;
};

// Fill `plan` for the given problem; returns false if no kernel fits.
bool plan_mode(const ModeArgs& a, int prec, int cplx, bool want_pro, bool want_epi,
               bool fcontig_ok, bool kcontig_ok, ModePlan* plan);
hipError_t launch_mode(const ModePlan& plan, const ModeArgs& a, hipStream_t s);

// Convert an FP64 master (device, column-major, ld) into fragment order.
// rowph / colph (device, complex FP64, may be null) scale row i / column j of
// a complex master by the given unit-modulus factors before conversion.
hipError_t launch_prepare(int prec, int cplx, const double* master, int64_t rows, int64_t cols,
                          int64_t ld, const double* rowph, const double* colph, void* out,
                          int KBT, int MFT, hipStream_t s);
size_t prepared_bytes(int prec, int KBT, int MFT);

// Two-pass deterministic FP64 sum of |x|^2 over `count` scalars (fp32 or
// fp64).  partial: device buffer of >= norm_partials() doubles.
int norm_partials();
hipError_t launch_norm2(const void* x, int64_t count, int is_f64, double* partial,
                        double* result, hipStream_t s);

}  // namespace mm
