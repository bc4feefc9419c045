// Internal interface between the host runtime (mumode_runtime.cpp) and the
// HIP kernels (mode_kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

enum KPrec { KP_F64 = 0, KP_F32 = 1, KP_BF16X3 = 2, KP_FP16X2 = 3, KP_BF16 = 4 };
// Fibre load paths: KCONTIG fibres contiguous (mu = 1, P = 1); FCONTIG
// fibres interleaved with P % 4 == 0 (16-byte loads along P); GENERIC any
// P (gather); PAIR P == 2, pairs of fibres interleaved (a real operator on
// the (re, im) planes of a complex state along mode 1: each 16-byte load
// holds two fibres' consecutive entries).
enum KLoad { KL_KCONTIG = 0, KL_FCONTIG = 1, KL_GENERIC = 2, KL_PAIR = 3 };

// Geometry of the MFMA fragment a precision uses: M rows and K values per
// fragment, K values each lane holds, operator pieces per value (FP16X2
// keeps three: hi * 2^11, hi, lo; see mode_tile.h).
// KPAD / MPAD: the prepared operator's K-blocks and M-fragments are padded
// (with zeros) to multiples of these, so that every tile shape reads whole
// chunks and whole row tiles.
struct FragGeom {
  int MB, NB, KB, KPL, NPC, KPAD, MPAD;
};
FragGeom frag_geom(int prec);
// Padded K-block and M-fragment counts of a prepared operator with Mr real
// rows and Kr real columns.
void op_blocks(int prec, int64_t Mr, int64_t Kr, int* KBT, int* MFT);

// Arguments of one mu-mode product launch (real-GEMM view, see
// mode_kernels.hip).  Complex tensors: P, Q, n, m count complex entries.
// Words per running-bound slot: the workgroups of a launch spread their
// atomic maxima over this many words, so they do not all queue on one.
constexpr int SMAX_WORDS = 8;

struct ModeArgs {
  const void* in;
  void* out;
  const void* A;       // operator in fragment order (mm_prepare_operator)
  int64_t P, Q, F;     // fibres: F = P*Q, entry (p, j, q) at p + P*(j + n*q)
  int n, m;            // mode length of input / output
  int Kr, Mr;          // real-GEMM K and M (2n, 2m when complex)
  int KBT, MFT;        // padded K-blocks and M-fragments of the prepared operator
  double s_pre;        // prologue phase: psi *= exp(-i s_pre |psi|^2) (0: off)
  double s_post;       // epilogue phase, same form
  // FP16X2 only: running bound of the state.  Each slot is SMAX_WORDS words;
  // the maximum over smax_in's words is the float bits of max |component| of
  // `in`; the launch raises smax_out (workgroup tile_x into word
  // tile_x % SMAX_WORDS) to that of `out` and clears smax_clr (the slot the
  // launch before it read).  The operator pieces represent L * 2^-a_exp.
  const uint32_t* smax_in;
  uint32_t* smax_out;
  uint32_t* smax_clr;
  int a_exp;
  // identity split: the operator pieces hold L - I (square L) and the
  // epilogue adds the input entry at the same position back in FP32 (after
  // the prologue phase when there is one)
  int idadd;
};

// Per-workgroup work item of a batched launch.
struct BatchItem {
  ModeArgs a;
  int64_t tile_x;
  int tile_y;
  int kind;            // complex * 100 + load path * 10 + tile class (0..2)
};

typedef void (*KernFn)(ModeArgs);
typedef void (*BatchFn)(const BatchItem*);

// Workgroup tile shape: WM x WN waves, each with WMF x WNF MFMA fragments,
// KCH K-blocks per LDS chunk.
struct TileShape {
  int WMF, WNF, WM, WN, KCH, OCC;
};

// Kernel tables, one per precision (kern_<prec>.hip).  cls selects the tile
// shape (0 default; 1, 2 regrouped waves for operators with at most 256 / 128
// real rows; 3..6 alternative split shapes).  nullptr if no instance exists.
KernFn pick_kernel_f64(int cplx, int ld, int pro, int epi, int cls, int full, int ida);
KernFn pick_kernel_f32(int cplx, int ld, int pro, int epi, int cls, int full, int ida);
KernFn pick_kernel_bf16x3(int cplx, int ld, int pro, int epi, int cls, int full, int ida);
KernFn pick_kernel_fp16x2(int cplx, int ld, int pro, int epi, int cls, int full, int ida);
KernFn pick_kernel_bf16(int cplx, int ld, int pro, int epi, int cls, int full, int ida);
bool batch_kind_f64(int cplx, int ld, int cls);
bool batch_kind_f32(int cplx, int ld, int cls);
bool batch_kind_bf16x3(int cplx, int ld, int cls);
bool batch_kind_fp16x2(int cplx, int ld, int cls);
bool batch_kind_bf16(int cplx, int ld, int cls);
bool tile_shape_f64(int cls, TileShape* out);
bool tile_shape_f32(int cls, TileShape* out);
bool tile_shape_bf16x3(int cls, TileShape* out);
bool tile_shape_fp16x2(int cls, TileShape* out);
bool tile_shape_bf16(int cls, TileShape* out);

bool tile_shape(int prec, int cls, TileShape* out);

// Three-product (Gauss) complex split kernels (kern_<prec>_g.hip), tile
// classes 8 and 9 of BF16X3 and FP16X2: complex operator and state,
// contiguous or strided fibres, operator prepared by launch_prepare_gauss.
KernFn pick_gauss_bf16x3(int ld, int pro, int epi, int cls, int full);
KernFn pick_gauss_fp16x2(int ld, int pro, int epi, int cls, int full);
bool gauss_shape_bf16x3(int cls, TileShape* out);
bool gauss_shape_fp16x2(int cls, TileShape* out);
inline bool is_gauss_class(int cls) { return cls == 8 || cls == 9; }
// Padded complex K-blocks (16 columns, a multiple of 4) and complex-row
// fragments (32 rows, a multiple of 8) of a three-product operator.
void gauss_blocks(int64_t rows, int64_t cols, int* JBT, int* MFT);
size_t gauss_prepared_bytes(int prec, int JBT, int MFT);
// master: complex FP64, column-major with leading dimension ld.
hipError_t launch_prepare_gauss(int prec, const double* master, int64_t rows, int64_t cols, int64_t ld, void* out,
                                int JBT, int MFT, int a_exp, hipStream_t s);

// Merged batched launch: one kernel per precision runs work items of every
// kind (complex / real, contiguous / strided fibres, tile class 0..2; all
// 256 threads), so every instance tile of one mode goes in a single launch.
BatchFn pick_batch_merged_f64();
BatchFn pick_batch_merged_f32();
BatchFn pick_batch_merged_bf16x3();
BatchFn pick_batch_merged_bf16();
BatchFn pick_batch_merged_f64_ida();
BatchFn pick_batch_merged_f32_ida();
BatchFn pick_batch_merged_bf16x3_ida();
BatchFn pick_batch_merged_bf16_ida();
// ida: the items' operators carry the identity split (a.idadd set on all)
hipError_t launch_mode_batch_merged(int prec, int ida, const BatchItem* items, int count, hipStream_t s);

// Per-launch plan chosen by the runtime.
struct ModePlan {
  int prec, cplx, load, pro, epi;
  int cls;             // tile shape class
  int grid_x, grid_y, threads;
  int nt;              // fibres per workgroup
  int mt_rows;         // real rows covered by one workgroup (multiple of MB)
  bool covers_all_rows;
  int full;            // every tile complete and output offsets fit 32 bits
  int gauss;           // three-product kernel: the operator's Gauss preparation
};

// Fill `plan` for the given problem; returns false if no kernel fits.
// batch: plan for the batched work-list kernel (tile classes 0..2 only).
// force_cls >= 0: use that tile class if an instance exists for the problem
// (the autotuner's choice), else fall back to the built-in choice.
bool plan_mode(const ModeArgs& a, int prec, int cplx, bool want_pro, bool want_epi,
               bool fcontig_ok, bool kcontig_ok, ModePlan* plan, bool batch = false, int force_cls = -1,
               bool gauss_ok = false);
// Number of tile classes of a precision (classes 0 .. n-1).
int num_classes(int prec);
// start / stop (optional): events recorded by the launch itself
hipError_t launch_mode(const ModePlan& plan, const ModeArgs& a, hipStream_t s, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr);
// Whole-run kernel for small states (kern_small.hip): one workgroup, every
// step and mode of an expstep.  m[k].A == nullptr skips mode k; every mode
// must be planned with tile class SMALL_RUN_CLASS covering all its rows, with
// in == out == the state.
#define SMALL_RUN_CLASS 2
struct SmallRun {
  ModeArgs m[6];
  int load[6];
  int tiles[6];   // fibre tiles of mode k (its plan's grid_x)
  int d, nsteps;
};
hipError_t launch_small_run(int prec, int cplx, const SmallRun& r, int* threads_out, hipStream_t s);
// Whole run of a 2-D real FP64 integrator (n1, n2 <= 64) in one workgroup
// with the state and the operators resident in LDS (kern_small.hip): U
// (n1 x n2, column-major) <- E1 U E2^T nsteps times; E1 / E2 are FP64
// masters (ld = rows), NULL leaves that mode unchanged.
hipError_t launch_small_lds(double* U, int n1, int n2, const double* E1, const double* E2, int nsteps,
                            hipStream_t s);

// Optional diagonal phase scaling of a complex master before conversion:
// L'[i,j] = exp(-i rc rx2[i]) L[i,j] exp(-i cc cx2[j]); rx2 / cx2 are device
// arrays (null = no factor).
struct PhaseScale {
  const double* rx2 = nullptr;
  double rc = 0.0;
  const double* cx2 = nullptr;
  double cc = 0.0;
};

// One operator preparation (the arguments of launch_prepare).
struct PrepJob {
  const double* master = nullptr;
  int64_t rows = 0, cols = 0, ld = 0;
  int cplx = 0;
  PhaseScale ph;
  void* out = nullptr;
  int KBT = 0, MFT = 0, a_exp = 0;
};
constexpr int MAX_PREP_JOBS = 6;
struct PrepJobs {
  PrepJob j[MAX_PREP_JOBS];
  int n = 0;
};
// Up to MAX_PREP_JOBS preparations of one precision in one launch.
hipError_t launch_prepare_multi(int prec, const PrepJobs& jobs, hipStream_t s);

// The collapsed harmonic-oscillator propagators of `steps` consecutive steps
// of the time-dependent splitting, for up to 6 modes of one precision, in
// one launch: step s, entry e gets the diagonal phase factors
// exp(-i ca x_i^2) on its rows and exp(-i cb x_j^2) on its columns, where
// cb and ca are the potential's flows over the step's two halves,
// (eps/2)(cos t - cos(t + tau/2)) and (eps/2)(cos(t + tau/2) - cos(t + tau))
// with t = t0 + s tau, formed on the device.
constexpr int MAX_STEP_MODES = 6;
struct StepPrepMode {
  const double* master = nullptr;   // complex FP64, n x n, ld = n
  int64_t n = 0;
  const double* x2 = nullptr;       // squared nodes of the mode
  char* out = nullptr;              // step s at out + s * stride
  size_t stride = 0;
  int KBT = 0, MFT = 0, a_exp = 0;
};
struct StepPrep {
  StepPrepMode m[MAX_STEP_MODES];
  int modes = 0, steps = 0;
  double t0 = 0.0, tau = 0.0, eps = 0.0;
};
hipError_t launch_prepare_steps(int prec, const StepPrep& p, hipStream_t s);

// Convert an FP64 master (device, column-major, ld) into fragment order.
// a_exp (FP16X2 only): the pieces represent master * 2^-a_exp.
hipError_t launch_prepare(int prec, int cplx, const double* master, int64_t rows, int64_t cols,
                          int64_t ld, PhaseScale ph, void* out, int KBT, int MFT, hipStream_t s,
                          int a_exp = 0);
// Scale exponent of an operator whose largest |real component| is amax:
// the scaled entries stay below 16 (so hi * 2^11 stays below 2^15).
int fp16x2_op_exp(double amax);
// Device matrix exponential helpers (complex FP64, column-major interleaved,
// n x n): X = f (A + g diag(d)) (d real, nullable); T = I + f W (W null:
// T = I); out[j] = sum_i |(A + g diag(d))_ij|.
hipError_t launch_expm_generator(const double* A, int n, const double* d, double gr, double gi, double fr, double fi,
                                 double* X, hipStream_t s);
hipError_t launch_expm_horner(double* T, const double* W, int n, double f, hipStream_t s);
hipError_t launch_expm_colsum(const double* A, int n, const double* d, double gr, double gi, double* out,
                              hipStream_t s);
// P = W + c[0] I + c[1] X + c[2] X2 + c[3] X3 (W nullable)
hipError_t launch_expm_ps(double* P, const double* W, const double* X, const double* X2, const double* X3, int n,
                          const double* c, hipStream_t s);
// out = Psi diag(exp(-i tau (k + 1/2))) Phi (Phi: K x m, Psi: m x K, real
// FP64 device masters with ld = rows; out: m x m complex FP64 interleaved).
hipError_t launch_hermite_collapse(const double* Phi, const double* Psi, int m, int K, double tau, double* out,
                                   hipStream_t s);
// Exact nonlinear flow of the Section 4.5 vortex problem over time s on a
// complex state (interleaved, d modes, column-major): v <- exp((i s/2)(1 -
// W^-1 |v|^2)) v with W^-1 = prod_k winv[k * 4096 + i_k] (device array).
hipError_t launch_vortex_phase(void* v, int is_f64, int d, const int64_t* dims, const double* winv, double s,
                               hipStream_t st);
// FP16X2 chain start: slots[0] = float bits of max |x_k| over `count` floats,
// slots[1] = slots[2] = 0.  partial: >= norm_partials() words.
hipError_t launch_maxabs(const float* x, int64_t count, uint32_t* partial, uint32_t* slots, hipStream_t s);
size_t prepared_bytes(int prec, int KBT, int MFT);

// Two-pass deterministic FP64 reductions (fp32 or fp64 data):
//   RED_SQ     sum x_k^2 over `count` scalars of x
//   RED_DOT_RE sum Re(conj(x_k) y_k) over `count` complex entries
//   RED_ABS4   sum |x_k|^4 over `count` complex entries
// partial: device buffer of >= norm_partials() doubles.
enum RedKind { RED_SQ = 0, RED_DOT_RE = 1, RED_ABS4 = 2 };
int norm_partials();
hipError_t launch_reduce(int kind, const void* x, const void* y, int64_t count, int is_f64,
                         double* partial, double* result, hipStream_t s);

}  // namespace mm
