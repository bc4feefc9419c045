// Host runtime of the mu-mode library: contexts, prepared operators,
// argument validation and dispatch of the mode-product kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <mutex>

#include "../../include/mumode.h"
#include "mm_internal.h"

// Device memory of gpe_strang_step_noalloc: the FP16X2 running-bound slots
// (3 x SMAX_WORDS words) and the max-abs pass's partial maxima, in a
// file-scope array each GPU holds for the life of the process, so that call
// allocates nothing.  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
constexpr int NOALLOC_SCRATCH_WORDS = 3 * mm::SMAX_WORDS + 1024;
static __device__ __align__(256) uint32_t scratch[NOALLOC_SCRATCH_WORDS];

struct mm_op_s {
  int64_t rows = 0, cols = 0;
  int cplx = 0;
  mm_prec prec = MM_PREC_FP64;
  double* dev_master = nullptr;  // FP64 master on the device, ld = rows
  void* prep = nullptr;          // fragment-order operator (own complexity)
  int KBT = 0, MFT = 0;
  int a_exp = 0;                 // FP16X2: the pieces represent L * 2^-a_exp
  int idsplit = 0;               // the master and pieces hold L - I; products add the input back
  void* prep_c = nullptr;        // real master promoted to complex (lazily)
  int KBT_c = 0, MFT_c = 0;
  double* dev_master_c = nullptr;
  // three-product (Gauss) preparation of a complex split operator: Re L, Im L
  // and Re L + Im L (none for real operators or the identity split)
  void* prep_g = nullptr;
  int JBT_g = 0, MFT_g = 0;
  int a_exp_g = 0;               // FP16X2: scale chosen from max(|Re|, |Im|, |Re + Im|)
};

struct mm_ctx_s {
  int device = 0;
  std::string err;
  std::vector<mm_op> ops;
  void* ws = nullptr;            // ping-pong buffer for products that cannot run in place
  size_t ws_bytes = 0;
  bool ws_user = false;          // ws belongs to the caller (mm_set_workspace)
  // autotuned tile class per problem shape: key (precision, complex, load
  // path, real rows Mr, real columns Kr, fibres F) -> (class, microseconds)
  std::map<std::array<int64_t, 6>, std::pair<int, double>> tune;
  int force_cls = -1;            // set while the autotuner times a class
  std::string tune_path;         // tune cache file (mm_create), "" if none
  std::array<int64_t, 6> last_key{};   // tune key of the last planned product
  bool small_run = true;         // whole-run single-workgroup kernel for small expsteps
  // in-call monitor (MM_OPT_MONITOR_EVERY): sum |T|^2 every mon_every steps
  // of mumode_expstep / gpe_strang_step, kept on the device until the call ends
  int mon_every = 0;
  // MM_OPT_FP16X2_CHAIN: an expstep / GPE call on the tensor the previous
  // such call ended with continues its FP16X2 running bound
  bool keep_chain = false;
  double* mon_dev = nullptr;
  size_t mon_cap = 0;
  std::vector<int> mon_steps;
  std::vector<double> mon_vals;
  double* red_partial = nullptr;
  double* red_result = nullptr;
  double* host_result = nullptr; // pinned
  // FP16X2 state bounds: three slots of SMAX_WORDS words rotate along a
  // chain of products (launch k reads slot k % 3, raises (k + 1) % 3,
  // clears (k + 2) % 3); words [3 SMAX_WORDS, + norm_partials()) are the
  // max-abs pass's partial maxima.  chain_end is the
  // output of the chain's last launch: a product whose input is anything
  // else (or the first one of an API call) starts a new chain with a
  // max-abs pass over its input.
  uint32_t* smax = nullptr;
  uint32_t* smax_static = nullptr;  // device address of `scratch` on this context's device
  const void* chain_end = nullptr;
  int sidx = 0;
  // device matrix exponential scratch: X, T, W (complex FP64 n x n each),
  // the prepared X / T, column sums
  double* ex_buf = nullptr;
  size_t ex_bytes = 0;
  void* ex_prep = nullptr;
  size_t ex_prep_bytes = 0;
  // per-mode scratch for operators re-prepared every step (ho_strang_step)
  void* step_prep[MM_MAXD] = {nullptr};
  size_t step_prep_bytes[MM_MAXD] = {0};
  // ho_strang_step: per mode, the collapsed propagator Psi diag(exp(-i tau
  // (k + 1/2))) Phi (FP64 complex master on the device) for the operators,
  // tau and precision of the last call that formed it
  struct HoMode {
    mm_op phi = nullptr, psi = nullptr;
    double tau = 0.0;
    int prec = -1;
    double* master = nullptr;
    size_t master_bytes = 0;
    mm_op_s op;
  };
  HoMode ho[MM_MAXD];
  double* x2 = nullptr;          // squared node coordinates, MM_MAXD * 4096 doubles
  double* x2_stage = nullptr;    // pinned staging of x2
  hipEvent_t x2_ev = nullptr;    // the last upload from x2_stage
  std::vector<double> x2_nodes[MM_MAXD];   // nodes of the last upload, per mode
  // vortex_strang_step: inverse dual-cell widths per mode (device, MM_MAXD *
  // 4096 doubles), uploaded from pinned staging when the weights change
  double* winv = nullptr;
  double* winv_stage = nullptr;
  hipEvent_t winv_ev = nullptr;
  std::vector<double> winv_w[MM_MAXD];
  // batched integrator: work items of the last batch signature, its
  // launch groups and the captured per-step graph
  struct BatchGroup { mm::ModePlan plan; int ida, offset, count; };
  mm::BatchItem* bitems = nullptr;
  size_t bitems_cap = 0;
  std::vector<BatchGroup> bgroups;
  std::vector<uint64_t> bsig;
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  // tile class of the batched step's products per (mode, complex), chosen by
  // mm_autotune_batched (-1: the planner's choice)
  int batch_cls[MM_MAXD][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}};
  hipStream_t cap_stream = nullptr;
  // optional per-launch timing (mm_profile_begin / mm_profile_end)
  bool profiling = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
};

namespace {

std::string g_create_err;

// Device address of `scratch` per device, looked up once per device with
// that device current.
std::mutex g_scratch_mu;
std::map<int, uint32_t*> g_scratch_addr;

hipError_t scratch_address(int device, uint32_t** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = (uint32_t*)p;
  *out = (uint32_t*)p;
  return hipSuccess;
}

mm_status fail(mm_ctx ctx, mm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else g_create_err = buf;
  return st;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, MM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

int kprec(mm_prec p) {
  switch (p) {
    case MM_PREC_FP64: return mm::KP_F64;
    case MM_PREC_FP32: return mm::KP_F32;
    case MM_PREC_SPLIT_BF16X3: return mm::KP_BF16X3;
    case MM_PREC_SPLIT_FP16X2: return mm::KP_FP16X2;
    default: return mm::KP_BF16;
  }
}

bool is_complex(mm_dtype t) { return t == MM_C64 || t == MM_C128; }
bool is_f64(mm_dtype t) { return t == MM_R64 || t == MM_C128; }
size_t dsize(mm_dtype t) { return t == MM_R32 ? 4 : (t == MM_C128 ? 16 : 8); }

int64_t numel(const mm_tensor* T) {
  int64_t n = 1;
  for (int k = 0; k < T->d; ++k) n *= T->dims[k];
  return n;
}

mm_status check_tensor(mm_ctx ctx, const mm_tensor* T, const char* name) {
  if (!T) return fail(ctx, MM_ERR_ARG, "%s is NULL", name);
  if (T->d < 1 || T->d > MM_MAXD) return fail(ctx, MM_ERR_SHAPE, "%s: d = %d outside [1, %d]", name, T->d, MM_MAXD);
  for (int k = 0; k < T->d; ++k)
    if (T->dims[k] <= 0) return fail(ctx, MM_ERR_SHAPE, "%s: dims[%d] = %lld <= 0", name, k, (long long)T->dims[k]);
  if (T->dtype < MM_R32 || T->dtype > MM_C128) return fail(ctx, MM_ERR_ARG, "%s: bad dtype", name);
  if (!T->data) return fail(ctx, MM_ERR_ARG, "%s: data is NULL", name);
  if (((uintptr_t)T->data) & 15) return fail(ctx, MM_ERR_ALIGN, "%s: data not 16-byte aligned", name);
  if (numel(T) > ((int64_t)1 << 40)) return fail(ctx, MM_ERR_SHAPE, "%s: too many entries", name);
  return MM_OK;
}

bool overlap(const mm_tensor* A, const mm_tensor* B) {
  const char* a0 = (const char*)A->data;
  const char* a1 = a0 + numel(A) * dsize(A->dtype);
  const char* b0 = (const char*)B->data;
  const char* b1 = b0 + numel(B) * dsize(B->dtype);
  return a0 < b1 && b0 < a1;
}

mm_status check_op_dtype(mm_ctx ctx, mm_op L, mm_dtype t) {
  if (L->cplx && !is_complex(t)) return fail(ctx, MM_ERR_DTYPE, "complex operator on a real tensor");
  const bool want64 = L->prec == MM_PREC_FP64;
  if (want64 != is_f64(t))
    return fail(ctx, MM_ERR_DTYPE, "operator precision %d does not match tensor dtype %d", (int)L->prec, (int)t);
  return MM_OK;
}

// Prepare (or reuse) the fragment-order operator for a given complexity.
mm_status ensure_prepared(mm_ctx ctx, mm_op L, bool cplx, hipStream_t s, void** prep, int* KBT, int* MFT) {
  const int kp = kprec(L->prec);
  const int64_t Mr = cplx ? 2 * L->rows : L->rows;
  const int64_t Kr = cplx ? 2 * L->cols : L->cols;
  int kbt = 0, mft = 0;
  mm::op_blocks(kp, Mr, Kr, &kbt, &mft);
  if (cplx == (bool)L->cplx) {
    *prep = L->prep;
    *KBT = L->KBT;
    *MFT = L->MFT;
    return MM_OK;
  }
  // real operator acting on a complex state: promote to complex once
  if (!L->prep_c) {
    const size_t nn = (size_t)L->rows * L->cols;
    std::vector<double> host(nn), cm(2 * nn, 0.0);
    HIPCHK(ctx, hipMemcpy(host.data(), L->dev_master, nn * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t e = 0; e < nn; ++e) cm[2 * e] = host[e];
    HIPCHK(ctx, hipMalloc((void**)&L->dev_master_c, 2 * nn * sizeof(double)));
    HIPCHK(ctx, hipMemcpy(L->dev_master_c, cm.data(), 2 * nn * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMalloc(&L->prep_c, mm::prepared_bytes(kp, kbt, mft)));
    HIPCHK(ctx, mm::launch_prepare(kp, 1, L->dev_master_c, L->rows, L->cols, L->rows, mm::PhaseScale(),
                                   L->prep_c, kbt, mft, s, L->a_exp));
    L->KBT_c = kbt;
    L->MFT_c = mft;
  }
  *prep = L->prep_c;
  *KBT = L->KBT_c;
  *MFT = L->MFT_c;
  return MM_OK;
}

// One mode product out = in x_mu L on a tensor with dims `dims` (input dims),
// optional fused phases.  `in` and `out` may be equal when the plan covers
// all rows in one workgroup (checked by the caller through *in_place_ok).
mm_status run_mode(mm_ctx ctx, const void* in, void* out, const int64_t* dims, int d, mm_dtype dt,
                   mm_op L, int mu, double s_pre, double s_post, hipStream_t s, mm::ModePlan* plan_out,
                   bool dry, const void* prep_override = nullptr, bool batch = false,
                   mm::ModeArgs* args_out = nullptr) {
  // A real operator on a complex state (with no fused phase) acts on the
  // (re, im) planes separately: the state is then the real tensor
  // (2, n_1, ..., n_d) and mode mu its mode mu + 1, i.e. two real fibres per
  // complex one (half the MFMA work of the complex block form, and no
  // promoted copy of the operator).
  const bool rview = !L->cplx && is_complex(dt) && !batch && s_pre == 0.0 && s_post == 0.0 && !prep_override;
  const bool cplx = is_complex(dt) && !rview;
  mm::ModeArgs a;
  int64_t P = rview ? 2 : 1, Q = 1;
  for (int k = 0; k < mu - 1; ++k) P *= dims[k];
  for (int k = mu; k < d; ++k) Q *= dims[k];
  a.in = in;
  a.out = out;
  a.A = nullptr;
  a.P = P;
  a.Q = Q;
  a.F = P * Q;
  a.n = (int)dims[mu - 1];
  a.m = (int)L->rows;
  a.Kr = (cplx ? 2 : 1) * a.n;
  a.Mr = (cplx ? 2 : 1) * a.m;
  a.s_pre = s_pre;
  a.s_post = s_post;
  a.smax_in = nullptr;
  a.smax_out = nullptr;
  a.smax_clr = nullptr;
  a.a_exp = L->a_exp;
  a.idadd = L->idsplit;
  const bool kcontig = (P == 1) && (a.Kr % 8 == 0);
  const bool fcontig = (P % 4 == 0);
  const bool pair = !kcontig && !cplx && P == 2 && a.Kr % 8 == 0;   // as the planner decides
  const int load = kcontig ? mm::KL_KCONTIG : (pair ? mm::KL_PAIR : (fcontig ? mm::KL_FCONTIG : mm::KL_GENERIC));
  // tune key: (precision, complex, load path, rows, columns, fibres); a
  // complex product with the fused prologue phase has its own entry (load
  // path + 8) and falls back to the plain one
  const bool pro_key = cplx && s_pre != 0.0;
  ctx->last_key = {(int64_t)kprec(L->prec), cplx ? 1 : 0, load + (pro_key ? 8 : 0), a.Mr, a.Kr, a.F};
  int force = ctx->force_cls;
  if (force < 0 && !ctx->tune.empty()) {
    auto it = ctx->tune.find(ctx->last_key);
    if (it == ctx->tune.end() && pro_key) {
      std::array<int64_t, 6> plain = ctx->last_key;
      plain[2] = load;
      it = ctx->tune.find(plain);
    }
    if (it != ctx->tune.end()) force = it->second.first;
  }
  // three-product kernels: complex operator with its Gauss preparation,
  // single-tensor products, whole staging tiles of 8 entries
  const bool gauss_ok = L->prep_g && cplx && !batch && !prep_override && !args_out && a.n % 8 == 0;
  mm::ModePlan plan;
  if (!mm::plan_mode(a, kprec(L->prec), cplx ? 1 : 0, s_pre != 0.0, s_post != 0.0, fcontig, kcontig, &plan, batch,
                     force, gauss_ok))
    return fail(ctx, MM_ERR_UNSUPPORTED, "no kernel plan for this shape");
  // batched work items run in place, so each must own all rows of its
  // fibres: a tuned class that splits the rows gives way to the built-in one
  if (batch && !plan.covers_all_rows && force >= 0 &&
      !mm::plan_mode(a, kprec(L->prec), cplx ? 1 : 0, s_pre != 0.0, s_post != 0.0, fcontig, kcontig, &plan, batch,
                     -1))
    return fail(ctx, MM_ERR_UNSUPPORTED, "no kernel plan for this shape");
  if (plan.gauss) {
    a.A = L->prep_g;
    a.KBT = L->JBT_g;
    a.MFT = L->MFT_g;
    a.a_exp = L->a_exp_g;
  } else if (prep_override) {
    a.A = prep_override;
    a.KBT = L->KBT;
    a.MFT = L->MFT;
  } else if (!dry) {
    void* prep = nullptr;
    int KBT = 0, MFT = 0;
    mm_status st = ensure_prepared(ctx, L, cplx, s, &prep, &KBT, &MFT);
    if (st != MM_OK) return st;
    a.A = prep;
    a.KBT = KBT;
    a.MFT = MFT;
  } else {
    mm::op_blocks(kprec(L->prec), a.Mr, a.Kr, &a.KBT, &a.MFT);
  }
  if (plan_out) *plan_out = plan;
  if (args_out) *args_out = a;
  if (dry) return MM_OK;
  if (plan.prec == mm::KP_FP16X2) {
    if (in != ctx->chain_end) {
      int64_t count = is_complex(dt) ? 2 : 1;
      for (int k = 0; k < d; ++k) count *= dims[k];
      HIPCHK(ctx, mm::launch_maxabs((const float*)in, count, ctx->smax + 3 * mm::SMAX_WORDS, ctx->smax, s));
      ctx->sidx = 0;
    }
    a.smax_in = ctx->smax + mm::SMAX_WORDS * ctx->sidx;
    a.smax_out = ctx->smax + mm::SMAX_WORDS * ((ctx->sidx + 1) % 3);
    a.smax_clr = ctx->smax + mm::SMAX_WORDS * ((ctx->sidx + 2) % 3);
    ctx->sidx = (ctx->sidx + 1) % 3;
    ctx->chain_end = out;
  }
  if (ctx->profiling) {
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, mm::launch_mode(plan, a, s, e0, e1));
    const int kind = plan.prec * 1000 + plan.cplx * 100 + plan.load * 10 + plan.pro * 2 + plan.epi;
    ctx->recs.push_back({kind, e0, e1});
    return MM_OK;
  }
  HIPCHK(ctx, mm::launch_mode(plan, a, s));
  return MM_OK;
}

mm_status ensure_ws(mm_ctx ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return MM_OK;
  if (ctx->ws_user)
    return fail(ctx, MM_ERR_NOMEM, "caller workspace of %zu bytes, %zu needed", ctx->ws_bytes, bytes);
  if (ctx->ws) {
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) return fail(ctx, MM_ERR_NOMEM, "workspace of %zu bytes", bytes);
  ctx->ws_bytes = bytes;
  return MM_OK;
}

// Drop the captured batch graph and its signature: its work items hold
// prepared-operator addresses and tile classes, so it must be rebuilt after
// an operator is destroyed or the tile choice changes.
void batch_invalidate(mm_ctx ctx) {
  if (!ctx->bexec && !ctx->bgraph && ctx->bsig.empty()) return;
  hipDeviceSynchronize();
  if (ctx->bexec) hipGraphExecDestroy(ctx->bexec);
  if (ctx->bgraph) hipGraphDestroy(ctx->bgraph);
  ctx->bexec = nullptr;
  ctx->bgraph = nullptr;
  ctx->bsig.clear();
}

// Tucker sweep over the modes with per-mode ops (square), in place on T.
// first_pre / last_post: phase coefficients fused into the first / last
// applied product (0 = none).
mm_status sweep(mm_ctx ctx, mm_tensor* T, const mm_op* E, double first_pre, double last_post, hipStream_t s) {
  int first = -1, last = -1;
  for (int k = 0; k < T->d; ++k)
    if (E[k]) {
      if (first < 0) first = k;
      last = k;
    }
  if (first < 0) return MM_OK;
  const size_t bytes = (size_t)numel(T) * dsize(T->dtype);
  void* cur = T->data;
  for (int k = first; k <= last; ++k) {
    if (!E[k]) continue;
    mm::ModePlan plan;
    mm_status st = run_mode(ctx, cur, cur, T->dims, T->d, T->dtype, E[k], k + 1, 0, 0, s, &plan, true);
    if (st != MM_OK) return st;
    void* dst = cur;
    if (!plan.covers_all_rows) {
      st = ensure_ws(ctx, bytes);
      if (st != MM_OK) return st;
      dst = (cur == T->data) ? ctx->ws : T->data;
    }
    st = run_mode(ctx, cur, dst, T->dims, T->d, T->dtype, E[k], k + 1, k == first ? first_pre : 0.0,
                  k == last ? last_post : 0.0, s, nullptr, false);
    if (st != MM_OK) return st;
    cur = dst;
  }
  if (cur != T->data) {
    HIPCHK(ctx, hipMemcpyAsync(T->data, cur, bytes, hipMemcpyDeviceToDevice, s));
    if (ctx->chain_end == cur) ctx->chain_end = T->data;
  }
  return MM_OK;
}

// Grow a device buffer owned by the context.
mm_status grow(mm_ctx ctx, void** p, size_t* have, size_t need) {
  if (*have >= need) return MM_OK;
  if (*p) {
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, hipFree(*p));
    *p = nullptr;
    *have = 0;
  }
  if (hipMalloc(p, need) != hipSuccess) return fail(ctx, MM_ERR_NOMEM, "scratch of %zu bytes", need);
  *have = need;
  return MM_OK;
}

// A throw-away operator record for products with a device-resident FP64
// master that is prepared by the caller (prep_override of run_mode).
mm_op_s scratch_op(int n, mm_prec prec, int a_exp) {
  mm_op_s o;
  o.rows = o.cols = n;
  o.cplx = 1;
  o.prec = prec;
  o.a_exp = a_exp;
  mm::op_blocks(kprec(prec), 2 * (int64_t)n, 2 * (int64_t)n, &o.KBT, &o.MFT);
  return o;
}

// out = exp(f (A + g diag(d))) for a complex n x n FP64 matrix A on the
// device (d real, nullable), by scaling and squaring of the Taylor
// polynomial: X = f (A + g diag d) / 2^q with ||X||_1 <= 1, the degree-18
// Taylor polynomial (truncation <= e/19! < 2.2e-17) evaluated by the
// Paterson-Stockmeyer scheme with blocks of four terms (X^2, X^3, X^4, then
// Horner in X^4: 7 matrix products instead of 18), then q squarings.  Every
// matrix product is a mode-1 product of the FP64 MFMA kernel.  bound: an
// upper bound of ||A + g diag d||_1 known to the caller, or < 0 to compute
// it here (synchronises s).
mm_status expm_device(mm_ctx ctx, int n, const double* A, const double* d, double gr, double gi, double fr,
                      double fi, double bound, double* out, hipStream_t s) {
  const size_t mat = (size_t)n * n * 2;
  mm_status st = grow(ctx, (void**)&ctx->ex_buf, &ctx->ex_bytes, sizeof(double) * (6 * mat + n));
  if (st != MM_OK) return st;
  mm_op_s op = scratch_op(n, MM_PREC_FP64, 0);
  const size_t pb = mm::prepared_bytes(mm::KP_F64, op.KBT, op.MFT);
  st = grow(ctx, &ctx->ex_prep, &ctx->ex_prep_bytes, 2 * pb);
  if (st != MM_OK) return st;
  double* X = ctx->ex_buf;
  double* X2 = X + mat;
  double* X3 = X2 + mat;
  double* Y = X3 + mat;     // X^4
  double* P = Y + mat;
  double* W = P + mat;
  double* cs = W + mat;
  void* prepX = ctx->ex_prep;
  void* prepY = (char*)ctx->ex_prep + pb;
  if (bound < 0) {
    HIPCHK(ctx, mm::launch_expm_colsum(A, n, d, gr, gi, cs, s));
    std::vector<double> h(n);
    HIPCHK(ctx, hipMemcpyAsync(h.data(), cs, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    bound = 0.0;
    for (double v : h) bound = std::max(bound, v);
  }
  if (!std::isfinite(bound)) return fail(ctx, MM_ERR_NONFINITE, "matrix holds NaN / Inf");
  const double fa = std::hypot(fr, fi) * bound;
  int q = 0;
  if (fa > 1.0) q = (int)std::ceil(std::log2(fa));
  if (q > 1000) return fail(ctx, MM_ERR_ARG, "exponent argument too large (norm %g)", fa);
  const double sc = std::ldexp(1.0, -q);
  const int64_t dims[2] = {n, n};
  // a product of two n x n matrices has only n fibres: where the default
  // FP64 tile would leave most CUs idle (fewer than 128 workgroups), the
  // one-wave tile of class 3 (32 real rows x 16 fibres) runs it
  const bool few = (int64_t)((n + 31) / 32) * ((2 * (int64_t)n + 511) / 512) < 128;
  auto mul = [&](const void* prep, const double* in, double* o) {
    const int keep = ctx->force_cls;
    if (few) ctx->force_cls = 3;
    mm_status r = run_mode(ctx, in, o, dims, 2, MM_C128, &op, 1, 0, 0, s, nullptr, false, prep);
    ctx->force_cls = keep;
    return r;
  };
  HIPCHK(ctx, mm::launch_expm_generator(A, n, d, gr, gi, fr * sc, fi * sc, X, s));
  HIPCHK(ctx, mm::launch_prepare(mm::KP_F64, 1, X, n, n, n, mm::PhaseScale(), prepX, op.KBT, op.MFT, s));
  if ((st = mul(prepX, X, X2)) != MM_OK) return st;
  if ((st = mul(prepX, X2, X3)) != MM_OK) return st;
  if ((st = mul(prepX, X3, Y)) != MM_OK) return st;
  HIPCHK(ctx, mm::launch_prepare(mm::KP_F64, 1, Y, n, n, n, mm::PhaseScale(), prepY, op.KBT, op.MFT, s));
  // coefficients 1/k!, k = 0..18, in blocks B_j = sum_i c_{4j+i} X^i
  double c[20] = {0};
  c[0] = 1.0;
  for (int k = 1; k <= 18; ++k) c[k] = c[k - 1] / k;
  HIPCHK(ctx, mm::launch_expm_ps(P, nullptr, X, X2, X3, n, c + 16, s));
  for (int j = 3; j >= 0; --j) {
    if ((st = mul(prepY, P, W)) != MM_OK) return st;   // P X^4 (polynomials in X commute)
    HIPCHK(ctx, mm::launch_expm_ps(P, W, X, X2, X3, n, c + 4 * j, s));
  }
  double* T = P;
  for (int r = 0; r < q; ++r) {
    HIPCHK(ctx, mm::launch_prepare(mm::KP_F64, 1, T, n, n, n, mm::PhaseScale(), prepX, op.KBT, op.MFT, s));
    if ((st = mul(prepX, T, W)) != MM_OK) return st;
    std::swap(T, W);
  }
  HIPCHK(ctx, hipMemcpyAsync(out, T, sizeof(double) * mat, hipMemcpyDeviceToDevice, s));
  return MM_OK;
}

// In-call monitor: FP64 sum |T|^2 after `step` steps into the next slot of
// the device log (no host synchronisation until monitor_end).
mm_status monitor_begin(mm_ctx ctx, int nsteps) {
  ctx->mon_steps.clear();
  ctx->mon_vals.clear();
  if (ctx->mon_every <= 0 || nsteps <= 0) return MM_OK;
  const size_t need = (size_t)(nsteps / ctx->mon_every + 2);
  if (ctx->mon_cap < need) {
    if (ctx->mon_dev) {
      HIPCHK(ctx, hipDeviceSynchronize());
      HIPCHK(ctx, hipFree(ctx->mon_dev));
      ctx->mon_dev = nullptr;
      ctx->mon_cap = 0;
    }
    if (hipMalloc((void**)&ctx->mon_dev, sizeof(double) * need) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "monitor log");
    ctx->mon_cap = need;
  }
  return MM_OK;
}

mm_status monitor_point(mm_ctx ctx, const mm_tensor* T, int step, hipStream_t s) {
  const size_t k = ctx->mon_steps.size();
  if (k >= ctx->mon_cap) return MM_OK;
  const int64_t count = numel(T) * (is_complex(T->dtype) ? 2 : 1);
  HIPCHK(ctx, mm::launch_reduce(mm::RED_SQ, T->data, nullptr, count, is_f64(T->dtype) ? 1 : 0, ctx->red_partial,
                                ctx->mon_dev + k, s));
  ctx->mon_steps.push_back(step);
  return MM_OK;
}

mm_status monitor_end(mm_ctx ctx, hipStream_t s) {
  const size_t k = ctx->mon_steps.size();
  if (k == 0) return MM_OK;
  ctx->mon_vals.resize(k);
  HIPCHK(ctx, hipMemcpyAsync(ctx->mon_vals.data(), ctx->mon_dev, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  for (size_t i = 0; i < k; ++i)
    if (!std::isfinite(ctx->mon_vals[i]))
      return fail(ctx, MM_ERR_NONFINITE, "sum |T|^2 is not finite after step %d", ctx->mon_steps[i]);
  return MM_OK;
}

// Whole run of a small expstep in one single-workgroup launch, when every
// operator is plain FP64 / FP32, the state is small enough to stay in one
// XCD's L2 (<= 2 MiB) and every mode fits one tile of the small-run class.
// *used = false (and nothing launched) when the problem does not qualify.
mm_status small_expstep(mm_ctx ctx, mm_tensor* T, const mm_op* E, int nsteps, hipStream_t s, bool* used) {
  *used = false;
  // 2-D real FP64 with both modes at most 64 long: state and operators stay
  // in one workgroup's LDS for the whole run
  if (T->d == 2 && T->dtype == MM_R64 && T->dims[0] <= 64 && T->dims[1] <= 64) {
    bool ok = E[0] || E[1];
    for (int k = 0; k < 2; ++k)
      if (E[k]) ok = ok && E[k]->prec == MM_PREC_FP64 && !E[k]->cplx && !E[k]->idsplit;
    if (ok) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (ctx->profiling) {
        HIPCHK(ctx, hipEventCreate(&e0));
        HIPCHK(ctx, hipEventCreate(&e1));
        HIPCHK(ctx, hipEventRecord(e0, s));
      }
      HIPCHK(ctx, mm::launch_small_lds((double*)T->data, (int)T->dims[0], (int)T->dims[1],
                                       E[0] ? E[0]->dev_master : nullptr, E[1] ? E[1]->dev_master : nullptr, nsteps,
                                       s));
      if (ctx->profiling) {
        HIPCHK(ctx, hipEventRecord(e1, s));
        ctx->recs.push_back({mm::KP_F64 * 1000 + 91, e0, e1});
      }
      *used = true;
      return MM_OK;
    }
  }
  const size_t bytes = (size_t)numel(T) * dsize(T->dtype);
  if (bytes > ((size_t)2 << 20) || T->d > 6) return MM_OK;
  const bool cplx = is_complex(T->dtype);
  mm::SmallRun r;
  std::memset(&r, 0, sizeof r);
  r.d = T->d;
  r.nsteps = nsteps;
  int kp = -1;
  for (int k = 0; k < T->d; ++k) {
    if (!E[k]) continue;
    const int p = kprec(E[k]->prec);
    if ((p != mm::KP_F64 && p != mm::KP_F32) || (kp >= 0 && p != kp)) return MM_OK;
    if (cplx && !E[k]->cplx) return MM_OK;   // real operator on complex planes: one launch per product
    if (E[k]->idsplit) return MM_OK;         // identity split: one launch per product
    kp = p;
    mm::ModePlan plan;
    mm::ModeArgs a;
    mm_status st = run_mode(ctx, T->data, T->data, T->dims, T->d, T->dtype, E[k], k + 1, 0, 0, s, &plan, true,
                            nullptr, false, &a);
    if (st != MM_OK) {
      ctx->err.clear();
      return MM_OK;
    }
    // one row tile of the small-run class must hold all rows of the mode
    mm::TileShape t;
    if (!mm::tile_shape(p, SMALL_RUN_CLASS, &t)) return MM_OK;
    const mm::FragGeom fgm = mm::frag_geom(p);
    const int rows = t.WM * t.WMF * fgm.MB;
    const int64_t nt = (int64_t)t.WN * t.WNF * fgm.NB;
    if (a.Mr > rows) return MM_OK;
    plan.grid_x = (int)((a.F + nt - 1) / nt);
    void* prep = nullptr;
    int KBT = 0, MFT = 0;
    st = ensure_prepared(ctx, E[k], cplx, s, &prep, &KBT, &MFT);
    if (st != MM_OK) return st;
    a.A = prep;
    r.m[k] = a;
    r.load[k] = plan.load;
    r.tiles[k] = plan.grid_x;
  }
  if (kp < 0) return MM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->profiling) {
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, hipEventRecord(e0, s));
  }
  HIPCHK(ctx, mm::launch_small_run(kp, cplx ? 1 : 0, r, nullptr, s));
  if (ctx->profiling) {
    HIPCHK(ctx, hipEventRecord(e1, s));
    ctx->recs.push_back({kp * 1000 + (cplx ? 100 : 0) + 90, e0, e1});
  }
  *used = true;
  return MM_OK;
}

}  // namespace

extern "C" {

const char* mm_version(void) { return "mumode-gfx950 0.1"; }

const char* mm_status_string(mm_status s) {
  switch (s) {
    case MM_OK: return "ok";
    case MM_ERR_ARG: return "invalid argument";
    case MM_ERR_SHAPE: return "invalid shape";
    case MM_ERR_DTYPE: return "dtype / precision mismatch";
    case MM_ERR_ALIGN: return "misaligned data";
    case MM_ERR_NOMEM: return "out of device memory";
    case MM_ERR_HIP: return "HIP runtime error";
    case MM_ERR_UNSUPPORTED: return "unsupported";
    case MM_ERR_NONFINITE: return "non-finite value";
    case MM_ERR_NODEVICE: return "no gfx950 device";
  }
  return "unknown status";
}

const char* mm_last_error(mm_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

mm_status mm_create(mm_ctx* out, int device, const char* tune_cache_path) {
  if (!out) return fail(nullptr, MM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(nullptr, MM_ERR_NODEVICE, "no HIP device visible");
  if (device < 0 || device >= count) return fail(nullptr, MM_ERR_NODEVICE, "device %d of %d", device, count);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, MM_ERR_NODEVICE, "device properties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, MM_ERR_NODEVICE, "device %d is %s, not gfx950", device, prop.gcnArchName);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, MM_ERR_HIP, "hipSetDevice");
  mm_ctx c = new mm_ctx_s;
  c->device = device;
  if (hipMalloc((void**)&c->red_partial, sizeof(double) * mm::norm_partials()) != hipSuccess ||
      hipMalloc((void**)&c->red_result, sizeof(double) * 4) != hipSuccess ||
      hipMalloc((void**)&c->smax, sizeof(uint32_t) * (3 * mm::SMAX_WORDS + mm::norm_partials())) != hipSuccess ||
      hipHostMalloc((void**)&c->host_result, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return fail(nullptr, MM_ERR_NOMEM, "context buffers");
  }
  {
    const hipError_t e = scratch_address(device, &c->smax_static);
    if (e != hipSuccess) {
      mm_destroy(c);
      return fail(nullptr, MM_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
  }
  if (tune_cache_path) {
    c->tune_path = tune_cache_path;
    if (FILE* f = std::fopen(tune_cache_path, "r")) {
      std::fclose(f);
      if (mm_tune_load(c, tune_cache_path) != MM_OK) {
        const std::string why = c->err;
        mm_destroy(c);
        return fail(nullptr, MM_ERR_ARG, "tune cache: %s", why.c_str());
      }
    }
  }
  *out = c;
  return MM_OK;
}

mm_status mm_op_destroy(mm_ctx ctx, mm_op op) {
  if (!ctx || !op) return MM_ERR_ARG;
  auto it = std::find(ctx->ops.begin(), ctx->ops.end(), op);
  if (it == ctx->ops.end()) return fail(ctx, MM_ERR_ARG, "operator not owned by this context");
  ctx->ops.erase(it);
  hipSetDevice(ctx->device);
  batch_invalidate(ctx);
  for (int k = 0; k < MM_MAXD; ++k)
    if (ctx->ho[k].phi == op || ctx->ho[k].psi == op) ctx->ho[k].phi = ctx->ho[k].psi = nullptr;
  hipDeviceSynchronize();
  if (op->dev_master) hipFree(op->dev_master);
  if (op->prep) hipFree(op->prep);
  if (op->prep_c) hipFree(op->prep_c);
  if (op->prep_g) hipFree(op->prep_g);
  if (op->dev_master_c) hipFree(op->dev_master_c);
  delete op;
  return MM_OK;
}

mm_status mm_destroy(mm_ctx ctx) {
  if (!ctx) return MM_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  while (!ctx->ops.empty()) mm_op_destroy(ctx, ctx->ops.back());
  for (auto& r : ctx->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  if (ctx->ws && !ctx->ws_user) hipFree(ctx->ws);
  for (int k = 0; k < MM_MAXD; ++k)
    if (ctx->step_prep[k]) hipFree(ctx->step_prep[k]);
  if (ctx->x2) hipFree(ctx->x2);
  if (ctx->x2_stage) hipHostFree(ctx->x2_stage);
  if (ctx->x2_ev) hipEventDestroy(ctx->x2_ev);
  if (ctx->winv) hipFree(ctx->winv);
  if (ctx->winv_stage) hipHostFree(ctx->winv_stage);
  if (ctx->winv_ev) hipEventDestroy(ctx->winv_ev);
  for (int k = 0; k < MM_MAXD; ++k)
    if (ctx->ho[k].master) hipFree(ctx->ho[k].master);
  if (ctx->bexec) hipGraphExecDestroy(ctx->bexec);
  if (ctx->bgraph) hipGraphDestroy(ctx->bgraph);
  if (ctx->bitems) hipFree(ctx->bitems);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  if (ctx->red_partial) hipFree(ctx->red_partial);
  if (ctx->red_result) hipFree(ctx->red_result);
  if (ctx->smax) hipFree(ctx->smax);
  if (ctx->mon_dev) hipFree(ctx->mon_dev);
  if (ctx->ex_buf) hipFree(ctx->ex_buf);
  if (ctx->ex_prep) hipFree(ctx->ex_prep);
  if (ctx->host_result) hipHostFree(ctx->host_result);
  delete ctx;
  return MM_OK;
}

mm_status mm_op_prepare(mm_ctx ctx, const mm_matrix* M, mm_prec prec, mm_op* out) {
  return mm_op_prepare_ex(ctx, M, prec, 0u, out);
}

mm_status mm_op_prepare_ex(mm_ctx ctx, const mm_matrix* M, mm_prec prec, unsigned flags, mm_op* out) {
  if (!ctx) return MM_ERR_ARG;
  if (!M || !out || !M->data) return fail(ctx, MM_ERR_ARG, "NULL matrix or output");
  *out = nullptr;
  if (flags & ~(unsigned)MM_OP_IDENTITY_SPLIT) return fail(ctx, MM_ERR_ARG, "unknown operator flags 0x%x", flags);
  const bool idsplit = (flags & MM_OP_IDENTITY_SPLIT) != 0;
  if (idsplit && M->rows != M->cols) return fail(ctx, MM_ERR_SHAPE, "identity split needs a square operator");
  if (M->dtype != MM_R64 && M->dtype != MM_C128) return fail(ctx, MM_ERR_DTYPE, "master must be MM_R64 or MM_C128");
  if (prec < MM_PREC_FP64 || prec > MM_PREC_BF16) return fail(ctx, MM_ERR_ARG, "bad precision");
  if (M->rows < 1 || M->cols < 1 || M->rows > 4096 || M->cols > 4096)
    return fail(ctx, MM_ERR_SHAPE, "operator %lld x %lld outside [1, 4096]", (long long)M->rows, (long long)M->cols);
  if (M->ld < M->rows) return fail(ctx, MM_ERR_SHAPE, "ld < rows");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  const int cplx = M->dtype == MM_C128;
  const int comps = cplx ? 2 : 1;
  // compact host copy (ld = rows)
  std::vector<double> host((size_t)M->rows * M->cols * comps);
  if (M->on_device) {
    std::vector<double> full((size_t)M->ld * M->cols * comps);
    HIPCHK(ctx, hipMemcpy(full.data(), M->data, full.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < M->cols; ++j)
      std::memcpy(&host[(size_t)j * M->rows * comps], &full[(size_t)j * M->ld * comps], sizeof(double) * M->rows * comps);
  } else {
    const double* src = (const double*)M->data;
    for (int64_t j = 0; j < M->cols; ++j)
      std::memcpy(&host[(size_t)j * M->rows * comps], src + (size_t)j * M->ld * comps, sizeof(double) * M->rows * comps);
  }
  for (double v : host)
    if (!std::isfinite(v)) return fail(ctx, MM_ERR_NONFINITE, "operator holds NaN / Inf");
  if (idsplit)   // L - I in FP64: the products carry only the departure from identity
    for (int64_t i = 0; i < M->rows; ++i) host[((size_t)i * M->rows + i) * comps] -= 1.0;
  double amax = 0.0;
  for (double v : host) amax = std::max(amax, std::fabs(v));
  mm_op op = new mm_op_s;
  op->rows = M->rows;
  op->cols = M->cols;
  op->cplx = cplx;
  op->prec = prec;
  op->idsplit = idsplit ? 1 : 0;
  op->a_exp = prec == MM_PREC_SPLIT_FP16X2 ? mm::fp16x2_op_exp(amax) : 0;
  const int kp = kprec(prec);
  mm::op_blocks(kp, comps * M->rows, comps * M->cols, &op->KBT, &op->MFT);
  // the three-product form of a complex split operator is prepared with it
  // (no product call allocates): Re L, Im L and Re L + Im L
  const bool gauss = cplx && !idsplit && (kp == mm::KP_FP16X2 || kp == mm::KP_BF16X3);
  if (gauss) {
    double gmax = 0.0;
    for (size_t e = 0; e + 1 < host.size(); e += 2)
      gmax = std::max(gmax, std::max(std::fabs(host[e]), std::max(std::fabs(host[e + 1]), std::fabs(host[e] + host[e + 1]))));
    op->a_exp_g = kp == mm::KP_FP16X2 ? mm::fp16x2_op_exp(gmax) : 0;
    mm::gauss_blocks(op->rows, op->cols, &op->JBT_g, &op->MFT_g);
  }
  if (hipMalloc((void**)&op->dev_master, host.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&op->prep, mm::prepared_bytes(kp, op->KBT, op->MFT)) != hipSuccess ||
      (gauss && hipMalloc(&op->prep_g, mm::gauss_prepared_bytes(kp, op->JBT_g, op->MFT_g)) != hipSuccess)) {
    if (op->dev_master) hipFree(op->dev_master);
    if (op->prep) hipFree(op->prep);
    delete op;
    return fail(ctx, MM_ERR_NOMEM, "operator buffers");
  }
  ctx->ops.push_back(op);
  HIPCHK(ctx, hipMemcpy(op->dev_master, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(ctx, mm::launch_prepare(kp, cplx, op->dev_master, op->rows, op->cols, op->rows, mm::PhaseScale(),
                                 op->prep, op->KBT, op->MFT, 0, op->a_exp));
  if (gauss)
    HIPCHK(ctx, mm::launch_prepare_gauss(kp, op->dev_master, op->rows, op->cols, op->rows, op->prep_g, op->JBT_g,
                                         op->MFT_g, op->a_exp_g, 0));
  HIPCHK(ctx, hipDeviceSynchronize());
  *out = op;
  return MM_OK;
}

mm_status mm_op_flags(mm_op op, unsigned* flags) {
  if (!op || !flags) return MM_ERR_ARG;
  *flags = op->idsplit ? (unsigned)MM_OP_IDENTITY_SPLIT : 0u;
  return MM_OK;
}

mm_status mm_op_info(mm_op op, int64_t* rows, int64_t* cols, int* is_complex_, mm_prec* prec) {
  if (!op) return MM_ERR_ARG;
  if (rows) *rows = op->rows;
  if (cols) *cols = op->cols;
  if (is_complex_) *is_complex_ = op->cplx;
  if (prec) *prec = op->prec;
  return MM_OK;
}

mm_status mumode_apply(mm_ctx ctx, mm_tensor* out, const mm_tensor* T, mm_op L, int mu, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, T, "T");
  if (st != MM_OK) return st;
  st = check_tensor(ctx, out, "out");
  if (st != MM_OK) return st;
  if (!L) return fail(ctx, MM_ERR_ARG, "operator is NULL");
  if (mu < 1 || mu > T->d) return fail(ctx, MM_ERR_SHAPE, "mu = %d outside [1, %d]", mu, T->d);
  if (L->cols != T->dims[mu - 1])
    return fail(ctx, MM_ERR_SHAPE, "operator has %lld columns, n_mu = %lld", (long long)L->cols, (long long)T->dims[mu - 1]);
  if (out->d != T->d || out->dtype != T->dtype) return fail(ctx, MM_ERR_SHAPE, "out must have T's order and dtype");
  for (int k = 0; k < T->d; ++k) {
    const int64_t want = (k == mu - 1) ? L->rows : T->dims[k];
    if (out->dims[k] != want) return fail(ctx, MM_ERR_SHAPE, "out dims[%d] = %lld, expected %lld", k, (long long)out->dims[k], (long long)want);
  }
  st = check_op_dtype(ctx, L, T->dtype);
  if (st != MM_OK) return st;
  if (overlap(out, T)) return fail(ctx, MM_ERR_ARG, "out overlaps T");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  return run_mode(ctx, T->data, out->data, T->dims, T->d, T->dtype, L, mu, 0, 0, (hipStream_t)stream, nullptr, false);
}

mm_status mumode_expstep(mm_ctx ctx, mm_tensor* T, const mm_op* E, int nsteps, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  ctx->mon_steps.clear();
  ctx->mon_vals.clear();
  mm_status st = check_tensor(ctx, T, "T");
  if (st != MM_OK) return st;
  if (!E) return fail(ctx, MM_ERR_ARG, "E is NULL");
  if (nsteps < 0) return fail(ctx, MM_ERR_ARG, "nsteps < 0");
  for (int k = 0; k < T->d; ++k) {
    if (!E[k]) continue;
    if (E[k]->rows != E[k]->cols || E[k]->cols != T->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "E[%d] must be %lld x %lld", k, (long long)T->dims[k], (long long)T->dims[k]);
    st = check_op_dtype(ctx, E[k], T->dtype);
    if (st != MM_OK) return st;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (!ctx->keep_chain || T->data != ctx->chain_end) ctx->chain_end = nullptr;
  if (ctx->small_run && nsteps >= 2 && ctx->mon_every <= 0) {
    bool used = false;
    st = small_expstep(ctx, T, E, nsteps, (hipStream_t)stream, &used);
    if (st != MM_OK || used) return st;
  }
  st = monitor_begin(ctx, nsteps);
  if (st != MM_OK) return st;
  for (int it = 0; it < nsteps; ++it) {
    st = sweep(ctx, T, E, 0.0, 0.0, (hipStream_t)stream);
    if (st != MM_OK) return st;
    if (ctx->mon_every > 0 && ((it + 1) % ctx->mon_every == 0 || it + 1 == nsteps)) {
      st = monitor_point(ctx, T, it + 1, (hipStream_t)stream);
      if (st != MM_OK) return st;
    }
  }
  return monitor_end(ctx, (hipStream_t)stream);
}

mm_status mumode_transform(mm_ctx ctx, mm_tensor* out, const mm_tensor* in, const mm_op* Phi, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, in, "in");
  if (st != MM_OK) return st;
  st = check_tensor(ctx, out, "out");
  if (st != MM_OK) return st;
  if (!Phi) return fail(ctx, MM_ERR_ARG, "Phi is NULL");
  if (out->d != in->d || out->dtype != in->dtype) return fail(ctx, MM_ERR_SHAPE, "out must have in's order and dtype");
  for (int k = 0; k < in->d; ++k) {
    if (Phi[k]) {
      if (Phi[k]->cols != in->dims[k]) return fail(ctx, MM_ERR_SHAPE, "Phi[%d] has %lld columns, expected %lld", k, (long long)Phi[k]->cols, (long long)in->dims[k]);
      st = check_op_dtype(ctx, Phi[k], in->dtype);
      if (st != MM_OK) return st;
    }
    const int64_t want = Phi[k] ? Phi[k]->rows : in->dims[k];
    if (out->dims[k] != want) return fail(ctx, MM_ERR_SHAPE, "out dims[%d] = %lld, expected %lld", k, (long long)out->dims[k], (long long)want);
  }
  if (overlap(out, in)) return fail(ctx, MM_ERR_ARG, "out overlaps in");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  // chain of rectangular products: in -> A -> B -> ... -> out, where the
  // intermediate tensors live in the workspace (two halves) and the last
  // product writes out.
  int last = -1, count = 0;
  for (int k = 0; k < in->d; ++k)
    if (Phi[k]) {
      last = k;
      ++count;
    }
  const size_t es = dsize(in->dtype);
  if (count == 0) {
    HIPCHK(ctx, hipMemcpyAsync(out->data, in->data, (size_t)numel(in) * es, hipMemcpyDeviceToDevice, s));
    return MM_OK;
  }
  // largest intermediate
  int64_t dims[MM_MAXD];
  for (int k = 0; k < in->d; ++k) dims[k] = in->dims[k];
  size_t maxb = 0;
  for (int k = 0; k < in->d; ++k) {
    if (!Phi[k]) continue;
    dims[k] = Phi[k]->rows;
    int64_t n = 1;
    for (int q = 0; q < in->d; ++q) n *= dims[q];
    maxb = std::max(maxb, (size_t)n * es);
  }
  const size_t half = (maxb + 255) / 256 * 256;
  if (count > 1) {
    st = ensure_ws(ctx, 2 * half);
    if (st != MM_OK) return st;
  }
  for (int k = 0; k < in->d; ++k) dims[k] = in->dims[k];
  const void* cur = in->data;
  int pp = 0;
  for (int k = 0; k < in->d; ++k) {
    if (!Phi[k]) continue;
    void* dst = (k == last) ? out->data : (void*)((char*)ctx->ws + pp * half);
    st = run_mode(ctx, cur, dst, dims, in->d, in->dtype, Phi[k], k + 1, 0, 0, s, nullptr, false);
    if (st != MM_OK) return st;
    dims[k] = Phi[k]->rows;
    cur = dst;
    pp ^= 1;
  }
  return MM_OK;
}

namespace {

mm_status gpe_strang_impl(mm_ctx ctx, mm_tensor* psi, const mm_op* E, double tau, double beta, int nsteps,
                          hipStream_t s, bool noalloc) {
  if (!ctx) return MM_ERR_ARG;
  ctx->mon_steps.clear();
  ctx->mon_vals.clear();
  mm_status st = check_tensor(ctx, psi, "psi");
  if (st != MM_OK) return st;
  if (!is_complex(psi->dtype)) return fail(ctx, MM_ERR_DTYPE, "psi must be complex");
  if (!E) return fail(ctx, MM_ERR_ARG, "E is NULL");
  if (nsteps < 0) return fail(ctx, MM_ERR_ARG, "nsteps < 0");
  if (!std::isfinite(tau) || !std::isfinite(beta)) return fail(ctx, MM_ERR_ARG, "tau / beta not finite");
  for (int k = 0; k < psi->d; ++k) {
    if (!E[k]) return fail(ctx, MM_ERR_ARG, "E[%d] is NULL", k);
    if (E[k]->rows != E[k]->cols || E[k]->cols != psi->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "E[%d] must be %lld x %lld", k, (long long)psi->dims[k], (long long)psi->dims[k]);
    st = check_op_dtype(ctx, E[k], psi->dtype);
    if (st != MM_OK) return st;
    if (noalloc && !E[k]->cplx)
      return fail(ctx, MM_ERR_UNSUPPORTED, "E[%d] is real: the allocation-free step takes complex operators", k);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (noalloc || !ctx->keep_chain || psi->data != ctx->chain_end) ctx->chain_end = nullptr;
  const double half = 0.5 * tau * beta, full = tau * beta;
  if (noalloc) {
    // every product must run in place (no workspace), i.e. its plan must
    // give one workgroup all rows of its fibres; checked for each plan the
    // sweeps below use (phase in the first product, in the last one only on
    // the last step)
    for (int k = 0; k < psi->d; ++k)
      for (int lastep = 0; lastep < 2; ++lastep) {
        mm::ModePlan plan;
        const double pre = k == 0 ? half : 0.0;
        const double post = (k == psi->d - 1 && lastep) ? half : 0.0;
        st = run_mode(ctx, psi->data, psi->data, psi->dims, psi->d, psi->dtype, E[k], k + 1, pre, post, s, &plan,
                      true);
        if (st != MM_OK) return st;
        if (!plan.covers_all_rows)
          return fail(ctx, MM_ERR_SHAPE,
                      "n_%d = %lld: the allocation-free step runs every product in place, which needs "
                      "n_mu <= 256", k + 1, (long long)psi->dims[k]);
      }
  }
  // merged steps: N(tau/2) [L N(tau)]^(nsteps-1) L N(tau/2); each N(tau)
  // between steps is fused into the staging of the next step's first product
  // (where it overlaps MFMA work), the last N(tau/2) into the final epilogue
  if (!noalloc) {
    st = monitor_begin(ctx, nsteps);
    if (st != MM_OK) return st;
  }
  for (int it = 0; it < nsteps; ++it) {
    const double pre = (it == 0) ? half : full;
    const double post = (it + 1 < nsteps) ? 0.0 : half;
    st = sweep(ctx, psi, E, pre, post, s);
    if (st != MM_OK) return st;
    // the phase flows keep |psi|, so the mass between merged steps is the
    // mass after the step
    if (!noalloc && ctx->mon_every > 0 && ((it + 1) % ctx->mon_every == 0 || it + 1 == nsteps)) {
      st = monitor_point(ctx, psi, it + 1, s);
      if (st != MM_OK) return st;
    }
  }
  return noalloc ? MM_OK : monitor_end(ctx, s);
}

}  // namespace

mm_status gpe_strang_step(mm_ctx ctx, mm_tensor* psi, const mm_op* E, double tau, double beta, int nsteps,
                          mm_stream stream) {
  return gpe_strang_impl(ctx, psi, E, tau, beta, nsteps, (hipStream_t)stream, false);
}

mm_status gpe_strang_step_noalloc(mm_ctx ctx, mm_tensor* psi, const mm_op* E, double tau, double beta, int nsteps,
                                  mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  if (3 * mm::SMAX_WORDS + mm::norm_partials() > NOALLOC_SCRATCH_WORDS)
    return fail(ctx, MM_ERR_UNSUPPORTED, "scratch array smaller than the FP16X2 bound slots and partials");
  // the running-bound slots and max-abs partials of the FP16X2 products come
  // from `scratch` (every chain starts with the max-abs pass, which writes
  // all of them, so nothing needs clearing); no monitor, no per-launch events
  uint32_t* own = ctx->smax;
  const bool prof = ctx->profiling;
  ctx->smax = ctx->smax_static;
  ctx->profiling = false;
  const mm_status st = gpe_strang_impl(ctx, psi, E, tau, beta, nsteps, (hipStream_t)stream, true);
  ctx->smax = own;
  ctx->profiling = prof;
  ctx->chain_end = nullptr;
  return st;
}

mm_status ho_strang_step(mm_ctx ctx, mm_tensor* psi, const mm_op* Phi_fwd, const mm_op* Psi_bwd,
                         const double* const* nodes, double t0, double tau, double eps, int nsteps, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, psi, "psi");
  if (st != MM_OK) return st;
  if (!is_complex(psi->dtype)) return fail(ctx, MM_ERR_DTYPE, "psi must be complex");
  if (!Phi_fwd || !Psi_bwd || !nodes) return fail(ctx, MM_ERR_ARG, "Phi_fwd / Psi_bwd / nodes is NULL");
  if (nsteps < 0) return fail(ctx, MM_ERR_ARG, "nsteps < 0");
  if (!std::isfinite(t0) || !std::isfinite(tau) || !std::isfinite(eps)) return fail(ctx, MM_ERR_ARG, "t0 / tau / eps not finite");
  for (int k = 0; k < psi->d; ++k) {
    const mm_op F = Phi_fwd[k], B = Psi_bwd[k];
    if (!F || !B || !nodes[k]) return fail(ctx, MM_ERR_ARG, "Phi_fwd[%d] / Psi_bwd[%d] / nodes[%d] is NULL", k, k, k);
    if (F->cplx || B->cplx) return fail(ctx, MM_ERR_DTYPE, "Phi_fwd[%d] / Psi_bwd[%d] must be real", k, k);
    if (F->idsplit || B->idsplit)
      return fail(ctx, MM_ERR_ARG, "Phi_fwd[%d] / Psi_bwd[%d]: prepared with the identity split", k, k);
    if (F->prec != B->prec) return fail(ctx, MM_ERR_DTYPE, "Phi_fwd[%d] and Psi_bwd[%d] differ in precision", k, k);
    if (F->cols != psi->dims[k] || B->rows != psi->dims[k] || F->rows != B->cols || F->rows > F->cols)
      return fail(ctx, MM_ERR_SHAPE, "mode %d: Phi_fwd must be K x %lld and Psi_bwd %lld x K, K <= %lld", k + 1,
                  (long long)psi->dims[k], (long long)psi->dims[k], (long long)psi->dims[k]);
    st = check_op_dtype(ctx, F, psi->dtype);
    if (st != MM_OK) return st;
    for (int64_t i = 0; i < psi->dims[k]; ++i)
      if (!std::isfinite(nodes[k][i])) return fail(ctx, MM_ERR_ARG, "nodes[%d] holds NaN / Inf", k);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  // the collapsed propagators of this tau, formed on the device once per
  // (operators, tau, precision)
  for (int k = 0; k < psi->d; ++k) {
    mm_ctx_s::HoMode& H = ctx->ho[k];
    const mm_op F = Phi_fwd[k], B = Psi_bwd[k];
    if (H.phi == F && H.psi == B && H.tau == tau && H.prec == (int)F->prec) continue;
    const int n = (int)psi->dims[k];
    st = grow(ctx, (void**)&H.master, &H.master_bytes, sizeof(double) * 2 * (size_t)n * n);
    if (st != MM_OK) return st;
    HIPCHK(ctx, mm::launch_hermite_collapse(F->dev_master, B->dev_master, n, (int)F->rows, tau, H.master, s));
    H.op = scratch_op(n, F->prec, 0);
    H.op.dev_master = H.master;
    if (F->prec == MM_PREC_SPLIT_FP16X2) {
      // operator scale from the largest entry (one read-back per formation)
      std::vector<double> h((size_t)2 * n * n);
      HIPCHK(ctx, hipMemcpyAsync(h.data(), H.master, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      double amax = 0.0;
      for (double v : h) amax = std::max(amax, std::fabs(v));
      H.op.a_exp = mm::fp16x2_op_exp(amax);
    }
    H.phi = F;
    H.psi = B;
    H.tau = tau;
    H.prec = (int)F->prec;
  }
  // squared node coordinates, uploaded when the nodes change (from pinned
  // staging, once the previous upload from it has completed)
  if (!ctx->x2) {
    if (hipMalloc((void**)&ctx->x2, sizeof(double) * MM_MAXD * 4096) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "node buffer");
    if (hipHostMalloc((void**)&ctx->x2_stage, sizeof(double) * MM_MAXD * 4096, hipHostMallocDefault) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "node staging");
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->x2_ev, hipEventDisableTiming));
  }
  bool changed = false;
  for (int k = 0; k < psi->d && !changed; ++k)
    changed = ctx->x2_nodes[k].size() != (size_t)psi->dims[k] ||
              std::memcmp(ctx->x2_nodes[k].data(), nodes[k], sizeof(double) * psi->dims[k]) != 0;
  if (changed) {
    HIPCHK(ctx, hipEventSynchronize(ctx->x2_ev));
    for (int k = 0; k < MM_MAXD; ++k) ctx->x2_nodes[k].clear();
    for (int k = 0; k < psi->d; ++k) {
      ctx->x2_nodes[k].assign(nodes[k], nodes[k] + psi->dims[k]);
      for (int64_t i = 0; i < psi->dims[k]; ++i) ctx->x2_stage[(size_t)k * 4096 + i] = nodes[k][i] * nodes[k][i];
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->x2, ctx->x2_stage, sizeof(double) * psi->d * 4096, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipEventRecord(ctx->x2_ev, s));
  }
  // per-step operators, prepared for blocks of up to 32 steps (and at most
  // 64 MiB) in one launch per precision, so no preparation sits between the
  // products of a step; without the time-dependent potential (eps = 0) they
  // are the same every step and are prepared once
  size_t need[MM_MAXD];
  size_t per_step = 0;
  for (int k = 0; k < psi->d; ++k) {
    const mm_op_s& L = ctx->ho[k].op;
    need[k] = (mm::prepared_bytes(kprec(L.prec), L.KBT, L.MFT) + 255) / 256 * 256;
    per_step += need[k];
  }
  int blk = eps != 0.0 ? std::min(nsteps, 32) : 1;
  while (blk > 1 && per_step * blk > ((size_t)64 << 20)) blk /= 2;
  blk = std::max(blk, 1);
  for (int k = 0; k < psi->d; ++k) {
    const size_t want = need[k] * blk;
    if (ctx->step_prep_bytes[k] < want) {
      if (ctx->step_prep[k]) {
        HIPCHK(ctx, hipDeviceSynchronize());
        HIPCHK(ctx, hipFree(ctx->step_prep[k]));
        ctx->step_prep[k] = nullptr;
        ctx->step_prep_bytes[k] = 0;
      }
      if (hipMalloc(&ctx->step_prep[k], want) != hipSuccess) return fail(ctx, MM_ERR_NOMEM, "step operators");
      ctx->step_prep_bytes[k] = want;
    }
  }
  auto prepare_block = [&](int it0, int steps) -> mm_status {
    // one launch per precision group of modes
    bool done[MM_MAXD] = {false};
    for (int k0 = 0; k0 < psi->d; ++k0) {
      if (done[k0]) continue;
      mm::StepPrep p;
      p.steps = steps;
      p.t0 = t0 + it0 * tau;
      p.tau = tau;
      p.eps = eps;
      for (int k = k0; k < psi->d && p.modes < mm::MAX_STEP_MODES; ++k) {
        if (done[k] || ctx->ho[k].op.prec != ctx->ho[k0].op.prec) continue;
        const mm_op_s& L = ctx->ho[k].op;
        mm::StepPrepMode& m = p.m[p.modes++];
        m.master = L.dev_master;
        m.n = L.rows;
        m.x2 = ctx->x2 + (size_t)k * 4096;
        m.out = (char*)ctx->step_prep[k];
        m.stride = need[k];
        m.KBT = L.KBT;
        m.MFT = L.MFT;
        m.a_exp = L.a_exp;
        done[k] = true;
      }
      HIPCHK(ctx, mm::launch_prepare_steps(kprec(ctx->ho[k0].op.prec), p, s));
    }
    return MM_OK;
  };
  const size_t bytes = (size_t)numel(psi) * dsize(psi->dtype);
  int blk0 = 0;   // first step of the prepared block
  for (int it = 0; it < nsteps; ++it) {
    if (it == 0 || (eps != 0.0 && it - blk0 >= blk)) {
      blk0 = it;
      st = prepare_block(it, eps != 0.0 ? std::min(blk, nsteps - it) : 1);
      if (st != MM_OK) return st;
    }
    const size_t sidx = eps != 0.0 ? (size_t)(it - blk0) : 0;
    void* cur = psi->data;
    for (int k = 0; k < psi->d; ++k) {
      mm_op_s* L = &ctx->ho[k].op;
      const void* prep = (const char*)ctx->step_prep[k] + sidx * need[k];
      mm::ModePlan plan;
      st = run_mode(ctx, cur, cur, psi->dims, psi->d, psi->dtype, L, k + 1, 0, 0, s, &plan, true);
      if (st != MM_OK) return st;
      void* dst = cur;
      if (!plan.covers_all_rows) {
        st = ensure_ws(ctx, bytes);
        if (st != MM_OK) return st;
        dst = (cur == psi->data) ? ctx->ws : psi->data;
      }
      st = run_mode(ctx, cur, dst, psi->dims, psi->d, psi->dtype, L, k + 1, 0, 0, s, nullptr, false, prep);
      if (st != MM_OK) return st;
      cur = dst;
    }
    if (cur != psi->data) {
      HIPCHK(ctx, hipMemcpyAsync(psi->data, cur, bytes, hipMemcpyDeviceToDevice, s));
      if (ctx->chain_end == cur) ctx->chain_end = psi->data;
    }
  }
  return MM_OK;
}

mm_status vortex_strang_step(mm_ctx ctx, mm_tensor* v, const mm_op* E, const double* const* w, double tau, int nsteps,
                             mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, v, "v");
  if (st != MM_OK) return st;
  if (!is_complex(v->dtype)) return fail(ctx, MM_ERR_DTYPE, "v must be complex");
  if (!E || !w) return fail(ctx, MM_ERR_ARG, "E / w is NULL");
  if (nsteps < 0) return fail(ctx, MM_ERR_ARG, "nsteps < 0");
  if (!std::isfinite(tau)) return fail(ctx, MM_ERR_ARG, "tau not finite");
  for (int k = 0; k < v->d; ++k) {
    if (!E[k] || !w[k]) return fail(ctx, MM_ERR_ARG, "E[%d] / w[%d] is NULL", k, k);
    if (E[k]->rows != E[k]->cols || E[k]->cols != v->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "E[%d] must be %lld x %lld", k, (long long)v->dims[k], (long long)v->dims[k]);
    if (v->dims[k] > 4096) return fail(ctx, MM_ERR_SHAPE, "n_%d > 4096", k + 1);
    st = check_op_dtype(ctx, E[k], v->dtype);
    if (st != MM_OK) return st;
    for (int64_t i = 0; i < v->dims[k]; ++i)
      if (!(w[k][i] > 0.0) || !std::isfinite(w[k][i])) return fail(ctx, MM_ERR_ARG, "w[%d][%lld] not a positive width", k, (long long)i);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (nsteps == 0) return MM_OK;
  if (!ctx->winv) {
    if (hipMalloc((void**)&ctx->winv, sizeof(double) * MM_MAXD * 4096) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "weight buffer");
    if (hipHostMalloc((void**)&ctx->winv_stage, sizeof(double) * MM_MAXD * 4096, hipHostMallocDefault) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "weight staging");
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->winv_ev, hipEventDisableTiming));
  }
  bool changed = false;
  for (int k = 0; k < v->d && !changed; ++k)
    changed = ctx->winv_w[k].size() != (size_t)v->dims[k] ||
              std::memcmp(ctx->winv_w[k].data(), w[k], sizeof(double) * v->dims[k]) != 0;
  if (changed) {
    HIPCHK(ctx, hipEventSynchronize(ctx->winv_ev));
    for (int k = 0; k < MM_MAXD; ++k) ctx->winv_w[k].clear();
    for (int k = 0; k < v->d; ++k) {
      ctx->winv_w[k].assign(w[k], w[k] + v->dims[k]);
      for (int64_t i = 0; i < v->dims[k]; ++i) ctx->winv_stage[(size_t)k * 4096 + i] = 1.0 / w[k][i];
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->winv, ctx->winv_stage, sizeof(double) * v->d * 4096, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipEventRecord(ctx->winv_ev, s));
  }
  const int f64 = is_f64(v->dtype) ? 1 : 0;
  // merged steps N(tau/2) [L N(tau)]^(nsteps-1) L N(tau/2): N keeps |v|, so
  // adjacent half steps compose; each N is one pass over the state (its
  // coefficient depends on the position through W^-1).  FP16X2: a rotation
  // raises a component by at most sqrt(2), which the state scale's headroom
  // covers (as for the fused prologue phase), so the running bound of the
  // last product carries over the pass to the next step's first product
  HIPCHK(ctx, mm::launch_vortex_phase(v->data, f64, v->d, v->dims, ctx->winv, 0.5 * tau, s));
  for (int it = 0; it < nsteps; ++it) {
    st = sweep(ctx, v, E, 0.0, 0.0, s);
    if (st != MM_OK) return st;
    HIPCHK(ctx, mm::launch_vortex_phase(v->data, f64, v->d, v->dims, ctx->winv, it + 1 < nsteps ? tau : 0.5 * tau, s));
  }
  ctx->chain_end = nullptr;
  return MM_OK;
}

mm_status mumode_expstep_batched(mm_ctx ctx, int count, mm_tensor* const* T, const mm_op* const* E, int nsteps,
                                 mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  if (count < 0 || nsteps < 0) return fail(ctx, MM_ERR_ARG, "count / nsteps < 0");
  if (count == 0 || nsteps == 0) return MM_OK;
  if (!T || !E) return fail(ctx, MM_ERR_ARG, "T / E is NULL");
  mm_status st;
  for (int i = 0; i < count; ++i) {
    char nm[32];
    snprintf(nm, sizeof nm, "T[%d]", i);
    st = check_tensor(ctx, T[i], nm);
    if (st != MM_OK) return st;
    if (!E[i]) return fail(ctx, MM_ERR_ARG, "E[%d] is NULL", i);
    for (int k = 0; k < T[i]->d; ++k) {
      mm_op L = E[i][k];
      if (!L) continue;
      if (L->rows != L->cols || L->cols != T[i]->dims[k])
        return fail(ctx, MM_ERR_SHAPE, "E[%d][%d] must be %lld x %lld", i, k, (long long)T[i]->dims[k], (long long)T[i]->dims[k]);
      st = check_op_dtype(ctx, L, T[i]->dtype);
      if (st != MM_OK) return st;
      if (L->prec == MM_PREC_SPLIT_FP16X2)
        return fail(ctx, MM_ERR_UNSUPPORTED, "E[%d][%d]: the batched step has no FP16X2 kernels "
                                             "(a state bound per instance would be needed)", i, k);
    }
    for (int j = 0; j < i; ++j)
      if (overlap(T[i], T[j])) return fail(ctx, MM_ERR_ARG, "T[%d] overlaps T[%d]", i, j);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  // signature of the batch: tensors and operators
  std::vector<uint64_t> sig;
  sig.push_back((uint64_t)count);
  for (int i = 0; i < count; ++i) {
    sig.push_back((uint64_t)(uintptr_t)T[i]->data);
    sig.push_back((uint64_t)T[i]->d * 16 + (uint64_t)T[i]->dtype);
    for (int k = 0; k < T[i]->d; ++k) {
      const mm_op L = E[i][k];
      sig.push_back((uint64_t)T[i]->dims[k]);
      sig.push_back((uint64_t)(uintptr_t)L);
      sig.push_back(L ? (uint64_t)L->prec : ~(uint64_t)0);
      sig.push_back(L ? (uint64_t)(uintptr_t)L->prep : 0);
    }
  }
  if (sig != ctx->bsig || !ctx->bexec) {
    // build the work items: per mode, one group per kernel (precision,
    // complexity, load path, tile class); every product runs in place
    std::vector<mm::BatchItem> items;
    std::vector<mm_ctx_s::BatchGroup> groups;
    for (int k = 0; k < MM_MAXD; ++k) {
      std::vector<std::pair<uint64_t, std::vector<mm::BatchItem>>> byk;
      std::vector<mm::ModePlan> plans;
      for (int i = 0; i < count; ++i) {
        if (k >= T[i]->d || !E[i][k]) continue;
        mm_op L = E[i][k];
        mm::ModePlan plan;
        const int forced = ctx->batch_cls[k][is_complex(T[i]->dtype) ? 1 : 0];
        const int keep_force = ctx->force_cls;
        if (forced >= 0) ctx->force_cls = forced;
        st = run_mode(ctx, T[i]->data, T[i]->data, T[i]->dims, T[i]->d, T[i]->dtype, L, k + 1, 0, 0, s, &plan, true,
                      nullptr, true);
        ctx->force_cls = keep_force;
        if (st != MM_OK) return st;
        if (!plan.covers_all_rows || plan.load == mm::KL_GENERIC)
          return fail(ctx, MM_ERR_UNSUPPORTED, "batched step needs n_mu <= 256 (complex) / 512 (real) and "
                                               "aligned fibres (instance %d, mode %d)", i, k + 1);
        void* prep = nullptr;
        int KBT = 0, MFT = 0;
        st = ensure_prepared(ctx, L, is_complex(T[i]->dtype), s, &prep, &KBT, &MFT);
        if (st != MM_OK) return st;
        mm::ModeArgs a;
        int64_t P = 1, Q = 1;
        for (int q = 0; q < k; ++q) P *= T[i]->dims[q];
        for (int q = k + 1; q < T[i]->d; ++q) Q *= T[i]->dims[q];
        const bool cplx = is_complex(T[i]->dtype);
        a.in = T[i]->data;
        a.out = T[i]->data;
        a.A = prep;
        a.P = P;
        a.Q = Q;
        a.F = P * Q;
        a.n = (int)T[i]->dims[k];
        a.m = (int)L->rows;
        a.Kr = (cplx ? 2 : 1) * a.n;
        a.Mr = (cplx ? 2 : 1) * a.m;
        a.KBT = KBT;
        a.MFT = MFT;
        a.s_pre = 0.0;
        a.s_post = 0.0;
        a.smax_in = nullptr;
        a.smax_out = nullptr;
        a.smax_clr = nullptr;
        a.a_exp = 0;
        a.idadd = L->idsplit;
        // one merged launch per (mode, precision, identity split); the item's
        // kind selects its tile code
        const uint64_t key = (uint64_t)plan.prec * 2 + (L->idsplit ? 1 : 0);
        const int kind = plan.cplx * 100 + plan.load * 10 + plan.cls;
        size_t g = 0;
        while (g < byk.size() && byk[g].first != key) ++g;
        if (g == byk.size()) {
          byk.push_back({key, {}});
          plans.push_back(plan);
        }
        for (int tx = 0; tx < plan.grid_x; ++tx) byk[g].second.push_back(mm::BatchItem{a, tx, 0, kind});
      }
      for (size_t g = 0; g < byk.size(); ++g) {
        // longest tiles first (work ~ K x M of the instance's product), so the
        // launch does not end on a few large tiles started last; the items
        // are independent, so the order changes no result
        std::stable_sort(byk[g].second.begin(), byk[g].second.end(),
                         [](const mm::BatchItem& x, const mm::BatchItem& y) {
                           return (int64_t)x.a.Kr * x.a.Mr > (int64_t)y.a.Kr * y.a.Mr;
                         });
        groups.push_back({plans[g], (int)(byk[g].first & 1), (int)items.size(), (int)byk[g].second.size()});
        items.insert(items.end(), byk[g].second.begin(), byk[g].second.end());
      }
    }
    if (items.size() > ctx->bitems_cap) {
      if (ctx->bitems) {
        HIPCHK(ctx, hipDeviceSynchronize());
        HIPCHK(ctx, hipFree(ctx->bitems));
        ctx->bitems = nullptr;
        ctx->bitems_cap = 0;
      }
      if (hipMalloc((void**)&ctx->bitems, items.size() * sizeof(mm::BatchItem)) != hipSuccess)
        return fail(ctx, MM_ERR_NOMEM, "batch work items");
      ctx->bitems_cap = items.size();
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    HIPCHK(ctx, hipMemcpy(ctx->bitems, items.data(), items.size() * sizeof(mm::BatchItem), hipMemcpyHostToDevice));
    ctx->bgroups = groups;
    // capture one step (all modes, all groups) as a graph
    if (ctx->bexec) {
      HIPCHK(ctx, hipGraphExecDestroy(ctx->bexec));
      ctx->bexec = nullptr;
    }
    if (ctx->bgraph) {
      HIPCHK(ctx, hipGraphDestroy(ctx->bgraph));
      ctx->bgraph = nullptr;
    }
    ctx->bsig.clear();
    if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (const auto& g : ctx->bgroups) {
      le = mm::launch_mode_batch_merged(g.plan.prec, g.ida, ctx->bitems + g.offset, g.count, ctx->cap_stream);
      if (le != hipSuccess) break;
    }
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(ctx, MM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
    }
    ctx->bgraph = graph;
    HIPCHK(ctx, hipGraphInstantiate(&ctx->bexec, ctx->bgraph, nullptr, nullptr, 0));
    ctx->bsig = sig;
  }
  for (int it = 0; it < nsteps; ++it) HIPCHK(ctx, hipGraphLaunch(ctx->bexec, s));
  return MM_OK;
}

mm_status mm_energy_gpe(mm_ctx ctx, const mm_tensor* psi, const mm_op* H, double beta, double cell,
                        double* host_out, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, psi, "psi");
  if (st != MM_OK) return st;
  if (!is_complex(psi->dtype)) return fail(ctx, MM_ERR_DTYPE, "psi must be complex");
  if (!H || !host_out) return fail(ctx, MM_ERR_ARG, "H / host_out is NULL");
  for (int k = 0; k < psi->d; ++k) {
    if (!H[k]) return fail(ctx, MM_ERR_ARG, "H[%d] is NULL", k);
    if (H[k]->rows != H[k]->cols || H[k]->cols != psi->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "H[%d] must be %lld x %lld", k, (long long)psi->dims[k], (long long)psi->dims[k]);
    st = check_op_dtype(ctx, H[k], psi->dtype);
    if (st != MM_OK) return st;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)numel(psi) * dsize(psi->dtype);
  st = ensure_ws(ctx, bytes);
  if (st != MM_OK) return st;
  const int64_t count = numel(psi);
  const int f64 = is_f64(psi->dtype) ? 1 : 0;
  double total = 0.0;
  for (int k = 0; k < psi->d; ++k) {
    st = run_mode(ctx, psi->data, ctx->ws, psi->dims, psi->d, psi->dtype, H[k], k + 1, 0, 0, s, nullptr, false);
    if (st != MM_OK) return st;
    HIPCHK(ctx, mm::launch_reduce(mm::RED_DOT_RE, psi->data, ctx->ws, count, f64, ctx->red_partial, ctx->red_result, s));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    total += ctx->host_result[0];
  }
  HIPCHK(ctx, mm::launch_reduce(mm::RED_ABS4, psi->data, nullptr, count, f64, ctx->red_partial, ctx->red_result, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  const double e = cell * (total + 0.5 * beta * ctx->host_result[0]);
  *host_out = e;
  if (!std::isfinite(e)) return fail(ctx, MM_ERR_NONFINITE, "energy is not finite");
  return MM_OK;
}

mm_status mm_profile_begin(mm_ctx ctx) {
  if (!ctx) return MM_ERR_ARG;
  for (auto& r : ctx->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ctx->recs.clear();
  ctx->profiling = true;
  return MM_OK;
}

mm_status mm_profile_end(mm_ctx ctx, int max_records, int* count, int* kinds, double* ms) {
  if (!ctx || !count) return MM_ERR_ARG;
  ctx->profiling = false;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  int n = 0;
  for (auto& r : ctx->recs) {
    HIPCHK(ctx, hipEventSynchronize(r.b));
    if (n < max_records && kinds && ms) {
      float t = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&t, r.a, r.b));
      kinds[n] = r.kind;
      ms[n] = t;
    }
    ++n;
  }
  for (auto& r : ctx->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ctx->recs.clear();
  *count = n;
  return MM_OK;
}

mm_status mm_norm2(mm_ctx ctx, const mm_tensor* T, double cell, double* host_out, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, T, "T");
  if (st != MM_OK) return st;
  if (!host_out) return fail(ctx, MM_ERR_ARG, "host_out is NULL");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int64_t count = numel(T) * (is_complex(T->dtype) ? 2 : 1);
  HIPCHK(ctx, mm::launch_reduce(mm::RED_SQ, T->data, nullptr, count, is_f64(T->dtype) ? 1 : 0, ctx->red_partial,
                                ctx->red_result, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  const double v = ctx->host_result[0] * cell;
  *host_out = v;
  if (!std::isfinite(v)) return fail(ctx, MM_ERR_NONFINITE, "norm is not finite");
  return MM_OK;
}

mm_status mm_set_workspace(mm_ctx ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return MM_ERR_ARG;
  if (dev_ptr && ((uintptr_t)dev_ptr & 255)) return fail(ctx, MM_ERR_ALIGN, "workspace not 256-byte aligned");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipDeviceSynchronize());
  if (ctx->ws && !ctx->ws_user) HIPCHK(ctx, hipFree(ctx->ws));
  ctx->ws = dev_ptr;
  ctx->ws_bytes = dev_ptr ? bytes : 0;
  ctx->ws_user = dev_ptr != nullptr;
  return MM_OK;
}

mm_status mm_autotune(mm_ctx ctx, const mm_tensor* T, const mm_op* E, int budget_ms, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, T, "T");
  if (st != MM_OK) return st;
  if (!E) return fail(ctx, MM_ERR_ARG, "E is NULL");
  if (budget_ms < 1) budget_ms = 1;
  for (int k = 0; k < T->d; ++k) {
    if (!E[k]) continue;
    if (E[k]->cols != T->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "E[%d] has %lld columns, n_%d = %lld", k, (long long)E[k]->cols, k + 1,
                  (long long)T->dims[k]);
    st = check_op_dtype(ctx, E[k], T->dtype);
    if (st != MM_OK) return st;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const bool cplx = is_complex(T->dtype);
  int modes = 0;
  for (int k = 0; k < T->d; ++k) modes += E[k] ? 1 : 0;
  if (modes == 0) return MM_OK;
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { hipEventDestroy(a); hipEventDestroy(b); }
  } guard{e0, e1};
  const double per_mode_ms = (double)budget_ms / modes;
  for (int k = 0; k < T->d; ++k) {
    mm_op L = E[k];
    if (!L) continue;
    // product of mode k+1 of T, out of place into the workspace
    int64_t odims[MM_MAXD];
    for (int q = 0; q < T->d; ++q) odims[q] = T->dims[q];
    odims[k] = L->rows;
    int64_t onum = 1;
    for (int q = 0; q < T->d; ++q) onum *= odims[q];
    st = ensure_ws(ctx, (size_t)onum * dsize(T->dtype));
    if (st != MM_OK) return st;
    const int kp = kprec(L->prec);
    const int ncls = mm::num_classes(kp);
    std::vector<int> cands;
    for (int c = 0; c < ncls; ++c) {
      mm::ModePlan plan;
      ctx->force_cls = c;
      st = run_mode(ctx, T->data, ctx->ws, T->dims, T->d, T->dtype, L, k + 1, 0, 0, s, &plan, true);
      ctx->force_cls = -1;
      if (st == MM_OK && plan.cls == c) cands.push_back(c);
    }
    if (cands.empty()) continue;
    // complex products with a complex operator are timed a second time with
    // the fused prologue phase (the first product of a Gross-Pitaevskii
    // step): the phase adds VALU work to the staging, which changes which
    // tile shape is fastest, so that choice is recorded under its own key
    const bool with_pro = cplx && L->cplx;
    const double per_cand_ms = per_mode_ms / cands.size() / (with_pro ? 2 : 1);
    for (int pass = 0; pass < (with_pro ? 2 : 1); ++pass) {
      const double s_pre = pass ? 1e-3 : 0.0;
      int best = -1;
      double best_ms = 0.0;
      std::array<int64_t, 6> key{};
      for (int c : cands) {
        ctx->force_cls = c;
        mm::ModePlan plan;
        if (pass) {   // classes without instances that carry the phase
          st = run_mode(ctx, T->data, ctx->ws, T->dims, T->d, T->dtype, L, k + 1, s_pre, 0, s, &plan, true);
          if (st != MM_OK || plan.cls != c) {
            ctx->err.clear();
            ctx->force_cls = -1;
            st = MM_OK;
            continue;
          }
        }
        // first launch: warm-up (and, for FP16X2, the bound of T in slot 0)
        ctx->chain_end = nullptr;
        st = run_mode(ctx, T->data, ctx->ws, T->dims, T->d, T->dtype, L, k + 1, s_pre, 0, s, &plan, false);
        if (st == MM_OK) {
          key = ctx->last_key;
          HIPCHK(ctx, hipEventRecord(e0, s));
          ctx->chain_end = T->data;
          ctx->sidx = 0;
          st = run_mode(ctx, T->data, ctx->ws, T->dims, T->d, T->dtype, L, k + 1, s_pre, 0, s, nullptr, false);
          HIPCHK(ctx, hipEventRecord(e1, s));
        }
        if (st != MM_OK) {
          ctx->force_cls = -1;
          return st;
        }
        HIPCHK(ctx, hipEventSynchronize(e1));
        float t1 = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t1, e0, e1));
        int reps = (int)std::min(20.0, std::max(2.0, per_cand_ms / std::max(1e-3, (double)t1)));
        HIPCHK(ctx, hipEventRecord(e0, s));
        for (int r = 0; r < reps && st == MM_OK; ++r) {
          ctx->chain_end = T->data;   // every repetition reads the bound of T (slot 0)
          ctx->sidx = 0;
          st = run_mode(ctx, T->data, ctx->ws, T->dims, T->d, T->dtype, L, k + 1, s_pre, 0, s, nullptr, false);
        }
        HIPCHK(ctx, hipEventRecord(e1, s));
        ctx->force_cls = -1;
        if (st != MM_OK) return st;
        HIPCHK(ctx, hipEventSynchronize(e1));
        float tr = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&tr, e0, e1));
        const double avg = (double)tr / reps;
        if (best < 0 || avg < best_ms) {
          best = c;
          best_ms = avg;
        }
      }
      if (best >= 0) ctx->tune[key] = {best, best_ms * 1e3};
    }
  }
  batch_invalidate(ctx);
  ctx->chain_end = nullptr;
  if (!ctx->tune_path.empty()) return mm_tune_save(ctx, ctx->tune_path.c_str());
  return MM_OK;
}

mm_status mm_autotune_batched(mm_ctx ctx, int count, mm_tensor* const* T, const mm_op* const* E, int budget_ms,
                              mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  if (count <= 0) return MM_OK;
  hipStream_t s = (hipStream_t)stream;
  // the (mode, complex) groups present in the batch
  bool present[MM_MAXD][2] = {};
  for (int i = 0; i < count; ++i) {
    if (!T || !T[i] || !E || !E[i]) return fail(ctx, MM_ERR_ARG, "T / E entry %d is NULL", i);
    for (int k = 0; k < T[i]->d && k < MM_MAXD; ++k)
      if (E[i][k]) present[k][is_complex(T[i]->dtype) ? 1 : 0] = true;
  }
  for (int k = 0; k < MM_MAXD; ++k) ctx->batch_cls[k][0] = ctx->batch_cls[k][1] = -1;
  batch_invalidate(ctx);
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { hipEventDestroy(a); hipEventDestroy(b); }
  } guard{e0, e1};
  // one captured step per candidate: a warm-up replay, then reps timed replays
  auto time_step = [&](double* ms) -> mm_status {
    mm_status st = mumode_expstep_batched(ctx, count, T, E, 1, stream);
    if (st != MM_OK) return st;
    HIPCHK(ctx, hipEventRecord(e0, s));
    st = mumode_expstep_batched(ctx, count, T, E, 1, stream);
    if (st != MM_OK) return st;
    HIPCHK(ctx, hipEventRecord(e1, s));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float t1 = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&t1, e0, e1));
    const int reps = (int)std::min(10.0, std::max(2.0, (double)budget_ms / 24.0 / std::max(1e-3, (double)t1)));
    HIPCHK(ctx, hipEventRecord(e0, s));
    st = mumode_expstep_batched(ctx, count, T, E, reps, stream);
    if (st != MM_OK) return st;
    HIPCHK(ctx, hipEventRecord(e1, s));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float tr = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&tr, e0, e1));
    *ms = (double)tr / reps;
    return MM_OK;
  };
  double best_ms = 0.0;
  mm_status st = time_step(&best_ms);
  if (st != MM_OK) return st;
  // coordinate descent over the groups: each group's class in turn, the
  // others held at their current choice
  for (int k = 0; k < MM_MAXD; ++k)
    for (int c = 0; c < 2; ++c) {
      if (!present[k][c]) continue;
      int best = -1;
      for (int cls = 0; cls <= 2; ++cls) {
        ctx->batch_cls[k][c] = cls;
        batch_invalidate(ctx);
        double ms = 0.0;
        st = time_step(&ms);
        if (st == MM_ERR_UNSUPPORTED) {
          ctx->err.clear();
          continue;
        }
        if (st != MM_OK) {
          ctx->batch_cls[k][c] = best;
          batch_invalidate(ctx);
          return st;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = cls;
        }
      }
      ctx->batch_cls[k][c] = best;
      batch_invalidate(ctx);
    }
  return MM_OK;
}

mm_status mm_autotune_batched_get(mm_ctx ctx, int mode, int is_complex_, int* cls) {
  if (!ctx || !cls || mode < 1 || mode > MM_MAXD || is_complex_ < 0 || is_complex_ > 1) return MM_ERR_ARG;
  *cls = ctx->batch_cls[mode - 1][is_complex_];
  return MM_OK;
}

mm_status mm_tune_count(mm_ctx ctx, int* count) {
  if (!ctx || !count) return MM_ERR_ARG;
  *count = (int)ctx->tune.size();
  return MM_OK;
}

mm_status mm_tune_get(mm_ctx ctx, int index, int64_t* key6, int* cls, double* us) {
  if (!ctx || index < 0 || index >= (int)ctx->tune.size()) return MM_ERR_ARG;
  auto it = ctx->tune.begin();
  std::advance(it, index);
  if (key6)
    for (int q = 0; q < 6; ++q) key6[q] = it->first[q];
  if (cls) *cls = it->second.first;
  if (us) *us = it->second.second;
  return MM_OK;
}

mm_status mm_tune_clear(mm_ctx ctx) {
  if (!ctx) return MM_ERR_ARG;
  batch_invalidate(ctx);
  ctx->tune.clear();
  for (int k = 0; k < MM_MAXD; ++k) ctx->batch_cls[k][0] = ctx->batch_cls[k][1] = -1;
  return MM_OK;
}

mm_status mm_tune_save(mm_ctx ctx, const char* path) {
  if (!ctx || !path) return MM_ERR_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(ctx, MM_ERR_ARG, "cannot write %s", path);
  std::fprintf(f, "mumode-tune 1\n");
  for (const auto& e : ctx->tune)
    std::fprintf(f, "%lld %lld %lld %lld %lld %lld %d %.3f\n", (long long)e.first[0], (long long)e.first[1],
                 (long long)e.first[2], (long long)e.first[3], (long long)e.first[4], (long long)e.first[5],
                 e.second.first, e.second.second);
  const bool ok = std::fclose(f) == 0;
  return ok ? MM_OK : fail(ctx, MM_ERR_ARG, "write of %s failed", path);
}

mm_status mm_tune_load(mm_ctx ctx, const char* path) {
  if (!ctx || !path) return MM_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, MM_ERR_ARG, "cannot read %s", path);
  char head[32] = {0};
  int ver = 0;
  if (std::fscanf(f, "%31s %d", head, &ver) != 2 || std::strcmp(head, "mumode-tune") != 0 || ver != 1) {
    std::fclose(f);
    return fail(ctx, MM_ERR_ARG, "%s is not a tune file", path);
  }
  std::map<std::array<int64_t, 6>, std::pair<int, double>> t;
  long long k[6];
  int c;
  double us;
  int n;
  while ((n = std::fscanf(f, "%lld %lld %lld %lld %lld %lld %d %lf", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &c,
                          &us)) == 8) {
    if (k[0] < 0 || k[0] > mm::KP_BF16 || c < 0 || c >= mm::num_classes((int)k[0])) {
      std::fclose(f);
      return fail(ctx, MM_ERR_ARG, "%s: bad entry", path);
    }
    t[{k[0], k[1], k[2], k[3], k[4], k[5]}] = {c, us};
  }
  const bool eof = n == EOF;
  std::fclose(f);
  if (!eof) return fail(ctx, MM_ERR_ARG, "%s: malformed line", path);
  batch_invalidate(ctx);
  for (const auto& e : t) ctx->tune[e.first] = e.second;
  return MM_OK;
}

mm_status mm_expm_device(mm_ctx ctx, int n, const double* A, double c_re, double c_im, double* out,
                         mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  if (!A || !out) return fail(ctx, MM_ERR_ARG, "A / out is NULL");
  if (n < 1 || n > 4096) return fail(ctx, MM_ERR_SHAPE, "n = %d outside [1, 4096]", n);
  if (((uintptr_t)A & 15) || ((uintptr_t)out & 15)) return fail(ctx, MM_ERR_ALIGN, "A / out not 16-byte aligned");
  if (!std::isfinite(c_re) || !std::isfinite(c_im)) return fail(ctx, MM_ERR_ARG, "c not finite");
  const char* a0 = (const char*)A;
  const char* o0 = (const char*)out;
  const size_t bytes = sizeof(double) * 2 * (size_t)n * n;
  if (a0 < o0 + bytes && o0 < a0 + bytes) return fail(ctx, MM_ERR_ARG, "out overlaps A");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  return expm_device(ctx, n, A, nullptr, 0.0, 0.0, c_re, c_im, -1.0, out, (hipStream_t)stream);
}

mm_status mumode_magnus_step(mm_ctx ctx, mm_tensor* T, const mm_matrix* B, const double* const* dg, const double* g,
                             double tau, int nsteps, mm_prec prec, mm_stream stream) {
  if (!ctx) return MM_ERR_ARG;
  mm_status st = check_tensor(ctx, T, "T");
  if (st != MM_OK) return st;
  if (!is_complex(T->dtype)) return fail(ctx, MM_ERR_DTYPE, "T must be complex");
  if (!B) return fail(ctx, MM_ERR_ARG, "B is NULL");
  if (nsteps < 0) return fail(ctx, MM_ERR_ARG, "nsteps < 0");
  if (!std::isfinite(tau)) return fail(ctx, MM_ERR_ARG, "tau not finite");
  if (prec < MM_PREC_FP64 || prec > MM_PREC_BF16) return fail(ctx, MM_ERR_ARG, "bad precision");
  if ((prec == MM_PREC_FP64) != is_f64(T->dtype))
    return fail(ctx, MM_ERR_DTYPE, "precision %d does not match tensor dtype %d", (int)prec, (int)T->dtype);
  const int d = T->d;
  bool any_t = false;
  for (int k = 0; k < d; ++k) {
    if (!B[k].data) continue;
    if (B[k].rows != T->dims[k] || B[k].cols != T->dims[k])
      return fail(ctx, MM_ERR_SHAPE, "B[%d] must be %lld x %lld", k, (long long)T->dims[k], (long long)T->dims[k]);
    if (B[k].dtype != MM_C128 && B[k].dtype != MM_R64) return fail(ctx, MM_ERR_DTYPE, "B[%d] must be MM_C128 or MM_R64", k);
    if (B[k].ld < B[k].rows) return fail(ctx, MM_ERR_SHAPE, "B[%d]: ld < rows", k);
    if (dg && dg[k]) any_t = true;
  }
  if (any_t && !g) return fail(ctx, MM_ERR_ARG, "g is NULL but a mode has a time-dependent part");
  if (nsteps == 0) return MM_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->chain_end = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int kp = kprec(prec);
  // per-mode device state: FP64 complex master, diagonal, exponential,
  // prepared exponential
  struct Mode {
    int n = 0;
    double* Bd = nullptr;
    double* dd = nullptr;
    double* E = nullptr;
    void* P = nullptr;
    double bnorm = 0.0, dmax = 0.0;
    // Gershgorin discs of the Hermitian part (B + B^H)/2: centres Re b_ii,
    // radii sum_{j != i} |b_ij + conj(b_ji)| / 2
    std::vector<double> hc, hr;
    mm_op_s op;
  };
  std::vector<Mode> modes(d);
  struct Guard {
    std::vector<Mode>* m;
    ~Guard() {
      hipDeviceSynchronize();
      for (auto& x : *m) {
        if (x.Bd) hipFree(x.Bd);
        if (x.dd) hipFree(x.dd);
        if (x.E) hipFree(x.E);
        if (x.P) hipFree(x.P);
      }
    }
  } guard{&modes};
  for (int k = 0; k < d; ++k) {
    if (!B[k].data) continue;
    Mode& M = modes[k];
    const int n = (int)T->dims[k];
    M.n = n;
    const int comps = B[k].dtype == MM_C128 ? 2 : 1;
    std::vector<double> full((size_t)B[k].ld * n * comps), host((size_t)n * n * 2, 0.0);
    if (B[k].on_device)
      HIPCHK(ctx, hipMemcpy(full.data(), B[k].data, full.size() * sizeof(double), hipMemcpyDeviceToHost));
    else
      std::memcpy(full.data(), B[k].data, full.size() * sizeof(double));
    std::vector<double> colsum(n, 0.0);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double re = full[((size_t)j * B[k].ld + i) * comps];
        const double im = comps == 2 ? full[((size_t)j * B[k].ld + i) * 2 + 1] : 0.0;
        if (!std::isfinite(re) || !std::isfinite(im)) return fail(ctx, MM_ERR_NONFINITE, "B[%d] holds NaN / Inf", k);
        host[2 * ((size_t)j * n + i)] = re;
        host[2 * ((size_t)j * n + i) + 1] = im;
        colsum[j] += std::hypot(re, im);
      }
    for (double v : colsum) M.bnorm = std::max(M.bnorm, v);
    M.hc.assign(n, 0.0);
    M.hr.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
      M.hc[i] = host[2 * ((size_t)i * n + i)];
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        const double re = host[2 * ((size_t)j * n + i)] + host[2 * ((size_t)i * n + j)];
        const double im = host[2 * ((size_t)j * n + i) + 1] - host[2 * ((size_t)i * n + j) + 1];
        M.hr[i] += 0.5 * std::hypot(re, im);
      }
    }
    if (hipMalloc((void**)&M.Bd, host.size() * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&M.E, host.size() * sizeof(double)) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "mode buffers");
    HIPCHK(ctx, hipMemcpy(M.Bd, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
    if (dg && dg[k]) {
      for (int i = 0; i < n; ++i) {
        if (!std::isfinite(dg[k][i])) return fail(ctx, MM_ERR_NONFINITE, "d[%d] holds NaN / Inf", k);
        M.dmax = std::max(M.dmax, std::fabs(dg[k][i]));
      }
      if (hipMalloc((void**)&M.dd, sizeof(double) * n) != hipSuccess) return fail(ctx, MM_ERR_NOMEM, "diagonal");
      HIPCHK(ctx, hipMemcpy(M.dd, dg[k], sizeof(double) * n, hipMemcpyHostToDevice));
    }
    M.op = scratch_op(n, prec, 0);
    if (hipMalloc(&M.P, mm::prepared_bytes(kp, M.op.KBT, M.op.MFT)) != hipSuccess)
      return fail(ctx, MM_ERR_NOMEM, "prepared operator");
  }
  const size_t bytes = (size_t)numel(T) * dsize(T->dtype);
  for (int it = 0; it < nsteps; ++it) {
    void* cur = T->data;
    for (int k = 0; k < d; ++k) {
      Mode& M = modes[k];
      if (!M.Bd) continue;
      if (it == 0 || M.dd) {
        // E_k = exp(tau (B_k + g diag d_k)) at the midpoint of the step
        double gr = 0.0, gi = 0.0;
        if (M.dd) {
          gr = g[2 * ((size_t)it * d + k)];
          gi = g[2 * ((size_t)it * d + k) + 1];
          if (!std::isfinite(gr) || !std::isfinite(gi)) return fail(ctx, MM_ERR_NONFINITE, "g not finite");
        }
        const double bound = M.bnorm + std::hypot(gr, gi) * M.dmax;
        st = expm_device(ctx, M.n, M.Bd, M.dd, gr, gi, tau, 0.0, bound, M.E, s);
        if (st != MM_OK) return st;
        // FP16X2 operator scale from a bound of max |E_ij|: |E_ij| <= ||E||_2
        // <= exp(tau mu(A)) with mu the logarithmic 2-norm, the largest
        // eigenvalue of the Hermitian part of A = B + g diag(d) (that part is
        // (B + B^H)/2 + Re(g) diag(d)), bounded by its Gershgorin discs; for
        // tau < 0 the same with -A.  For a skew-Hermitian (unitary-flow)
        // generator the bound is 1, the true size of the entries.
        if (prec == MM_PREC_SPLIT_FP16X2) {
          double mu = -HUGE_VAL;
          const double sg = tau >= 0.0 ? 1.0 : -1.0;
          for (int i = 0; i < M.n; ++i) {
            const double c = M.hc[i] + (M.dd ? gr * dg[k][i] : 0.0);
            mu = std::max(mu, sg * c + M.hr[i]);
          }
          M.op.a_exp = mm::fp16x2_op_exp(std::exp(std::min(700.0, std::fabs(tau) * mu)));
        } else {
          M.op.a_exp = 0;
        }
        HIPCHK(ctx, mm::launch_prepare(kp, 1, M.E, M.n, M.n, M.n, mm::PhaseScale(), M.P, M.op.KBT, M.op.MFT, s,
                                       M.op.a_exp));
      }
      mm::ModePlan plan;
      st = run_mode(ctx, cur, cur, T->dims, d, T->dtype, &M.op, k + 1, 0, 0, s, &plan, true, M.P);
      if (st != MM_OK) return st;
      void* dst = cur;
      if (!plan.covers_all_rows) {
        st = ensure_ws(ctx, bytes);
        if (st != MM_OK) return st;
        dst = (cur == T->data) ? ctx->ws : T->data;
      }
      st = run_mode(ctx, cur, dst, T->dims, d, T->dtype, &M.op, k + 1, 0, 0, s, nullptr, false, M.P);
      if (st != MM_OK) return st;
      cur = dst;
    }
    if (cur != T->data) {
      HIPCHK(ctx, hipMemcpyAsync(T->data, cur, bytes, hipMemcpyDeviceToDevice, s));
      if (ctx->chain_end == cur) ctx->chain_end = T->data;
    }
  }
  return MM_OK;
}

mm_status mm_set_option(mm_ctx ctx, int option, int64_t value) {
  if (!ctx) return MM_ERR_ARG;
  switch (option) {
    case MM_OPT_SMALL_RUN:
      ctx->small_run = value != 0;
      return MM_OK;
    case MM_OPT_MONITOR_EVERY:
      if (value < 0 || value > (1 << 30)) return fail(ctx, MM_ERR_ARG, "monitor interval %lld", (long long)value);
      ctx->mon_every = (int)value;
      return MM_OK;
    case MM_OPT_FP16X2_CHAIN:
      if (value != 0 && value != 1) return fail(ctx, MM_ERR_ARG, "MM_OPT_FP16X2_CHAIN takes 0 or 1");
      ctx->keep_chain = value != 0;
      ctx->chain_end = nullptr;
      return MM_OK;
    default:
      return fail(ctx, MM_ERR_ARG, "unknown option %d", option);
  }
}

mm_status mm_monitor_log(mm_ctx ctx, int max_records, int* count, int* steps, double* sums) {
  if (!ctx || !count) return MM_ERR_ARG;
  const int k = (int)ctx->mon_vals.size();
  for (int i = 0; i < k && i < max_records; ++i) {
    if (steps) steps[i] = ctx->mon_steps[i];
    if (sums) sums[i] = ctx->mon_vals[i];
  }
  *count = k;
  return MM_OK;
}

}  // extern "C"
