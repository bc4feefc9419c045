/*
 * mumode.h -- C ABI of the MI355X (gfx950) mu-mode product library.
 *
 * The library applies small dense n_mu x n_mu (or m x n_mu) matrices along
 * the modes of a d-dimensional tensor (the mu-mode product of Definition 2.1
 * of Caliari, Cassini, Einkemmer, Ostermann, Zivcovich, "A mu-mode integrator
 * for solving evolution equations in Kronecker form"), and builds on it the
 * mu-mode integrator (Section 2, equation dd-tensor), tensor spectral
 * transforms (Section 3, equations real2spec / spec2real) and Strang
 * splitting steps whose linear part is the integrator (Sections 4.3-4.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Tensors are dense and column-major: entry (i_1, ..., i_d) sits at linear
 *    index i_1 + n_1 (i_2 + n_2 (i_3 + ...)) (0-based; Section 4.1 gives the
 *    1-based form).  Complex values are interleaved (re, im).  Tensor data
 *    pointers are DEVICE pointers, 16-byte aligned.
 *  - Matrices handed to mm_op_prepare are column-major FP64 masters
 *    (L[i + j*ld]), real (MM_R64) or complex interleaved (MM_C128), in host
 *    memory (on_device = 0) or device memory (on_device = 1).
 *  - dtype <-> precision: an FP64-prepared operator acts on MM_R64 / MM_C128
 *    tensors; every other precision acts on MM_R32 / MM_C64 tensors.  A real
 *    operator may act on a complex tensor (applied to re and im); a complex
 *    operator on a real tensor is MM_ERR_DTYPE.
 *  - Ownership: the caller owns tensors, matrices and streams.  The context
 *    owns operators (mm_op) and its device workspace; mm_destroy frees them.
 *  - All tensor work is enqueued asynchronously on `stream` (0 = the null
 *    stream); only the monitors (mm_norm2, mm_energy_gpe) synchronise.
 *  - Every argument is validated before anything is launched.  No exception
 *    crosses the ABI; failures return an mm_status, with detail text from
 *    mm_last_error(ctx).  One context per host thread.
 */
#ifndef MUMODE_H
#define MUMODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_ERR_ARG = 1,         /* null pointer, aliasing, bad enum, nsteps < 0     */
  MM_ERR_SHAPE = 2,       /* d out of [1, MM_MAXD], dim <= 0, mu out of range,
                             op cols != n_mu, non-square op where required,
                             size above the supported maximum                 */
  MM_ERR_DTYPE = 3,       /* tensor dtype does not match the op precision     */
  MM_ERR_ALIGN = 4,       /* tensor data not 16-byte aligned                  */
  MM_ERR_NOMEM = 5,       /* device allocation failed                         */
  MM_ERR_HIP = 6,         /* a HIP runtime call failed (text in last_error)   */
  MM_ERR_UNSUPPORTED = 7, /* valid request the library does not implement    */
  MM_ERR_NONFINITE = 8,   /* a monitor found NaN / Inf                        */
  MM_ERR_NODEVICE = 9     /* no usable gfx950 device                          */
} mm_status;

typedef enum { MM_R32 = 0, MM_R64 = 1, MM_C64 = 2, MM_C128 = 3 } mm_dtype;

/* Arithmetic of the contractions.
 *  MM_PREC_FP64         FP64 MFMA, FP64 state.
 *  MM_PREC_FP32         FP32 MFMA, FP32 state.
 *  MM_PREC_SPLIT_BF16X3 operator and state split into three RNE bfloat16
 *                       pieces each (x = x0 + x1 + x2); the six piece
 *                       products x_a y_b with a + b <= 2 run on BF16 MFMA with
 *                       FP32 accumulation.
 *  MM_PREC_SPLIT_FP16X2 operator and state split into two RNE half-precision
 *                       pieces each, the low piece scaled by 2^11
 *                       (x = h + 2^-11 l); the three products h_A h_B,
 *                       h_A l_B, l_A h_B run on FP16 MFMA with FP32
 *                       accumulation (half the MFMA work of BF16X3, about
 *                       two bits less accurate).  The state is scaled by a
 *                       power of two from a bound of its largest component
 *                       that the library keeps on the device along each
 *                       chain of products (one extra max-abs pass over the
 *                       input at the start of every call); the operator by
 *                       a power of two fixed at preparation.  Not available
 *                       in mumode_expstep_batched (MM_ERR_UNSUPPORTED).
 *  MM_PREC_BF16         one bfloat16 piece each (single BF16 MFMA product);
 *                       reported for comparison only.                        */
typedef enum {
  MM_PREC_FP64 = 0,
  MM_PREC_FP32 = 1,
  MM_PREC_SPLIT_BF16X3 = 2,
  MM_PREC_SPLIT_FP16X2 = 3,
  MM_PREC_BF16 = 4
} mm_prec;

#define MM_MAXD 6

typedef struct mm_ctx_s* mm_ctx;
typedef struct mm_op_s* mm_op;
typedef struct ihipStream_t* mm_stream; /* same object as hipStream_t */

typedef struct {
  int d;                   /* order of the tensor, 1..MM_MAXD                  */
  int64_t dims[MM_MAXD];   /* n_1..n_d (entries beyond d ignored)              */
  mm_dtype dtype;
  void* data;              /* device pointer, column-major, 16-byte aligned    */
} mm_tensor;

typedef struct {
  int64_t rows, cols, ld;  /* ld >= rows                                        */
  mm_dtype dtype;          /* MM_R64 or MM_C128                                 */
  const void* data;        /* column-major FP64 master                          */
  int on_device;           /* 0: host pointer, 1: device pointer                */
} mm_matrix;

/* ------------------------------------------------------------ context ---- */

/* Create a context on HIP device `device` (checks it is gfx950).
 * tune_cache_path (nullable): a tune file (mm_tune_save format) that the
 * context reads at creation when it exists, and to which mm_autotune writes
 * the context's entries after every tuning run, so tile choices persist
 * across processes; a missing file is not an error, a malformed one is
 * (MM_ERR_ARG, no context).  Returns MM_ERR_NODEVICE if there is no usable
 * device; *out is NULL on failure. */
mm_status mm_create(mm_ctx* out, int device, const char* tune_cache_path);
/* Free every operator and buffer the context owns.  NULL is accepted. */
mm_status mm_destroy(mm_ctx ctx);
/* Static description of a status code. */
const char* mm_status_string(mm_status s);
/* Detail text of the last failure on this context ("" if none); valid until
 * the next call on ctx.  With ctx == NULL: the last mm_create failure. */
const char* mm_last_error(mm_ctx ctx);
/* Library version string. */
const char* mm_version(void);

/* ---------------------------------------------------------- operators ---- */

/* Prepare a matrix L (rows m x cols n) for the given precision: copy the FP64
 * master to the device and convert / split it into the layout the kernels
 * read.  The context owns *out.  m, n in [1, 4096]. */
mm_status mm_op_prepare(mm_ctx ctx, const mm_matrix* master, mm_prec prec, mm_op* out);
/* mm_op_prepare with flags:
 *   MM_OP_IDENTITY_SPLIT  square L only: the prepared pieces hold L - I,
 *     formed from the FP64 master, and every product adds its input entry
 *     back in FP32 in the epilogue (after a fused prologue phase), so the
 *     result is still T x_mu L.  For the near-identity exponentials of small
 *     time steps the MFMA accumulation then carries only the small
 *     departure from identity: the operator's representation error and the
 *     rounding of the accumulation scale with |L - I| instead of |L|, which
 *     keeps the split schemes' drift over long runs below the FP32 path's
 *     (R15).  Costs one extra read of the input per product.  Not accepted
 *     as a Hermite transform of ho_strang_step.
 * MM_ERR_ARG for unknown flags, MM_ERR_SHAPE for a non-square L with
 * MM_OP_IDENTITY_SPLIT. */
enum { MM_OP_IDENTITY_SPLIT = 1 };
mm_status mm_op_prepare_ex(mm_ctx ctx, const mm_matrix* master, mm_prec prec, unsigned flags, mm_op* out);
mm_status mm_op_destroy(mm_ctx ctx, mm_op op);
/* Flags an operator was prepared with. */
mm_status mm_op_flags(mm_op op, unsigned* flags);
/* Shape / type query of a prepared operator (any out pointer may be NULL). */
mm_status mm_op_info(mm_op op, int64_t* rows, int64_t* cols, int* is_complex, mm_prec* prec);

/* ------------------------------------------------------ tensor products -- */

/* S = T x_mu L (Definition 2.1): S(.., i, ..) = sum_j L[i,j] T(.., j, ..).
 * mu is 1-based.  out->dims must equal T->dims with dims[mu-1] replaced by
 * L's rows; out must not overlap T (MM_ERR_ARG). */
mm_status mumode_apply(mm_ctx ctx, mm_tensor* out, const mm_tensor* T, mm_op L, int mu,
                       mm_stream stream);

/* mu-mode integrator (Section 2, equation dd-tensor), in place, nsteps times:
 * T <- T x_1 E[0] x_2 E[1] ... x_d E[d-1].  E[k] == NULL leaves mode k+1
 * unchanged.  Every non-NULL E[k] must be square n_{k+1} x n_{k+1}. */
mm_status mumode_expstep(mm_ctx ctx, mm_tensor* T, const mm_op* E, int nsteps, mm_stream stream);

/* Tucker operator with rectangular matrices (Section 3, equations
 * real2spec and spec2real): out = in x_1 Phi[0] ... x_d Phi[d-1], with
 * out->dims[k] = rows of Phi[k] (in->dims[k] if Phi[k] == NULL).  out must
 * not overlap in. */
mm_status mumode_transform(mm_ctx ctx, mm_tensor* out, const mm_tensor* in, const mm_op* Phi,
                           mm_stream stream);

/* Strang splitting for the cubic Gross-Pitaevskii equation
 * i psi_t = H psi + beta |psi|^2 psi with H in Kronecker form (Section 4.5:
 * linear part by the integrator, nonlinear part integrated exactly).  One step
 * is N(tau/2) L(tau) N(tau/2) with L(tau) = x_1 E[0] ... x_d E[d-1],
 * E[k] = exp(-i tau H_{k+1}), and N(s) psi = exp(-i s beta |psi|^2) psi.
 * Adjacent half steps of N are merged (exact, since N keeps |psi|), and each
 * N is fused into the neighbouring mode product.  psi is complex (MM_C64 or
 * MM_C128), updated in place. */
mm_status gpe_strang_step(mm_ctx ctx, mm_tensor* psi, const mm_op* E, double tau, double beta,
                          int nsteps, mm_stream stream);

/* gpe_strang_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and kernels, bit for bit, with no hipMalloc, hipFree
 * or other allocating call.  The device memory the split FP16X2 products need
 * besides psi (the running-bound slots and the max-abs partial maxima,
 * 4192 bytes) is a fixed array in the library that each GPU holds until the
 * process ends; every call on one GPU shares it (each call's first product
 * rewrites all of it), so calls that overlap on one GPU, from any context or
 * stream, race.  Limits: every n_mu <= 256 (each product runs in place, no
 * workspace; MM_ERR_SHAPE otherwise), complex operators only (a real
 * operator on a complex state needs a promoted copy: MM_ERR_UNSUPPORTED), no
 * in-call monitor (MM_OPT_MONITOR_EVERY is ignored) and no per-launch
 * profiling records.  Operators are prepared beforehand (mm_op_prepare
 * allocates). */
mm_status gpe_strang_step_noalloc(mm_ctx ctx, mm_tensor* psi, const mm_op* E, double tau, double beta,
                                  int nsteps, mm_stream stream);

/* Strang step for the harmonic oscillator with a time-dependent potential,
 * i psi_t = -1/2 Laplace psi + 1/2 |x|^2 (1 + eps sin t) psi, in nodal
 * Hermite space (Section 3, equations real2spec / spec2real; the Hermite
 * part is exact, Section 4.3).  One step from t: P(t+tau/2, t+tau) L(tau)
 * P(t, t+tau/2), where L(tau) = x_1 Lh[0] ... x_d Lh[d-1] with the collapsed
 * propagator Lh[k] = Psi_bwd[k] diag(exp(-i tau (j + 1/2))) Phi_fwd[k]
 * (phi_j has oscillator energy j + 1/2), and P(a,b) is the exact flow of the
 * remainder, exp(-i (eps/2) |x|^2 (cos a - cos b)).
 *   Phi_fwd[k] : forward transform of mode k+1, K x n_{k+1} (K <= n_{k+1}
 *                Hermite functions), Phi[j, l] = phi_j(X_l) w_l, prepared
 *                from a real FP64 master (mm_hermite_matrices).
 *   Psi_bwd[k] : backward transform, n_{k+1} x K, Psi[l, j] = phi_j(X_l),
 *                same precision as Phi_fwd[k].
 *   nodes[k]   : host array of the n_{k+1} quadrature nodes X_l of mode k+1.
 * Lh[k] is formed on the device in FP64 from the operators' masters when the
 * operators, tau or the precision differ from the previous call on this
 * context (for MM_PREC_SPLIT_FP16X2 that formation reads the largest entry
 * back and synchronises `stream` once); later calls with the same ones reuse
 * it.  The node squares are uploaded only when the nodes change.  P is
 * separable over the modes, so each step folds it into the operators as
 * diagonal factors (re-prepared on the device every step when eps != 0) and
 * needs no pointwise pass.  psi is complex, updated in place; the caller
 * advances t0 by nsteps*tau.  Otherwise nothing synchronises. */
mm_status ho_strang_step(mm_ctx ctx, mm_tensor* psi, const mm_op* Phi_fwd, const mm_op* Psi_bwd,
                         const double* const* nodes, double t0, double tau, double eps, int nsteps,
                         mm_stream stream);

/* Strang splitting for the vortex-reconnection problem of Section 4.5 in
 * its symmetrised form, v_t = (i/2) M_W v + (i/2)(1 - W^-1 |v|^2) v, where
 * v = W^(1/2) u, M_W is the Kronecker sum of the modes' symmetrised
 * non-uniform Neumann operators (mm_nonuniform_neumann_d2) and W the
 * Kronecker product of their dual-cell widths.  One step is N(tau/2) L(tau)
 * N(tau/2) with L(tau) = x_1 E[0] ... x_d E[d-1], E[k] = exp(i tau/2 M_k),
 * and N(s) v = exp((i s/2)(1 - W^-1 |v|^2)) v, the exact nonlinear flow
 * (|v| is constant along it).  Adjacent half steps of N are merged; each N
 * is one pass over the state (its coefficient varies with the position).
 *   w[k]: host array of the n_{k+1} dual-cell widths of mode k+1 (the w of
 *         mm_nonuniform_neumann_d2), uploaded when they change.
 * v is complex, updated in place. */
mm_status vortex_strang_step(mm_ctx ctx, mm_tensor* v, const mm_op* E, const double* const* w, double tau,
                             int nsteps, mm_stream stream);

/* Batched integrator: count independent instances, each
 * T[i] <- T[i] x_1 E[i][0] ... x_{d_i} E[i][d_i - 1], nsteps times, in place.
 * Instances may differ in d, dims, dtype (real / complex) and precision.  One
 * step of the whole batch is a single HIP graph (captured on the first call
 * with a given set of tensors and operators, replayed afterwards): for each
 * mode, one launch per precision covers every instance's fibre tiles (each
 * work item selects its tile code: real / complex, fibre load path, tile
 * shape).  Requires every n_mu <= 256 (complex) / 512 (real) and P % 4 == 0
 * for the strided modes (MM_ERR_UNSUPPORTED otherwise).  E[i] is an array of
 * d_i operators (NULL entries leave the mode unchanged). */
mm_status mumode_expstep_batched(mm_ctx ctx, int count, mm_tensor* const* T, const mm_op* const* E, int nsteps,
                                 mm_stream stream);

/* Exponential midpoint rule (the second-order Magnus integrator of Section
 * 4.4, equation mag2) for u' = A(t) u with A(t) in Kronecker-sum form whose
 * mode parts depend on time as A_mu(t) = B_mu + g_mu(t) diag(d_mu):
 * each step u <- exp(tau A(t_n + tau/2)) u is the mu-mode integrator with
 * E_mu = exp(tau A_mu(t_n + tau/2)) (the exponential of a Kronecker sum is
 * the Kronecker product of the mode exponentials, Section 2).  The
 * exponentials of the time-dependent modes are formed on the device every
 * step in FP64 (scaling and squaring of the Taylor polynomial, products on
 * FP64 MFMA, as mm_expm_device), prepared in `prec` and applied; modes
 * without a time-dependent part are exponentiated once per call.
 *   B[k]   : n_k x n_k FP64 master (MM_C128 or MM_R64, host or device);
 *            B[k].data == NULL leaves mode k+1 unchanged.
 *   d      : NULL, or d[k] a host array of n_k reals (NULL: no
 *            time-dependent part on mode k+1).
 *   g      : host array of nsteps * T->d complex coefficients (re, im),
 *            g[2*(n*d + k)] = Re g_{k+1}(t_n + tau/2); may be NULL when no
 *            mode has a time-dependent part.  The caller evaluates them.
 * T is complex (MM_C128 with MM_PREC_FP64, MM_C64 otherwise), in place.
 * Allocates per-call device buffers (freed before returning, which
 * synchronises the device). */
mm_status mumode_magnus_step(mm_ctx ctx, mm_tensor* T, const mm_matrix* B, const double* const* d, const double* g,
                             double tau, int nsteps, mm_prec prec, mm_stream stream);

/* exp(c A) of a complex n x n FP64 matrix on the device (A, out: device
 * pointers, column-major interleaved, leading dimension n, not
 * overlapping): scaling to ||c A / 2^q||_1 <= 1, the degree-18 Taylor
 * polynomial (truncation below 2.2e-17) by the Paterson-Stockmeyer scheme
 * (7 matrix products), q squarings; each
 * matrix product runs on the FP64 MFMA mode-product kernel (the Taylor
 * approach Section 5.3 uses on the GPU).  Computes ||A||_1 on the device and
 * synchronises `stream`. */
mm_status mm_expm_device(mm_ctx ctx, int n, const double* A, double c_re, double c_im, double* out,
                         mm_stream stream);

/* Discrete GPE energy cell * [Re sum conj(psi) (sum_mu psi x_mu H[mu-1])
 * + (beta/2) sum |psi|^4], FP64 accumulation on the device; H[k] are the 1-D
 * Hamiltonians prepared in psi's precision.  The Hamiltonian of the
 * Gross-Pitaevskii problem of Section 4.5 is the Kronecker sum of the H[k]
 * (Section 2), so its quadratic form is the sum over the modes of
 * <psi, psi x_mu H[mu-1]>; the quartic term is the nonlinearity's energy.
 * The Strang step of gpe_strang_step conserves this energy up to O(tau^2).
 * Synchronises `stream`. */
mm_status mm_energy_gpe(mm_ctx ctx, const mm_tensor* psi, const mm_op* H, double beta, double cell,
                        double* host_out, mm_stream stream);

/* Discrete mass cell * sum |T|^2, accumulated in FP64 on the device: the
 * squared L2 norm that the unitary Schroedinger and Gross-Pitaevskii flows
 * conserve (Section 2 names the conserved mass among the invariants an
 * integrator should keep; every mode exponential of a Hermitian generator is
 * unitary, so each mu-mode step keeps it up to rounding).  Synchronises
 * `stream`.  Returns MM_ERR_NONFINITE if T holds NaN / Inf. */
mm_status mm_norm2(mm_ctx ctx, const mm_tensor* T, double cell, double* host_out, mm_stream stream);

/* ---------------------------------------------------- tuning, memory ---- */

/* Autotuner for the mode-product kernels.  For every mode k with E[k] !=
 * NULL, times each tile shape (workgroup layout, fibres per workgroup, K
 * depth of the LDS chunk, one or two workgroups per CU) that has a kernel
 * for the product T x_{k+1} E[k], out of place into the context workspace
 * (T is read, not modified), and records the fastest for that problem shape
 * (precision, real / complex, fibre load path, rows, columns, number of
 * fibres).  A complex product with a complex operator is timed a second
 * time with the fused prologue phase (the first product of a
 * Gross-Pitaevskii step), whose staging work can change the fastest shape,
 * and that choice is recorded under its own key (load path + 8).  Later
 * launches of the same shape on this context use the recorded shape (a
 * product with the prologue phase its own entry if there is one, else the
 * plain one); shapes never tuned use the built-in choice.  budget_ms bounds the timing loop (at least two
 * timed repetitions per candidate).  Synchronises `stream`.  The products
 * along the modes of an expstep, a Strang step or a batch all have the shape
 * tuned here when called with the same T and E. */
mm_status mm_autotune(mm_ctx ctx, const mm_tensor* T, const mm_op* E, int budget_ms, mm_stream stream);
/* Autotuner of the batched step (mumode_expstep_batched with the same
 * count, T and E): for each mode and each of real / complex instances, the
 * tile class of that group's products in the merged launches (0..2, or the
 * planner's own choice) is chosen by timing whole batched steps, one group
 * at a time with the others held (coordinate descent).  Tiles that are
 * fastest for an instance alone need not be fastest inside the merged
 * launch, where every instance's tiles share the GPU, so the choice is made
 * on the batch itself.  Runs the step in place on T several times (the
 * tensors' contents afterwards are those of an unspecified number of
 * steps).  The choice is kept by the context for later batched steps and
 * cleared by mm_tune_clear.  budget_ms bounds the timed replays per
 * candidate (at least two).  Synchronises `stream`. */
mm_status mm_autotune_batched(mm_ctx ctx, int count, mm_tensor* const* T, const mm_op* const* E, int budget_ms,
                              mm_stream stream);
/* The class chosen for mode `mode` (1-based) of real (is_complex = 0) or
 * complex instances; -1 when the planner's choice is kept. */
mm_status mm_autotune_batched_get(mm_ctx ctx, int mode, int is_complex, int* cls);
/* Number of recorded tune entries, and entry `index` (0-based):
 * key6 = {precision, complex, load path (0 contiguous fibres, 1 strided,
 * 2 gather, 3 paired real fibres; + 8 for a product with the fused prologue
 * phase), real rows, real columns, fibres}, the tile class and its time in
 * microseconds (any out pointer may be NULL). */
mm_status mm_tune_count(mm_ctx ctx, int* count);
mm_status mm_tune_get(mm_ctx ctx, int index, int64_t* key6, int* cls, double* us);
/* Forget every recorded entry. */
mm_status mm_tune_clear(mm_ctx ctx);
/* Write the entries to a text file / add the entries of such a file (an
 * entry already present is replaced).  MM_ERR_ARG if the file cannot be
 * opened or is malformed (nothing is added then). */
mm_status mm_tune_save(mm_ctx ctx, const char* path);
mm_status mm_tune_load(mm_ctx ctx, const char* path);

/* Context options.
 *   MM_OPT_SMALL_RUN (default 1): mumode_expstep with nsteps >= 2, plain
 *     FP64 or FP32 operators, a state of at most 2 MiB and modes of at most
 *     128 real rows runs all steps in one single-workgroup launch (the
 *     launch latency otherwise dominates such problems); 0 uses one launch
 *     per product.
 *   MM_OPT_MONITOR_EVERY (default 0 = off): mumode_expstep and
 *     gpe_strang_step record the FP64 sum |T|^2 (the discrete mass without the
 *     cell volume, §2) after every `value` steps and after the last one, on
 *     the device, and read the log back once when the call ends (one
 *     synchronisation per call); a non-finite entry makes the call return
 *     MM_ERR_NONFINITE.  The Strang phase flows keep |psi|, so the merged
 *     steps give the mass at the step times.  Disables MM_OPT_SMALL_RUN.
 *   MM_OPT_FP16X2_CHAIN (default 0): with 1, a mumode_expstep or
 *     gpe_strang_step call whose tensor is the one the previous such call on
 *     this context ended with (same data pointer, no other library call in
 *     between) continues that call's running bound of the state instead of
 *     starting with a max-abs pass over it (one read of the state saved per
 *     call, ~15 % of an nsteps = 1 FP16X2 call at n = 256).  The caller
 *     guarantees that nothing wrote the tensor in between and that the two
 *     calls are ordered on the device (same stream, or the earlier one
 *     complete); a call on another tensor, any other entry point or setting
 *     the option again starts a new chain.
 * MM_ERR_ARG for an unknown option or value. */
enum { MM_OPT_SMALL_RUN = 1, MM_OPT_MONITOR_EVERY = 2, MM_OPT_FP16X2_CHAIN = 3 };
mm_status mm_set_option(mm_ctx ctx, int option, int64_t value);

/* Monitor log of the last mumode_expstep / gpe_strang_step call on this
 * context: *count entries (step count after which it was taken, sum |T|^2);
 * at most max_records are written to steps / sums (either may be NULL). */
mm_status mm_monitor_log(mm_ctx ctx, int max_records, int* count, int* steps, double* sums);

/* Hand the context a caller-owned device workspace (256-byte aligned) for
 * products that cannot run in place and for the transform chain; the
 * context then never allocates one and returns MM_ERR_NOMEM when a call
 * needs more than `bytes`.  dev_ptr == NULL returns to a library-owned
 * workspace.  The caller keeps the memory alive while the context may use
 * it.  Synchronises the device (any earlier library workspace is freed). */
mm_status mm_set_workspace(mm_ctx ctx, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------ timing ---- */

/* Start recording a pair of HIP events for every mode-product kernel launch
 * of this context (on the launch stream), stamped by the launch itself
 * (hipExtLaunchKernelGGL start / stop events: the kernel's execution time,
 * no marker packets between launches).  Clears earlier records. */
mm_status mm_profile_begin(mm_ctx ctx);
/* Stop recording, wait for the recorded events and return, per launch in
 * issue order, a kernel kind code (prec*1000 + complex*100 + load*10 +
 * prologue*2 + epilogue; load 0 = contiguous fibres, 1 = strided fibres,
 * 2 = generic gather) and its duration in ms.  At most max_records entries
 * are written to kinds / ms (either may be NULL); *count receives the total
 * number of launches recorded. */
mm_status mm_profile_end(mm_ctx ctx, int max_records, int* count, int* kinds, double* ms);

/* ------------------------------------------ FP64 operator formation (host) */

/* Second-order centred second difference h^-2 (1, -2, 1) on n nodes of
 * [a, b] (Section 4.1): bc = 0 Dirichlet (n interior nodes,
 * h = (b-a)/(n+1)), bc = 1 periodic (h = (b-a)/n).  out: n*n doubles,
 * column-major, caller-owned. */
mm_status mm_fd2_matrix(int n, double a, double b, int bc, double* out);

/* exp(c A) for a complex n x n matrix A (column-major interleaved, n*n*2
 * doubles) and complex scalar c = c_re + i c_im, by scaling and squaring of a
 * truncated Taylor series in FP64 (host).  out: n*n*2 doubles. */
mm_status mm_expm(int n, const double* A, double c_re, double c_im, double* out);

/* Gauss-Hermite nodes X (m doubles, ascending) and Hermite-function weights
 * w_l = 1/(m phi_{m-1}(X_l)^2) (Section 3). */
mm_status mm_hermite_nodes(int m, double* X, double* w);

/* Hermite transform matrices at the m Gauss-Hermite nodes (Section 3):
 * forward Phi[k,l] = phi_k(X_l) w_l and backward Psi[l,k] = phi_k(X_l), both
 * m x m column-major real (either pointer may be NULL). */
mm_status mm_hermite_matrices(int m, double* Phi, double* Psi);

/* Collapsed exact harmonic-oscillator propagator in nodal Hermite space:
 * out = Psi diag(exp(-i tau (k + 1/2))) Phi (m x m complex, column-major
 * interleaved), Phi / Psi as in mm_hermite_matrices. */
mm_status mm_hermite_ho_exponential(int m, double tau, double* out);

/* 1-D Schroedinger Hamiltonian H = -1/2 D2 + (omega2 / 2) diag(x^2), D2 the
 * Dirichlet second difference of mm_fd2_matrix on the n interior nodes
 * x_j = a + j h of [a, b] (h = (b-a)/(n+1)): omega2 = 1 is the harmonic trap
 * of the Gross-Pitaevskii set-up (Section 4.5, with the trap of the
 * Section 4.3 oscillator), omega2 = 0 the free particle.  out: n*n doubles,
 * column-major.  MM_ERR_SHAPE for n < 1 or b <= a. */
mm_status mm_schrodinger_fd_hamiltonian(int n, double a, double b, double omega2, double* out);

/* E = exp(-i tau H), H as in mm_schrodinger_fd_hamiltonian: the exact flow
 * over tau of i psi_t = H psi, the mode exponential of the mu-mode integrator
 * (Section 2) for the Schroedinger and Gross-Pitaevskii set-ups (Taylor
 * scaling and squaring of mm_expm).  out: n*n complex (interleaved),
 * column-major.  n <= 4096. */
mm_status mm_schrodinger_fd_exponential(int n, double a, double b, double omega2, double tau, double* out);

/* Generator (i/2)(d^2/dx^2 - x^2) of one mode of the Section 4.4 Hamiltonian in
 * nodal Hermite space: Psi diag(-i (k + 1/2)) Phi (m x m complex, purely
 * imaginary, column-major interleaved; Phi / Psi as in mm_hermite_matrices). */
mm_status mm_hermite_ho_generator(int m, double* out);

/* Centred second difference of even order `order` (2..16) on n periodic
 * nodes of [a, b) (h = (b-a)/n), the symmetric circulant of the classical
 * central weights (Section 4.1, Test 2 varies the order).  out: n*n doubles,
 * column-major.  n >= order + 1. */
mm_status mm_fd2_periodic_order(int n, double a, double b, int order, double* out);

/* Fourier spectral second derivative on n periodic nodes of [a, b) (the
 * full matrix that Section 4.1 contrasts with sparse stencils), from its
 * closed form; for even n the Nyquist mode gets -(pi n / (b-a))^2.  out: n*n
 * doubles, column-major. */
mm_status mm_fourier_d2(int n, double a, double b, double* out);

/* 1-D operators of the pipe-flow problem of Section 4.2,
 * c_t = alpha (c_rr + c_r / r + c_zz) - s(z) c_z with
 * s(z) = 2 + tanh(4(z - 5/2)) - tanh(4(z - 5)), second-order centred
 * differences: A_r (n_r x n_r) on r_i = r_min + i h, h = (r_max - r_min)/
 * (n_r - 1), homogeneous Neumann at both ends (mirrored ghost values); A_z
 * (n_z x n_z) on z_j = j h, j = 1..n_z, h = z_max / n_z, c = 0 at z = 0 and
 * homogeneous Neumann at z_max.  The generator of the 2-D problem is the
 * Kronecker sum of the two (mode 1 = r, mode 2 = z).  Column-major. */
mm_status mm_pipe_flow_operators(int n_r, int n_z, double r_min, double r_max, double z_max, double alpha,
                                 double* A_r, double* A_z);

/* Second derivative on the non-uniform nodes x[0] < ... < x[n-1] (both
 * ends are boundary nodes) with homogeneous Neumann conditions, in the
 * symmetrised form of Section 4.5: the conservative three-point scheme
 * (D u)_j = (1/w_j) [(u_{j+1} - u_j)/h_j - (u_j - u_{j-1})/h_{j-1}],
 * h_j = x[j+1] - x[j], dual cells w_j = (h_{j-1} + h_j)/2 (w_0 = h_0/2,
 * w_{n-1} = h_{n-2}/2), no flux through the ends, is D = W^-1 S with S
 * symmetric; the variable v = W^(1/2) u makes it M = W^(-1/2) S W^(-1/2),
 * symmetric, and sum_j w_j |u_j|^2 = |v|^2.  In d dimensions the generator
 * of the transformed problem is the Kronecker sum of the modes' M and the
 * weight the Kronecker product of their W.  M: n*n doubles, column-major;
 * w: n doubles (nullable).  MM_ERR_ARG for n outside [2, 4096] or NULL x /
 * M, MM_ERR_SHAPE for nodes not strictly increasing. */
mm_status mm_nonuniform_neumann_d2(int n, const double* x, double* M, double* w);

#ifdef __cplusplus
}
#endif

#endif /* MUMODE_H */
