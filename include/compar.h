/*
 * compar.h -- C ABI of libcompar, a runtime that exposes several implementation
 * variants of a component interface and picks one per call from the runtime
 * context, after COMPAR (Memeti, "Enabling Dynamic Selection of Implementation
 * Variants in Component-Based Parallel Programming for Heterogeneous Systems").
 *
 * The paper's directives become calls:
 *   - method_declare(interface, name, target)   -> cmp_variant_register   (Sec. 2.1)
 *   - parameter(name, type, size, access_mode)  -> cmp_param_desc lists    (Sec. 2.1)
 *   - compar initialize / terminate             -> cmp_init / cmp_terminate (Sec. 2.1)
 *   - generated task creation and submission    -> cmp_gemm / cmp_call_host (Sec. 2.2.2)
 *   - the runtime's choice of codelet per task  -> cmp_select              (Sec. 2.2.2)
 *   - resource restriction by environment       -> cmp_set_variant_mask    (Sec. 3.2)
 *
 * The built-in interface is "gemm": C = alpha * A * B + beta * C over float
 * matrices (the paper's matrix-multiplication interface of Sec. 2.1, in BLAS
 * form), with four hand-written HIP variants for gfx950 registered by cmp_init:
 *
 *   id 0 "f32_simt"  FP32 FMA on the vector ALUs            stated bound 1e-5
 *   id 1 "bf16x3"    bf16 hi/lo split, three MFMA products  stated bound 1e-5
 *   id 2 "fp8r"      E4M3 + one residual pass, four MFMA
 *                    products with per-128x128-tile scales  stated bound 1e-3
 *   id 3 "bf16"      bf16 operands, one MFMA product        stated bound 1e-2
 *
 * and two optional built-ins that cmp_register_builtin adds on request:
 *
 *   "fp6x3"          OCP MX FP6 (E2M3) with one E8M0 scale
 *                    per 32 K values and one residual level,
 *                    three products hi.hi + hi.lo + lo.hi on
 *                    the scaled MFMA at the FP6 rate        stated bound 1e-2
 *   "host_f32"       FP32 GEMM on the host CPU (the paper's
 *                    CPU codelet beside the GPU ones)      stated bound 1e-5
 *
 * "Stated bound" is the relative Frobenius error ||C - C_exact||_F/||C_exact||_F
 * the variant is registered with; a call with tolerance tol may only run
 * variants whose bound is <= tol (the "context match" step of OpenMP's
 * declare variant, which COMPAR extends, Sec. 2.1), and among those the
 * selector picks the one with the lowest measured or predicted time.
 * The built-in bounds are the errors the variants meet on operands with
 * independent entries (normal, uniform, and normal(0,1) * 2^u with u drawn per
 * entry in [-20, 20]) up to K = 8192, NOT worst-case bounds: correlated
 * operands keep the rounding errors from averaging out.  Constant operands
 * A = B = c give fp8r 3.78e-3 (c = 1.033203125), bf16x3 2.94e-5
 * (c = 1.0039134), and K = 8192 equal products summed in one FP32 accumulator
 * drift by up to ~1e-4 (every variant accumulates in FP32).  A caller that
 * needs the tolerance guaranteed sets CMP_FLAG_VERIFY: the FP64 probe then
 * checks every result against tol and falls back to a tighter variant.
 *
 * Conventions for every function:
 *   - Returns a cmp_status; CMP_OK is 0 and every error is negative.  No C++
 *     exception crosses this boundary.  cmp_last_error(ctx) returns a message
 *     for the last failing call on that context.
 *   - Matrices are row-major with leading dimensions in elements.  A, B, C in
 *     cmp_gemm_args are DEVICE pointers owned by the caller; they must stay
 *     valid until the work queued on `stream` has finished.  The library never
 *     frees caller memory.  Host arrays (history rows, network parameters,
 *     features) are read or written during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     GEMM calls are asynchronous on that stream unless stated otherwise.
 *     After one call of a shape on a context (which sizes the workspace and
 *     records the selection), further calls of that shape with the built-in
 *     GPU variants only enqueue kernels and stream/event waits, so they can be
 *     captured into a graph (stream capture) and replayed; verify mode and the
 *     host variant synchronise and cannot.
 *   - A cmp_ctx is not thread-safe: use one context per host thread.  It also
 *     serves one stream at a time: all image variants of a context share one
 *     device workspace (their pre-pass images), so calls on two streams of
 *     one context must be ordered by the caller (e.g. an event wait).
 *   - The workspace grows on demand: a call that needs more than the current
 *     size synchronises the device, frees the old buffer and allocates a
 *     larger one.  A graph captured earlier still refers to the old buffer,
 *     so growth invalidates captured graphs: call cmp_reserve for the largest
 *     shape before capturing; a reservation pins the workspace, and a later
 *     variant that would need more fails with CMP_ENOMEM instead of moving it
 *     (cmp_gemm then falls back to another admissible variant, see
 *     cmp_reserve).
 *   - Name strings are copied on registration.
 */
#ifndef COMPAR_H
#define COMPAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cmp_status {
    CMP_OK = 0,
    CMP_EINVAL = -1,        /* null pointer, negative size, ld < columns, tol <= 0, bad id */
    CMP_EDUP = -2,          /* duplicate interface, parameter or variant name (Sec. 2.2.1) */
    CMP_ESIG = -3,          /* variant signature differs from the interface's (Sec. 2.1) */
    CMP_ENOTFOUND = -4,     /* unknown interface or variant name */
    CMP_ENOVARIANT = -5,    /* no enabled variant's stated bound is within tol */
    CMP_EUNSUPPORTED = -6,  /* operation needs a GPU context, or an unsupported dtype */
    CMP_EHIP = -7,          /* a HIP runtime call failed (message has hipGetErrorString) */
    CMP_ENOMEM = -8,        /* workspace allocation failed */
    CMP_ECHECK = -9,        /* verify mode: residual check failed after the fallback */
    CMP_ENODATA = -10       /* selector has no history / network to use */
} cmp_status;

typedef enum cmp_target {           /* target clause of method_declare (Sec. 2.1) */
    CMP_TARGET_HIP = 1,             /* variant enqueues HIP work on the given stream */
    CMP_TARGET_HOST = 2             /* variant runs synchronously on the calling host thread */
} cmp_target;

typedef enum cmp_dtype {            /* type clause of parameter (Sec. 2.1) */
    CMP_F32 = 0, CMP_BF16 = 1, CMP_F8E4M3 = 2, CMP_F64 = 3, CMP_I32 = 4, CMP_I64 = 5
} cmp_dtype;

typedef enum cmp_access {           /* access_mode clause of parameter (Sec. 2.1) */
    CMP_READ = 1, CMP_WRITE = 2, CMP_READWRITE = 3
} cmp_access;

typedef enum cmp_selector_kind {
    CMP_SEL_STATIC = 0,     /* fixed choice per tolerance: lowest total recorded time */
    CMP_SEL_NN = 1,         /* history nearest neighbour in (log2 M, log2 N, log2 K) */
    CMP_SEL_MLP = 2         /* learned network predicting ln(time) per variant */
} cmp_selector_kind;

enum {
    CMP_FLAG_VERIFY = 1u,   /* after each cmp_gemm, run the FP64 Freivalds probe and fall
                               back to the next tighter variant if it exceeds tol */
    CMP_FLAG_LOG = 2u       /* append one JSON line per cmp_gemm call to the log sink
                               (cmp_set_log_file; stderr by default), see below */
};

/* One parameter of an interface (the parameter directive, Sec. 2.1).  `extent`
 * lists 0..4 sizes (0 = scalar, 1 = vector, 2 = matrix, ...); each is the name
 * of another parameter of the interface or a decimal literal. */
typedef struct cmp_param_desc {
    const char *name;
    int32_t type;           /* cmp_dtype */
    int32_t ndim;           /* 0..4 */
    const char *extent[4];
    int32_t mode;           /* cmp_access */
} cmp_param_desc;

/* Arguments of the built-in "gemm" interface: C = alpha * A * B + beta * C.
 * A is M x K (lda >= K), B is K x N (ldb >= N), C is M x N (ldc >= N), all
 * float32 row-major device pointers.  BLAS semantics: beta == 0 never reads C;
 * alpha == 0 or K == 0 never reads A or B; M == 0 or N == 0 is a no-op. */
typedef struct cmp_gemm_args {
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    float alpha, beta;
    const float *A;
    const float *B;
    float *C;
} cmp_gemm_args;

/* The runtime context a selection is made for (Sec. 1: input size and
 * system configuration; here also the caller's error tolerance). */
typedef struct cmp_context {
    int64_t M, N, K;
    int32_t dtype;          /* cmp_dtype of the operands; only CMP_F32 is supported */
    double tol;             /* relative Frobenius tolerance, > 0 */
} cmp_context;

/* A variant of an interface.  `args` points to the interface's argument
 * struct (cmp_gemm_args for "gemm"); `workspace` is library-owned device
 * memory of at least the size the variant's cmp_ws_fn asked for (NULL if it
 * asked for 0); `user` is the pointer given at registration. */
typedef int (*cmp_variant_fn)(const void *args, void *workspace, size_t ws_bytes,
                              void *stream, void *user);
/* Workspace bytes a variant needs for `args` (may be NULL: none). */
typedef size_t (*cmp_ws_fn)(const void *args, void *user);

typedef struct cmp_ctx cmp_ctx;

/* ---- lifetime (compar initialize / terminate, Sec. 2.1) ---------------- */

/* Create a context on HIP device `device` and register the "gemm" interface
 * with its four built-in variants.  device < 0 creates a host-only context
 * (no GPU touched, no built-in variants): host variants, registry, history
 * and selection logic work; GPU entry points return CMP_EUNSUPPORTED.
 * Environment: COMPAR_VARIANTS=<name,name,...> restricts the enabled gemm
 * variants, COMPAR_SELECTOR=static|nn|mlp picks the selector,
 * COMPAR_FORCE=<name> forces one variant, COMPAR_FAULT=<name>:<n> makes every
 * n-th call of that variant fail with CMP_EHIP (for testing the fallback). */
int cmp_init(int device, cmp_ctx **out);
/* Release the workspace, history and network; `ctx` is invalid afterwards.
 * Waits for the library's own streams, not for the caller's. NULL is a no-op. */
int cmp_terminate(cmp_ctx *ctx);
const char *cmp_last_error(const cmp_ctx *ctx);
const char *cmp_status_string(int status);
/* Library version string, and the device this context runs on (-1 = host). */
const char *cmp_version(void);
int cmp_device(const cmp_ctx *ctx, int *device, char *arch, size_t arch_len,
               int *cu_count, int *clock_khz);

/* ---- registry (method_declare and parameter, Sec. 2.1; semantic checks, Sec. 2.2.1) */

/* Declare an interface with its parameter list.  CMP_EDUP if the interface
 * exists or two parameters share a name; CMP_EINVAL on a bad descriptor or an
 * extent naming no parameter. */
int cmp_interface_declare(cmp_ctx *ctx, const char *iface, int nparams,
                          const cmp_param_desc *params);
/* Register a variant.  `params` may be NULL when the interface already exists
 * (later variants share the first one's signature, Sec. 2.1); if given, it must
 * equal the interface's list (CMP_ESIG otherwise), and if the interface does not
 * exist yet it is declared with it.  err_bound > 0 is the stated relative
 * Frobenius bound.  *id_out receives the variant's index in its interface. */
int cmp_variant_register(cmp_ctx *ctx, const char *iface, const char *name, int target,
                         int nparams, const cmp_param_desc *params,
                         cmp_variant_fn fn, cmp_ws_fn ws, double err_bound,
                         void *user, int *id_out);
int cmp_variant_count(cmp_ctx *ctx, const char *iface, int *n);
/* Name (pointer valid until cmp_terminate), target and stated bound of a variant. */
int cmp_variant_info(cmp_ctx *ctx, const char *iface, int id, const char **name,
                     int *target, double *err_bound);
int cmp_variant_find(cmp_ctx *ctx, const char *iface, const char *name, int *id);
/* Enable only the variants whose bit is set (bit i = id i); the analogue of the
 * paper's CPU-only / GPU-only runs (Sec. 3.2). */
int cmp_set_variant_mask(cmp_ctx *ctx, const char *iface, uint64_t mask);
/* Force one variant for every call of the interface (id < 0 clears it). */
int cmp_force_variant(cmp_ctx *ctx, const char *iface, int id);

/* ---- selection (the runtime's choice of codelet, Sec. 2.2.2) ------------ */

int cmp_selector_set(cmp_ctx *ctx, int kind);
/* Flags: a combination of CMP_FLAG_VERIFY and CMP_FLAG_LOG (CMP_EINVAL for
 * other bits). */
int cmp_set_flags(cmp_ctx *ctx, uint32_t flags);
/* Per-call log (the performance-history record of each task, Sec. 3.2).  With
 * CMP_FLAG_LOG set, every cmp_gemm call appends one JSON object per line:
 *   {"call": n, "M": .., "N": .., "K": .., "tol": .., "selector": s,
 *    "variant": name, "id": i, "predicted_us": p, "measured_us": t,
 *    "residual": r, "fallbacks": f}
 * s is "nn", "mlp" or "static" (the context's selector), "forced" (a forced
 * variant) or "only" (one admissible variant).  p is the time the selector
 * ranked the chosen variant by (the network's prediction, or the recorded
 * median at the history's nearest shape that timed it), null when none (the
 * static choice, a forced or only variant, or a fallback's variant).  t is the
 * duration of the run that produced C, from a HIP event pair on the stream
 * around all the work the variant queued (host variants: the host clock);
 * null when the call was made while the stream was being captured.  r is the
 * verify-mode probe estimate (null without CMP_FLAG_VERIFY).  f counts the
 * fallbacks this call took.  Records are written in call order once their
 * events have completed: at a later cmp_gemm call, cmp_log_flush, a change of
 * sink or cmp_terminate.  The environment variable COMPAR_LOG=<path> at
 * cmp_init opens that file and sets CMP_FLAG_LOG.
 * path NULL or "" selects stderr; otherwise the file is opened for appending
 * (CMP_EINVAL if it cannot be).  Records still pending go to the old sink
 * first. */
int cmp_set_log_file(cmp_ctx *ctx, const char *path);
/* Wait for the pending log records' events and write them. */
int cmp_log_flush(cmp_ctx *ctx);
/* Split-K of the built-in MFMA variants (bf16x3, fp8r, bf16).  With fewer
 * 256 x 256 output tiles than compute units, these variants can cut K into
 * slices run by separate workgroups, each writing an M x N float partial sum
 * to the variant's workspace, then add the partials in slice order (so the
 * result does not depend on scheduling).  splits = 0 (the default) lets a cost
 * model choose per call; splits >= 1 forces that many slices, at most 64 and
 * at most one per 64-byte K block, every slice non-empty (1 disables split-K).
 * This is a tuning and testing knob: the sum order, hence the rounding, of a
 * result depends on the slice count, and a forced count applies to every
 * shape, so the workspace grows by splits x M x N floats (CMP_ENOMEM if that
 * allocation fails). */
int cmp_set_split_k(cmp_ctx *ctx, int splits);
/* Size the shared device workspace for every enabled built-in GPU variant of
 * "gemm" on an M x N x K product (pre-pass images plus the split-K partial sums
 * of the current split setting) and pin it: later calls never reallocate it
 * (so graphs captured after the reservation stay valid).  A variant that would
 * need more fails with CMP_ENOMEM: cmp_gemm_variant returns that status, while
 * cmp_gemm treats it like any failing variant and falls back once to the best
 * other admissible variant (f32_simt needs no workspace), failing with
 * CMP_ENOMEM only if that one does not fit either.  M = N = K = 0 releases the
 * pin (the buffer is kept).  Synchronises the device when the buffer grows. */
int cmp_reserve(cmp_ctx *ctx, int64_t M, int64_t N, int64_t K);
/* Register an optional built-in variant of "gemm" by name: "fp6x3" (GPU
 * contexts only) or "host_f32" (CMP_TARGET_HOST).  It takes the next free id
 * (*id, may be NULL).  CMP_EDUP if already registered, CMP_ENOTFOUND for an
 * unknown name.  "host_f32" in a GPU context copies A, B (and C when
 * beta != 0) from the device after the work queued on `stream`, multiplies on
 * up to 16 host threads and copies C back before the call returns
 * (synchronous); in a host-only context the cmp_gemm_args pointers are host
 * memory and are used in place.  The learned selector's network predicts the
 * four default built-ins; for other variants it uses the history's nearest
 * timed shape. */
int cmp_register_builtin(cmp_ctx *ctx, const char *name, int *id);
/* Slice count a call of built-in variant `id` of "gemm" would use for an
 * M x N x K product under the current setting (1 for f32_simt and for
 * variants registered by the caller). */
int cmp_split_k(cmp_ctx *ctx, int id, int64_t M, int64_t N, int64_t K, int *splits);
/* Admissible variants for ctx->tol as a bit mask (bit i = id i). */
int cmp_admissible(cmp_ctx *ctx, const char *iface, const cmp_context *c, uint64_t *mask);
/* Choose a variant for one context: admissible set, then the selector's
 * argmin of time; ties go to the tighter stated bound, then the lower id.
 * Falls back STATIC <- NN <- MLP when a selector has no data. */
int cmp_select(cmp_ctx *ctx, const char *iface, const cmp_context *c, int *id_out);
/* Same for n contexts at once; with the MLP selector all cache misses are
 * predicted by one launch of the inference kernel. */
int cmp_select_batch(cmp_ctx *ctx, const char *iface, int n, const cmp_context *c, int *ids_out);

/* ---- execution (task creation and submission, Sec. 2.2.2) --------------- */

/* Run "gemm" with the variant selected for (M, N, K, F32, tol).  Asynchronous
 * on `stream` (except in verify mode, which synchronises the stream to read
 * the probe).  *chosen (may be NULL) receives the variant id that ran. */
int cmp_gemm(cmp_ctx *ctx, const cmp_gemm_args *args, double tol, void *stream, int *chosen);
/* Serve a stream of `n` "gemm" requests in order, each as one cmp_gemm: its
 * own context (shape, tols[i]) selects its variant (Sec. 2.2.2: one task per
 * request, the codelet chosen at run time).  flags[i] & CMP_FLAG_VERIFY
 * switches verify mode on for request i (flags may be NULL: the context's
 * flags apply to every request; the context's flags are the same afterwards).
 * sync != 0: each request is complete before the next is submitted, and
 * lat_us[i] receives its latency in microseconds, host submission to
 * completion on `stream`; sync == 0: the requests are only enqueued (lat_us
 * unused).  chosen[i] receives the variant id that ran.  chosen and lat_us
 * may be NULL.  Requests may share operands and C: they run in stream order.
 * Stops at the first request that fails and returns its status; *done (may
 * be NULL) receives the number of requests served before it. */
int cmp_gemm_stream(cmp_ctx *ctx, int n, const cmp_gemm_args *reqs, const double *tols,
                    const uint32_t *flags, int sync, void *stream, int *chosen, double *lat_us,
                    int *done);
/* Run one named variant of "gemm" by id, bypassing selection. */
int cmp_gemm_variant(cmp_ctx *ctx, int id, const cmp_gemm_args *args, void *stream);
/* Run a host-target variant of any interface (synchronous), bypassing selection. */
int cmp_call_host(cmp_ctx *ctx, const char *iface, int id, const void *args);

/* For callers that cannot allocate device memory (code under their own graph
 * capture, serving loops or harnesses that forbid hipMalloc): cmp_gemm_variant
 * with the variant's workspace (pre-pass images, split-K partial sums) taken
 * from a fixed array of CMP_STATIC_WS_BYTES in the library's device code
 * instead of the context's workspace.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine; per-kernel timing is
 * suspended for it, since that creates events) and only enqueues kernels and
 * event waits on `stream`.  The caller passes A, B, C as for cmp_gemm_variant.
 * Each GPU holds its own copy of the array, created with the library's code
 * on that device and kept until the process ends; every call on one GPU, from
 * any context, shares it and it keeps the last call's contents, so calls that
 * overlap in time on one GPU (two streams, two host threads) race: order them.
 * Errors: CMP_ENOMEM (message names the bytes) when the variant needs more
 * workspace for this shape than the array holds (e.g. bf16x3 and fp8r fit up
 * to 4096^3, bf16 beyond); CMP_EUNSUPPORTED for a host context or a
 * CMP_TARGET_HOST variant; CMP_EHIP if the array's device address could not be
 * obtained at cmp_init; otherwise as cmp_gemm_variant.  Results are
 * bit-identical to cmp_gemm_variant's (the same kernels). */
#define CMP_STATIC_WS_BYTES ((size_t)128 << 20)
int cmp_gemm_variant_static(cmp_ctx *ctx, int id, const cmp_gemm_args *args, void *stream);

/* ---- timing and history (performance history, Sec. 3.2) --------------- */

/* Time one variant: `warmup` untimed calls, then `reps` calls each bracketed
 * by HIP events on `stream` (host variants: steady clock).  Outputs in ms. */
int cmp_time_variant(cmp_ctx *ctx, int id, const cmp_gemm_args *args, int warmup, int reps,
                     void *stream, float *median_ms, float *min_ms, float *mean_ms);
/* Time every enabled gemm variant on each of `nshapes` (M, N, K) triples
 * (mnk[3*s + 0..2]) and append the results to the history.  A, B, C are device
 * buffers holding at least max(M*K), max(K*N), max(M*N) floats; each shape uses
 * them with tight leading dimensions, alpha = 1, beta = 0.  Shapes already in
 * the history for a variant are skipped, so an interrupted calibration resumes. */
int cmp_calibrate(cmp_ctx *ctx, int nshapes, const int64_t *mnk, const float *A,
                  const float *B, float *C, int warmup, int reps, void *stream);
int cmp_history_add(cmp_ctx *ctx, int64_t M, int64_t N, int64_t K, int id, int reps,
                    float median_ms, float min_ms, float mean_ms);
int cmp_history_count(cmp_ctx *ctx, int *n);
int cmp_history_get(cmp_ctx *ctx, int row, int64_t *mnk, int *id, int *reps,
                    float *median_ms, float *min_ms, float *mean_ms);
int cmp_history_clear(cmp_ctx *ctx);
/* Persist / reload the history as text with a header naming the device
 * (arch, CU count, clock) and library version; load rejects (CMP_EINVAL) a
 * file recorded on a different device signature unless `force` is non-zero. */
int cmp_history_save(cmp_ctx *ctx, const char *path);
int cmp_history_load(cmp_ctx *ctx, const char *path, int force);

/* ---- learned selector (performance models trained from history, Sec. 3.2, 5) */

/* The network is 4 -> 64 -> 64 -> 4 with ReLU, 4740 float parameters packed
 * layer by layer as [W (out x in, row-major), b (out)].  Inputs are
 * (log2 M, log2 N, log2 K, log10 tol) standardised by per-feature mean and
 * population deviation; outputs are ln(median microseconds) of variants 0..3,
 * standardised per output the same way. */
int cmp_mlp_param_count(void);
int cmp_mlp_set_params(cmp_ctx *ctx, const float *params, int n);
int cmp_mlp_get_params(cmp_ctx *ctx, float *params, int n);
/* Standardisation statistics (4 floats each); get works after training. */
int cmp_mlp_set_norm(cmp_ctx *ctx, const float *mu_x, const float *sd_x,
                     const float *mu_y, const float *sd_y);
int cmp_mlp_get_norm(cmp_ctx *ctx, float *mu_x, float *sd_x, float *mu_y, float *sd_y);
/* Train on the GPU from the current parameters: computes the standardisation
 * of raw features X (n x 4) and raw targets Y (n x 4, ln microseconds) on the
 * host, then runs `steps` full-batch Adam steps (beta1 0.9, beta2 0.999,
 * eps 1e-8, fresh moments) in one resident kernel.  loss_trace (may be NULL)
 * receives the loss before each step.  Synchronous.  n <= 8192. */
int cmp_mlp_train(cmp_ctx *ctx, int n, const float *X, const float *Y, int steps, float lr,
                  float *loss_trace);
/* One loss and gradient evaluation on the GPU for standardised X, Y (n x 4). */
int cmp_mlp_grad(cmp_ctx *ctx, int n, const float *Xs, const float *Ys, float *loss, float *grad);
/* Batched inference kernel: standardised network outputs for standardised X. */
int cmp_mlp_infer(cmp_ctx *ctx, int n, const float *Xs, float *Yout);
/* Build features and ln-time targets from the history (shapes with a
 * recorded time for all four built-in variants; tol feature drawn per row from
 * the three classes by splitmix64(seed)), initialise the parameters
 * Kaiming-uniform from splitmix64(seed), train, and enable the network for
 * CMP_SEL_MLP.  *final_loss (may be NULL) receives the last loss. */
int cmp_mlp_fit_history(cmp_ctx *ctx, int steps, float lr, uint64_t seed, float *final_loss);
/* Persist / reload the network (parameters and the four standardisation
 * vectors) as text, with the same header as the history (device signature,
 * library version; values printed with 9 significant digits, so a reload is
 * bit-exact).  Save: CMP_ENODATA when the network has no parameters.  Load:
 * CMP_EINVAL for a file that is not a network file, is malformed, has the
 * wrong parameter count or non-positive deviations, or was saved on a
 * different device signature (unless `force` is non-zero); on success the
 * network is enabled for CMP_SEL_MLP and the decision cache cleared. */
int cmp_mlp_save(cmp_ctx *ctx, const char *path);
int cmp_mlp_load(cmp_ctx *ctx, const char *path, int force);

/* ---- verification (FP64 residual probe) -------------------------------- */

/* Freivalds probe of a finished product: with x = probe (host array of N
 * doubles, copied to the device), returns ||C x - (alpha A (B x) + beta C0 x)||
 * / ||alpha A (B x) + beta C0 x|| computed in FP64 on the GPU.  c0 (device,
 * ld = args->ldc) is the C before the product; it is read only if beta != 0.
 * Synchronises `stream`. */
int cmp_freivalds(cmp_ctx *ctx, const cmp_gemm_args *args, const float *c0, const double *probe,
                  void *stream, double *estimate);
/* Probe estimate of the last cmp_gemm in verify mode, and the number of
 * fallbacks cmp_gemm has taken on this context (re-runs after a failing
 * variant and after a failed verify-mode probe). */
int cmp_last_verify(cmp_ctx *ctx, double *estimate, int *fallbacks);

/* ---- operand pre-pass (exposed for bit-exact checking) ------------------ */

/* bf16 split of a rows x cols float32 device matrix X (ld ldx) into hi and lo
 * (device, rows x cols uint16 bit patterns, row-major, tight): hi = RNE(x),
 * lo = RNE(x - hi).  lo may be NULL.  Asynchronous on stream. */
int cmp_split_bf16(cmp_ctx *ctx, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                   uint16_t *hi, uint16_t *lo, void *stream);
/* E4M3 tile quantisation with one residual pass (128 x 128 tiles, OCP E4M3,
 * power-of-two scales 2^e with amax * 2^e <= 448 < amax * 2^(e+1)): q and rq
 * are rows x cols bytes (device, tight), qscale and rscale the E8M0 bytes
 * (127 - e) per tile, tile-row-major ceil(rows/128) x ceil(cols/128). */
int cmp_quant_fp8(cmp_ctx *ctx, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                  uint8_t *q, uint8_t *qscale, uint8_t *rq, uint8_t *rscale, void *stream);
/* OCP MX FP6 (E2M3) quantisation with one residual level, blocks of 32
 * consecutive K values, each with an E8M0 scale byte 127 - e where e is the
 * largest integer with max|x| * 2^e <= 7.5; q = RNE_e2m3(x * 2^e), then the
 * FP32 residual quantised the same way with its own block scale (OCP MX
 * specification v1.0, E2M3 and E8M0 formats).  A block holding a NaN or an
 * infinity gets scale byte 0xff (E8M0 NaN) at both levels and zero codes.
 * transpose = 0: K runs along the rows of X (rows x cols); outputs q and rq
 * are rows x cols bytes and the scales rows x ceil(cols / 32).
 * transpose != 0: K runs down the columns of X (X is K x N = rows x cols);
 * outputs are cols x rows bytes (X transposed) and the scales
 * cols x ceil(rows / 32).  One code per byte (low 6 bits: sign bit 5,
 * exponent bits 4-3, fraction bits 2-0); device memory, tight, row-major. */
int cmp_quant_mx6(cmp_ctx *ctx, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                  int transpose, uint8_t *q, uint8_t *qscale, uint8_t *rq, uint8_t *rscale,
                  void *stream);

/* Operand images of a built-in pre-passed variant (bf16, bf16x3, fp8r,
 * fp6x3), exposed so that the pre-pass a variant runs on its hot path can be
 * checked bit for bit: cmp_prepass_images launches exactly the kernels, with
 * the same launch configuration, that the variant launches on A and B before
 * its GEMM kernel, but writes the images to `out` instead of the library's
 * workspace.  The images are the variant's panel images (bf16, E4M3, MX FP6
 * encodings as in cmp_split_bf16, cmp_quant_fp8, cmp_quant_mx6, of A and of
 * B transposed), zero-padded to Mp x Kp and Np x Kp:
 *   bf16 / FP8 codes: element (row, k) of an image with Kb bytes of K per row
 *     (Kb = 2 Kp or Kp) is at byte b(row, kbyte) with kbyte = 2 k or k, where
 *     b = ((row / 256) * (Kb / 64) + kbyte / 64) * 16384 + (row % 256) * 64
 *         + (((kbyte / 16) % 4) ^ ((row % 256) / 4 % 4)) * 16 + kbyte % 16;
 *   FP8 tile scales: one E8M0 byte per 128 x 128 tile, tile-row-major
 *     (Mp / 128) x (Kp / 128) (A) or (Np / 128) x (Kp / 128) (B^T);
 *   MX FP6: per 256-row by 64-value K block, a 12 KiB code block (48 bytes
 *     per row: [half 0 bytes 0-15 | half 1 bytes 0-15 | half 0 bytes 16-23 |
 *     half 1 bytes 16-23], the 32 codes of a half packed 6 bits each, code j
 *     at bit 6 j) and a 1 KiB scale block (4 bytes per row: half 0 hi,
 *     half 0 lo, half 1 hi, half 1 lo); block (rb, kb) is block rb * (Kp / 64)
 *     + kb of its array.
 * Image order (offset[i]): bf16: A hi, B^T hi; bf16x3: A hi, B^T hi, A lo,
 * B^T lo; fp8r: A q, A r, B^T q, B^T r, then the tile scales of A q, A r,
 * B^T q, B^T r; fp6x3: A hi, A lo, B^T hi, B^T lo, A scales, B^T scales.
 * Unused entries have offset -1.  CMP_EUNSUPPORTED for a variant without a
 * pre-pass; CMP_EINVAL for M, N or K < 1, null pointers, or out_bytes < total.
 * alpha, beta and C of args are ignored.  Asynchronous on stream. */
typedef struct cmp_image_layout {
    int64_t Mp, Np, Kp;
    int32_t count;          /* number of images */
    int64_t offset[8];      /* byte offset of image i in `out` (-1: unused) */
    int64_t bytes[8];       /* its size in bytes */
    int64_t total;          /* bytes `out` must hold */
} cmp_image_layout;
int cmp_prepass_layout(cmp_ctx *ctx, int id, int64_t M, int64_t N, int64_t K,
                       cmp_image_layout *layout);
int cmp_prepass_images(cmp_ctx *ctx, int id, const cmp_gemm_args *args, void *out,
                       size_t out_bytes, void *stream);

/* ---- grouped launches: many GEMMs of uneven shapes ---------------------- */

/* A plan runs `count` independent gemm problems (each problem's own alpha,
 * beta and leading dimensions; device pointers owned by the caller and fixed
 * for the plan's lifetime) as ONE persistent kernel whose
 * workgroups take tiles of the concatenated tile list from a device counter
 * as they finish their previous one, problems ordered by decreasing K (the
 * longest tiles first).  A launch zeroes the plan's counter first (a one-lane
 * kernel on the same stream, no memset, so the pair can be captured), and two
 * launches of one plan must not run at the same time (they would share the
 * counter and the problems' C).  A configuration is a tile shape and an
 * arithmetic, one of cmp_grouped_config_count(): the first ones are FP32 SIMT
 * tiles, bit-identical to cmp_gemm_variant with "f32_simt" per problem; the
 * last one runs the "bf16x3" variant's arithmetic (one launch splitting every
 * problem's A and B into bf16 hi / lo images in a workspace the plan owns,
 * then one persistent launch of 256 x 256 MFMA tiles), bit-identical to an
 * unsplit (cmp_set_split_k(1)) "bf16x3" call per problem, and available only
 * when every non-empty problem has alpha != 0 and K > 0 (otherwise
 * CMP_EUNSUPPORTED).  Both arithmetics state the 1e-5 bound.
 * cmp_grouped_config_variant gives the built-in variant id whose results a
 * configuration reproduces.  config < 0 runs the autotuner, which times every
 * available configuration `reps` times on this group (the bf16x3 one with its
 * pre-pass) and keeps the fastest (it runs the products, so C is overwritten:
 * with beta != 0, re-initialise C afterwards).  The launch is also captured in
 * a hipGraph (cmp_grouped_graph_launch).  The plan borrows the context:
 * destroy it before cmp_terminate. */
typedef struct cmp_grouped_plan cmp_grouped_plan;
int cmp_grouped_config_count(void);
int cmp_grouped_config_info(int config, int *bm, int *bn, int *bk);
int cmp_grouped_config_variant(int config, int *variant);
int cmp_grouped_plan_create(cmp_ctx *ctx, int count, const cmp_gemm_args *problems, int config,
                            int reps, void *stream, cmp_grouped_plan **out);
/* config_ms (may be NULL) receives the autotuner's median ms per configuration
 * (NaN where not timed). */
int cmp_grouped_plan_info(const cmp_grouped_plan *plan, int *config, int *problems, int *tiles,
                          int *grid, float *config_ms);
int cmp_grouped_launch(cmp_grouped_plan *plan, void *stream);
int cmp_grouped_graph_launch(cmp_grouped_plan *plan, void *stream);
int cmp_grouped_plan_destroy(cmp_grouped_plan *plan);

/* ---- per-kernel timing (tracing of the built-in variants) ---------------- */

/* When enabled, every kernel launch of the built-in variants is bracketed by
 * a HIP event pair on its launch stream (adds two event records per launch). */
int cmp_kernel_timing(cmp_ctx *ctx, int enable);
/* Totals per kernel name, in name order: idx-th kernel's name, launch count and
 * summed duration in ms (waits for the recorded events).  CMP_ENOTFOUND past
 * the last kernel; idx < 0 resets the totals. */
int cmp_kernel_stats(cmp_ctx *ctx, int idx, char *name, size_t name_len, long long *launches,
                     double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* COMPAR_H */
