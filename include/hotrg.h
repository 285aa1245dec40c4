/*
 * hotrg.h -- C ABI of the MI355X HOTRG coarse-graining library (libhotrg.so).
 *
 * The library runs the Higher Order Tensor Renormalization Group of
 * Yamashita & Sakurai (arXiv 2110.03607) on one gfx950 GPU: the Gram matrices
 * that decide the truncation (Sections 3.2 and 4.2.4), their eigendecomposition
 * (Section 4.2.5), the choice and truncation of the isometries (Sections 2,
 * 4.2.6-4.2.7), the new-tensor contraction in the prime chain / bottleneck /
 * non-prime chain order (Section 4.2.9, eqs. TU1-TUNCD, BottleneckPart,
 * AfterBNNCD-AfterBN1), the renaming of Section 3.1.3, and the lnZ/V
 * bookkeeping of Section 4.1.1 (eqs. eq_lnZ, K_recurrence).
 *
 * Conventions
 *  - Every pointer argument named *_dev is a device pointer (HIP device memory
 *    of the current device); every other pointer is host memory.
 *  - The caller owns all memory.  The library allocates no device memory: the
 *    caller passes a workspace of at least hotrg_workspace_bytes() bytes, which
 *    must stay valid until hotrg_destroy() returns.
 *  - All work is enqueued on the HIP stream passed to hotrg_init (a hipStream_t
 *    passed as void*; NULL means the default stream).  hotrg_step only enqueues
 *    work; errors found on the device surface at the next synchronising call
 *    (hotrg_log_z, hotrg_step_info, hotrg_spectrum, hotrg_grad) and are sticky.
 *  - Functions return a status code (HOTRG_OK on success); nothing throws or
 *    aborts across this interface.  hotrg_last_error() describes the last error.
 *
 * Local-tensor layout on the device (the "storage order")
 *  For a d-dimensional lattice the local tensor with legs
 *      c, n_1, ..., n_{d-1}   (unprimed half)   and   c', n'_1, ..., n'_{d-1}
 *  is stored row-major as T[c][n_1]...[n_{d-1}][c'][n'_1]...[n'_{d-1}], i.e. as
 *  an H x H matrix with H = chi_c * prod_j chi_{n_j}.  c/c' is the Current
 *  direction, n_j/n'_j the direction Next j (Section 3.1.2-3.1.3).
 */
#ifndef HOTRG_H
#define HOTRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define HOTRG_OK         0
#define HOTRG_E_ARG      1  /* invalid argument (NULL, out of range, unsupported) */
#define HOTRG_E_STATE    2  /* call not allowed in the current state of the handle */
#define HOTRG_E_NUMERIC  3  /* trace <= 0 or not finite, eigensolver did not converge */
#define HOTRG_E_OOM      4  /* workspace smaller than hotrg_workspace_bytes() */
#define HOTRG_E_DEVICE   5  /* HIP runtime error */
#define HOTRG_E_NOT_PSD  6  /* the bond weight matrix W has a negative eigenvalue */

/* ---- models (Section 2, eqs. 1-2) ------------------------------------- */
#define HOTRG_ISING 0  /* s = +-1, f = beta J s s', g = beta h s               */
#define HOTRG_POTTS 1  /* q states, f = beta J delta(s, s'), g = 0 (h must be 0) */

/* ---- precision forms of the contraction ------------------------------ */
#define HOTRG_FP64        0  /* FP64 operands, FP64 MFMA, FP64 master tensor        */
#define HOTRG_FP32        1  /* FP32 operands, FP32 MFMA, FP32 master tensor        */
#define HOTRG_BF16        2  /* BF16 operands (RNE), FP32 accumulate                */
#define HOTRG_FP16        3  /* FP16 operands (RNE, power-of-two scaled), FP32 acc. */
#define HOTRG_SPLIT_BF16  4  /* x = hi + lo in BF16; hi*hi + hi*lo + lo*hi, FP32 acc. */
#define HOTRG_SPLIT_FP16  5  /* x = hi + lo in FP16 (scaled); 3 products, FP32 acc.   */

typedef struct hotrg_model {
    int kind;     /* HOTRG_ISING or HOTRG_POTTS                      */
    int d;        /* lattice dimension: 2, 3 or 4                    */
    int q;        /* number of spin states (2 for Ising, >= 2 Potts) */
    double J;     /* coupling (J >= 0; J < 0 gives HOTRG_E_NOT_PSD)  */
    double h;     /* field (Ising only)                              */
} hotrg_model;

/* ---- normalisation factor f^(p) (Section 3.1.3: any f is admissible; lnZ/V does not
 * depend on it, eqs. eq_lnZ, K_recurrence) ------------------------------------------ */
#define HOTRG_NORM_TRACE   0  /* f^(p) = 1 / Tr T^(p)    (the paper's example)            */
#define HOTRG_NORM_MAXABS  1  /* f^(p) = 1 / max |T^(p)| (the largest element becomes 1)  */

/* ---- choice between U and U' (Section 4.2.6: any rational criterion may be used) ---- */
#define HOTRG_CHOOSE_EPSILON 0  /* Section 2: U if epsilon < epsilon', otherwise U'      */
#define HOTRG_CHOOSE_U       1  /* always U (the non-prime side); epsilons still recorded */
#define HOTRG_CHOOSE_UPRIME  2  /* always U' (the prime side)                            */

typedef struct hotrg_opts {
    int precision;    /* HOTRG_FP64 .. HOTRG_SPLIT_FP16                          */
    int max_steps;    /* capacity of the per-step record (diagnostics), >= 1      */
    int chunk;        /* new-tensor columns per chunk in units of (n'_1..,c') groups;
                         0 = automatic.  Bounds the memory of the prime-chain output
                         (the paper's loop over n'_1, Section 4.2.9).            */
    int record_grad;  /* 1: carry d/dbeta through every step (FP64 / FP32 forms,
                         beta > 0, norm = HOTRG_NORM_TRACE); hotrg_grad then
                         returns d(lnZ/V)/dbeta                                    */
    int norm;         /* HOTRG_NORM_TRACE (0) or HOTRG_NORM_MAXABS                 */
    int choice;       /* HOTRG_CHOOSE_EPSILON (0), HOTRG_CHOOSE_U, HOTRG_CHOOSE_UPRIME */
} hotrg_opts;

typedef struct hotrg_handle hotrg_handle;

/* Per-step diagnostics (gauge-invariant quantities), see hotrg_step_info. */
#define HOTRG_MAX_DIRS 4
typedef struct hotrg_step_record {
    int    p;                          /* step number, 1-based                          */
    int    axis;                       /* lattice axis that was coarse-grained          */
    int    dims_before[HOTRG_MAX_DIRS];/* chi_c, chi_{n_1}, .., chi_{n_{d-1}} before      */
    double trace;                      /* Tr T^(p) of the new tensor (before f^(p))     */
    double lnz_per_site;               /* ln Z^(p) / V^(p)                               */
    double gu_wen;                     /* (tr Y)^2 / tr(Y^2), eq. ratio_X               */
    int    chi_new[HOTRG_MAX_DIRS];    /* index j-1: chi_{n_j}^(new)                    */
    double eps[HOTRG_MAX_DIRS];        /* epsilon^(j)  (0 when not truncated)           */
    double eps_p[HOTRG_MAX_DIRS];      /* epsilon'^(j)                                  */
    int    chose_prime[HOTRG_MAX_DIRS];/* 1 when U'^(j) was adopted                     */
    int    truncated[HOTRG_MAX_DIRS];  /* 1 when chi_{n_j}^2 > chi (decomposition done) */
    int    kept[HOTRG_MAX_DIRS];       /* leading columns kept; the rest of the chi_new
                                          columns were zeroed because the cut split a
                                          multiplet of equal eigenvalues             */
} hotrg_step_record;

/* Bytes of device workspace needed for (model, chi, opts).  Returns 0 for an
 * invalid argument. */
size_t hotrg_workspace_bytes(const hotrg_model* model, int chi, const hotrg_opts* opts);

/* Build the initial tensor of eq. (4) on the device, normalise it by
 * f^(0) = 1/Tr T (Section 3.1.3) and record lnZ/V at p = 0.  The first Current
 * direction is lattice axis 0.  beta >= 0 and finite; chi >= q and chi <= 32 (d = 2), 16
 * (d = 3), 12 (d = 4: the register width of the 4D chain kernels).  d = 4 runs have no
 * derivative mode and are not batched.
 * Errors: HOTRG_E_ARG, HOTRG_E_NOT_PSD, HOTRG_E_OOM, HOTRG_E_DEVICE. */
int hotrg_init(const hotrg_model* model, double beta, int chi, const hotrg_opts* opts,
               void* workspace_dev, size_t workspace_bytes, void* hip_stream,
               hotrg_handle** out);

/* Bytes of device workspace for a run started from a supplied tensor (hotrg_init_tensor);
 * 0 for an invalid argument. */
size_t hotrg_tensor_workspace_bytes(int d, const int* dims, int chi, const hotrg_opts* opts);

/* Start a run from a caller-supplied local tensor instead of a lattice model: the method of
 * Sections 3-4 coarse-grains any translation-invariant network of one local tensor.  T0_dev is
 * FP64 device memory in the storage order above with dims[0] = chi_c (lattice axis 0, the first
 * Current direction), dims[j] = chi_{n_j}; 1 <= dims[i], chi <= 32 (d = 2), 16 (d = 3), 12 (d = 4).
 * T0
 * is read (the caller keeps ownership; it may be freed once the stream has passed this call),
 * normalised by f^(0) = 1/Tr T0 (Section 3.1.3), and lnZ/V at p = 0 is ln Tr T0.  opts.record_grad
 * must be 0.  A non-positive or non-finite Tr T0 is reported as HOTRG_E_NUMERIC by the first
 * synchronising call (sticky).  Errors: HOTRG_E_ARG, HOTRG_E_OOM, HOTRG_E_DEVICE. */
int hotrg_init_tensor(int d, const int* dims, const double* T0_dev, int chi, const hotrg_opts* opts,
                      void* workspace_dev, size_t workspace_bytes, void* hip_stream, hotrg_handle** out);

/* Enqueue one coarse-graining step along lattice axis `axis` (0 <= axis < d).
 * Any order is allowed; following the cycle 0, 1, .., d-1, 0, .. of the
 * renaming in Section 3.1.3 needs no re-layout.  The lattice volume doubles.
 * Errors: HOTRG_E_ARG, HOTRG_E_STATE (failed handle, or more than max_steps
 * steps), HOTRG_E_DEVICE. */
int hotrg_step(hotrg_handle* h, int axis);

/* Synchronise and return ln Z^(p) / V^(p) (Section 4.1.1) after the steps so
 * far, in FP64, and the number of steps done (either pointer may be NULL).
 * Errors: HOTRG_E_NUMERIC (sticky), HOTRG_E_DEVICE. */
int hotrg_log_z(hotrg_handle* h, double* lnz_per_site, int* steps_done);

/* Synchronise and copy the diagnostics of step `step` (1-based). */
int hotrg_step_info(hotrg_handle* h, int step, hotrg_step_record* out);

/* Synchronise and copy the normalised eigenvalues lambda_l / lambda_1 (descending)
 * of A^(dir) (side 0) or A'^(dir) (side 1) at step `step`; dir is 1-based.
 * Writes min(cap, available) values and sets *n.  Untruncated steps have none. */
int hotrg_spectrum(hotrg_handle* h, int step, int dir, int side, double* out, int cap, int* n);

/* ---- live timing (HIP events on the library's stream) ----------------------
 * Phases of hotrg_step, timed per launch while profiling is enabled. */
#define HOTRG_T_DECOMP      0  /* Gram matrices + eigendecomposition + choice (4.2.4-4.2.7) */
#define HOTRG_T_PRIME       1  /* prime chain into the B operand (eqs. TU1..TUNCD)          */
#define HOTRG_T_BOTTLENECK  2  /* bottleneck GEMM (eq. BottleneckPart), one entry per chunk */
#define HOTRG_T_NONPRIME    3  /* non-prime chain + renaming (eqs. AfterBNNCD..AfterBN1)    */
#define HOTRG_T_TRACE       4  /* trace, lnZ/V, normalisation (4.2.11, 4.2.15-4.2.17)        */
#define HOTRG_T_CONTRACT    5  /* whole new-tensor contraction incl. the A operand          */
#define HOTRG_T_STEP        6  /* whole hotrg_step                                          */
#define HOTRG_T_COUNT       7
typedef struct hotrg_timing {
    double ms[HOTRG_T_COUNT];     /* summed duration of the phase                     */
    long   count[HOTRG_T_COUNT];  /* number of timed launches (or steps) of the phase */
    double flops_bottleneck;      /* algorithmic flops of the timed bottleneck GEMMs:
                                     2 * M * N * K of the unpadded operands          */
    double flops_contract;        /* algorithmic flops of the whole contraction:
                                     bottleneck + prime chain + non-prime chain      */
} hotrg_timing;

/* Enable (1) or disable (0) timing; enabling clears the accumulators. */
int hotrg_profile(hotrg_handle* h, int enable);

/* Synchronise and return the accumulated timings since profiling was enabled. */
int hotrg_timings(hotrg_handle* h, hotrg_timing* out);

/* Synchronise and return d(lnZ^(p)/V^(p))/dbeta after the steps so far (minus the internal
 * energy per site).  Requires record_grad = 1 at init (else HOTRG_E_STATE).  The derivative
 * is carried forward through every step by the product rule: bond factor, Gram matrices,
 * the leading eigenvectors (over the discarded ones; the choice U/U' and the truncation are
 * held fixed), the multilinear new tensor, trace and normalisation (Sections 2-4). */
int hotrg_grad(hotrg_handle* h, double* dlnz_dbeta_per_site);

/* Release the handle (idempotent on NULL).  Does not free the workspace. */
void hotrg_destroy(hotrg_handle* h);

/* Message describing the last error on h (owned by h), or a static string
 * for h == NULL. */
const char* hotrg_last_error(const hotrg_handle* h);

/* ---- kernel-level entry points (same kernels as hotrg_step) --------------
 * They take FP64 device buffers in the storage order above, apply the given
 * precision form inside, and use the caller's workspace (>= the value returned by
 * hotrg_debug_workspace_bytes).  They synchronise the stream before returning. */

/* Workspace bytes for the kernel-level entry points with local dims
 * dims[0] = chi_c, dims[1..d-1] = chi_{n_j} and new dims kdims[0..d-2]. */
size_t hotrg_debug_workspace_bytes(int d, const int* dims, const int* kdims, int precision);

/* New tensor from T (dims as above) and isometries U_j (row-major
 * chi_{n_j}^2 x kdims[j-1], row index (hat check) = hat + chi_{n_j} * check,
 * Section 3.2).  Writes T^next in the storage order of the renamed tensor
 * (Section 3.1.3: c^bar = n_1, n^bar_j = n_{j+1}, n^bar_{d-1} = c), not normalised. */
int hotrg_debug_contract(int d, const int* dims, const int* kdims, int precision,
                         const double* T_dev, const double* const* U_dev,
                         double* Tnext_dev, void* workspace_dev, size_t workspace_bytes,
                         void* hip_stream);

/* Gram matrices A^(j) (side 0) and A'^(j) (side 1) of Section 3.2 for direction
 * j = dir (1-based): A_dev receives chi_{n_j}^2 x chi_{n_j}^2 FP64, row-major. */
int hotrg_debug_gram(int d, const int* dims, int dir, int side, const double* T_dev,
                     double* A_dev, void* workspace_dev, size_t workspace_bytes,
                     void* hip_stream);

/* Workspace bytes for hotrg_debug_eigh. */
size_t hotrg_debug_eigh_workspace_bytes(int n, int batch);

/* Symmetric eigendecomposition (FP64; Householder tridiagonalisation, bisection,
 * inverse iteration -- the solver used for A and A' in Section 4.2.5) of `batch`
 * (1..4) row-major n x n matrices (1 <= n <= 1024): eigenvalues descending into
 * w_dev[batch][n], eigenvectors as columns of V_dev[batch][n][n] (row-major).
 * A_dev is overwritten.  Errors: HOTRG_E_ARG, HOTRG_E_OOM, HOTRG_E_DEVICE, and
 * HOTRG_E_NUMERIC when the tridiagonal form has a non-finite entry, an eigenvalue is not
 * resolved within the bisection's iteration cap, or an eigenpair's residual
 * ||T z - lambda z|| exceeds 1e-9 |T| (the same failure makes hotrg_step's run fail).  A vector
 * that inverse iteration leaves above that bound is first rebuilt in the orthogonal complement of
 * the earlier vectors, which is a near-null space when its eigenvalue lies at rounding level in a
 * positive semidefinite matrix (a Gram matrix of lower rank than the kept count); the bound is
 * then checked again. */
int hotrg_debug_eigh(int n, int batch, double* A_dev, double* w_dev, double* V_dev,
                     void* workspace_dev, size_t workspace_bytes, void* hip_stream);

/* The eigensolver of a truncating step (Section 4.2.5: only the kept eigenvectors of A and A' are
 * needed): as hotrg_debug_eigh for the leading kvec (1 <= kvec <= n) eigenvectors only.
 * w_dev[b][i] receives the eigenvalues resolved one by one, descending (all n up to n = 256,
 * else the leading max(kvec + 1, 24)), zeros after them; tail_dev[b] the sum of the others
 * (trace of the tridiagonal form minus the resolved ones; 0 when all are resolved); columns
 * 0 .. kvec-1 of V_dev[b] (row-major n x n) the eigenvectors, the other columns untouched.
 * Workspace: hotrg_debug_eigh_workspace_bytes(n, batch).  Errors as hotrg_debug_eigh. */
int hotrg_debug_eigh_lead(int n, int batch, int kvec, double* A_dev, double* w_dev, double* V_dev, double* tail_dev,
                          void* workspace_dev, size_t workspace_bytes, void* hip_stream);

/* ---- measurement -------------------------------------------------------------------------
 * Issue rate of the MFMA instruction a precision form contracts with (FP64: v_mfma_f64_16x16x4,
 * FP32: v_mfma_f32_16x16x4_f32, 16-bit forms: v_mfma_f32_16x16x32_{f16,bf16}), in TFLOP/s, from
 * a kernel whose waves run only independent MFMAs on register operands: the ceiling a
 * contraction kernel of that form can reach on this GPU at its clock under load.  Synchronises
 * `hip_stream`.  Errors: HOTRG_E_ARG, HOTRG_E_DEVICE. */
int hotrg_probe_mfma_rate(int precision, double* tflops, void* hip_stream);

/* ---- allocation-free variant of hotrg_debug_eigh ------------------------------------------
 * For callers that cannot allocate device memory or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same eigensolver and results
 * as hotrg_debug_eigh; its scratch (2 n^2 doubles per matrix) lives in a static device array of
 * hotrg_eigh_noalloc_max_bytes() = 16 MiB that each device holds until the process ends, so
 * batch * 2 * n^2 * 8 <= 16 MiB (n = 1024: batch 1; n <= 724: batch 2; n <= 512: batch 4).
 * Larger requests return HOTRG_E_ARG with nothing enqueued.  The call only enqueues work on
 * `hip_stream` (no allocation, no synchronisation): *status_dev (a device int) is set to 0 and
 * then, if the decomposition failed (as hotrg_debug_eigh's HOTRG_E_NUMERIC), to the first cause
 * found: 1 a non-finite entry, 2 an eigenvalue interval still open at the bisection's iteration
 * cap, 3 an eigenpair residual above its bound.  All calls on
 * one device share the static array: calls that overlap on one device (different streams or
 * host threads without ordering between them) race and give undefined results.
 * Errors: HOTRG_E_ARG, HOTRG_E_DEVICE. */
size_t hotrg_eigh_noalloc_max_bytes(void);
int hotrg_eigh_noalloc(int n, int batch, double* A_dev, double* w_dev, double* V_dev, int* status_dev,
                       void* hip_stream);

/* ---- batched runs: a sweep of independent instances (models, beta, chi) --------------
 * The same coarse-graining step (Sections 3-4) applied to many independent runs, e.g. a
 * temperature sweep with mixed d and chi.  hotrg_batch_step advances every instance by one
 * step along its natural axis cycle (0, 1, .., d-1, 0, ..): the records and Gram matrices of
 * all instances, ONE eigensolver launch over all their Gram matrices, then choice,
 * contraction, trace and normalisation of each instance.  Once every instance has reached
 * dims that a step no longer changes, the step is recorded into a HIP graph (two graphs, for
 * the alternating tensor buffers; the step counter lives on the device) and each later step
 * is one graph launch.  Recording needs a non-NULL stream; on the NULL stream every step is
 * enqueued kernel by kernel.
 * Memory: one caller-owned workspace (256-byte aligned) holding every instance's state and
 * one scratch area sized for the largest instance (instances run one after the other on
 * the stream).  opts applies to all instances; record_grad must be 0. */
typedef struct {
    hotrg_model model;
    double beta;
    int chi;
    int pad;
} hotrg_instance;

typedef struct hotrg_batch hotrg_batch;

/* Workspace bytes for the batch, 0 if an instance or opts is invalid. */
size_t hotrg_batch_workspace_bytes(const hotrg_instance* inst, int n, const hotrg_opts* opts);

/* Builds every instance's initial tensor on `hip_stream` (asynchronous).  Errors as
 * hotrg_init (checked per instance), plus HOTRG_E_ARG for n < 1 or record_grad != 0. */
int hotrg_batch_init(const hotrg_instance* inst, int n, const hotrg_opts* opts, void* workspace,
                     size_t workspace_bytes, void* hip_stream, hotrg_batch** out);

/* One step of every instance (enqueue only; the first steps with new dims may upload an
 * eigensolver descriptor table).  Errors: HOTRG_E_ARG, HOTRG_E_STATE (failed, or max_steps
 * reached), HOTRG_E_DEVICE. */
int hotrg_batch_step(hotrg_batch* b);

/* Synchronise; lnZ/V of every instance into lnz_per_site[n]; steps done into *steps_done
 * (may be NULL).  Device errors of any instance surface here (HOTRG_E_NUMERIC, ...). */
int hotrg_batch_log_z(hotrg_batch* b, double* lnz_per_site, int* steps_done);

/* Autotuner (optional, before the first step; synchronises): for every distinct (d, chi)
 * among the instances, times the saturated new-tensor contraction of one of them with each
 * candidate launch shape (GEMM tiles: 288 x 288 with the non-prime chain in the epilogue for 3D
 * chi = 12 in the reduced forms, 256 x 256 in the reduced forms, 128 x 128 in the 16-bit forms;
 * column chunks of the planned size, 1/2 and 1/4 of it) and keeps the fastest for that class.
 * *nclasses (may be NULL) receives the number of classes.  Errors: HOTRG_E_STATE after the
 * first step, HOTRG_E_DEVICE. */
int hotrg_batch_tune(hotrg_batch* b, int* nclasses);

/* Result of the autotuner for class cls (0 .. nclasses-1): d, chi, the GEMM tile edge used
 * (288, 256 or 128; 0 in the FP64 form, whose GEMM is not a candidate), pair groups per chunk, and the
 * contraction time in ms.  Any output pointer may be NULL.  HOTRG_E_ARG if cls is out of
 * range. */
int hotrg_batch_tuning(hotrg_batch* b, int cls, int* d, int* chi, int* gemm_tile, int* chunk_pairs, double* ms);

/* Steps run as graph launches and steps enqueued kernel by kernel so far. */
int hotrg_batch_info(hotrg_batch* b, int* graph_launches, int* eager_steps);

/* Instance i as a handle for the read-only queries (hotrg_step_info, hotrg_spectrum,
 * hotrg_log_z); it must not be stepped or destroyed.  NULL if i is out of range. */
hotrg_handle* hotrg_batch_instance(hotrg_batch* b, int i);

/* Waits for the batch's stream, then frees the recorded graphs and the instances (the workspace
 * stays the caller's).  Idempotent on NULL. */
void hotrg_batch_destroy(hotrg_batch* b);

/* Message of the last error of b (NULL: of the last failed hotrg_batch_init). */
const char* hotrg_batch_last_error(const hotrg_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* HOTRG_H */
