/*
 * dd.h -- divergence-distance fields and steepest-descent paths on MI355X.
 *
 * C ABI of libdd.so.  The library evaluates, for a target interior vertex t,
 * the total-variation and Kullback-Leibler divergence distances between the
 * discrete Poisson-kernel row of t and the row of every interior vertex x
 * (Section IV, eqs. 34 and 35 of Chen, Gotsman, Hormann, "Path Planning with
 * Divergence-Based Distance Functions"), and traces the edge-based
 * steepest-descent path of Section IV ("Gradient-descent path generation").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns dd_status (DD_OK == 0).  No C++ exception crosses
 *   this boundary.  On failure dd_last_error() returns a message for the most
 *   recent failure on the calling thread; on DD_EINVAL nothing has been written
 *   to any output.
 * - Vertex ids are 0-based interior-vertex ids in [0, N).  Boundary vertices
 *   are not rows: P here is the interior block P_IB of eq. (33).
 * - "Device pointer" means memory on the handle's GPU (hipMalloc, or a torch
 *   CUDA tensor); "host pointer" means ordinary CPU memory.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Field kernels are enqueued on it asynchronously; outputs are valid once
 *   the stream reaches that point.
 * - One dd_kernel may be used from several host threads and streams at once;
 *   per-call scratch memory is stream-ordered (hipMallocAsync on `stream`).
 *   The calls that change a handle (dd_attach_mesh, dd_free_kernel) must not
 *   overlap other calls on the same handle.
 *
 * Error bounds
 * ------------
 * Field entry points can report, per field, a bound {abs, rel} such that
 *     |d_hat(x) - d(x)| <= abs + rel * |d_hat(x)|      for every x,
 * where d_hat is the returned FP32 field and d the exact FP64 evaluation of
 * the same definition on the kernel matrix exactly as it was passed to the
 * load call (upcast to FP64).
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_EINVAL = 1,   /* bad argument or bad input data; nothing written */
  DD_ENOMEM = 2,   /* the HBM footprint does not fit in free device memory */
  DD_EDEVICE = 3,  /* a HIP runtime call failed */
  DD_ESTATE = 4,   /* freed, foreign or mismatched handle */
  DD_ENOCONV = 5   /* an iterative solve stopped at its iteration cap above its
                      tolerance; outputs hold the last iterate */
} dd_status;

typedef enum {
  DD_TV = 0,  /* total variation, eq. (34): sum_b |P_tb - P_xb|, range [0, 2] */
  DD_KL = 1,  /* Kullback-Leibler, eq. (35): sum_b P_tb log(P_tb / P_xb), target row as reference */
  /* Two more f-divergences d = sum_b P_tb f(P_xb / P_tb) (Section VI names the
   * family); dense handles only, a truncated (CSR) handle rejects them with
   * DD_EINVAL. */
  DD_CHI2 = 2,      /* chi-squared, f(u) = (u - 1)^2: sum_b (P_xb - P_tb)^2 / P_tb,
                       +inf when P_xb > 0 where P_tb = 0 */
  DD_HELLINGER = 3  /* squared Hellinger, f(u) = (sqrt u - 1)^2:
                       sum_b (sqrt P_xb - sqrt P_tb)^2, range [0, 2] */
} dd_kind;

/* The two families Section VI names, as kind values (dense handles only):
 *   DD_KIND_POWER(k)         f(u) = |1 - u|^k, integer 1 <= k <= 16:
 *                            sum_b |P_xb - P_tb|^k / P_tb^(k-1) (k = 1 is TV,
 *                            k = 2 chi-squared; +inf as for chi-squared)
 *   DD_KIND_ALPHA_EIGHTHS(m) alpha-divergence with alpha = m/8, -7 <= m <= 7:
 *                            4/(1 - alpha^2) sum_b (P_tb - P_tb^((1-alpha)/2)
 *                            P_xb^((1+alpha)/2)) (m = 0 is twice Hellinger) */
#define DD_KIND_POWER(k) (100 + (k))
#define DD_KIND_ALPHA_EIGHTHS(m) (208 + (m))

/* Operand form of the batched-KL contraction (see dd_batch_distance_fields). */
typedef enum {
  DD_FORM_NONE = -1,   /* do not build a batched-KL operand */
  DD_FORM_F32 = 0,     /* FP32 log-kernel, FP32 MFMA */
  DD_FORM_F16X3 = 1,   /* FP16 hi+lo split of the log-kernel and of the targets, 3 MFMA products */
  DD_FORM_BF16X3 = 2,  /* BF16 hi+lo split (8 + 8 significant bits, no scaling of the targets),
                          3 MFMA products; a looser stated bound (3 x 2^-16 relative per term) */
  DD_FORM_F16 = 3      /* the FP16 hi parts alone (11 significant bits each), one MFMA product:
                          2 bytes per operand entry, half the bytes of F16X3; stated bound
                          2^-10 + 2^-22 relative per term on top of the accumulation */
} dd_form;

/* Storage of the stored values of a truncated (CSR) handle, as read by the
 * field entry points.  The FP32 values stay resident in both forms: the path
 * entry points re-decide near-ties from them (or from the FP64 input). */
typedef enum {
  DD_CSR_F32 = 0,   /* FP32 values: 6 bytes per stored entry with the column */
  DD_CSR_F16 = 1    /* FP16 values scaled per row by a power of two (row max in
                       [2^14, 2^15)): 4 bytes per stored entry; each value is
                       within 2^-11 relative of the FP32 value, and the stated
                       bounds include that rounding.  Needs every row's floor
                       phi_x >= 2^-28 max_b P_xb and max_b P_xb >= 2^-100. */
} dd_csr_values;

typedef enum {
  DD_PATH_REACHED = 0,   /* the walk arrived at the target */
  DD_PATH_STUCK = 1,     /* no neighbour strictly lower: a local minimum (or plateau) */
  DD_PATH_MAX_STEPS = 2  /* max_steps moves made without arriving */
} dd_path_status;

typedef struct dd_ctx dd_ctx;
typedef struct dd_kernel dd_kernel;

/* Interior-vertex adjacency (the triangulation edges between interior
 * vertices), CSR on the host.  Neighbour lists must be sorted ascending, hold
 * no duplicates and no self loops.  Copied by the load call. */
typedef struct {
  int32_t n;               /* must equal N */
  const int64_t* row_ptr;  /* [n+1], row_ptr[0] == 0, non-decreasing */
  const int32_t* col;      /* [row_ptr[n]] ids in [0, n) */
} dd_adjacency;

typedef struct {
  int32_t gemm_form;     /* dd_form built for dd_batch_distance_fields with DD_KL; with
                            tau > 0 the floored operand (dense loads, FP32 values only) */
  double tau;            /* > 0: keep only the truncation of P (CSR form); 0: dense */
  int32_t tau_relative;  /* 1: keep P_xb >= tau * max_b P_xb; 0: keep P_xb >= tau */
  int32_t validate;      /* 1: reject rows that are not probability vectors */
  int32_t csr_values;    /* dd_csr_values of a truncated handle (ignored when dense) */
} dd_load_opts;

typedef struct {
  double abs;
  double rel;
} dd_error_bound;

typedef struct {
  int32_t n;           /* N, interior rows */
  int32_t b_in;        /* columns as loaded */
  int32_t b;           /* columns kept (all-zero columns dropped) */
  int32_t is_csr;      /* 1 if the handle holds the truncated (CSR) form */
  int64_t nnz;         /* stored nonzeros of the CSR form (0 if dense) */
  int32_t gemm_form;   /* dd_form built, or DD_FORM_NONE */
  int32_t has_adjacency;
  size_t hbm_bytes;    /* device memory held by the handle */
  int32_t csr_values;  /* dd_csr_values read by the field entry points (truncated handles) */
} dd_kernel_info;

/* Create a context on HIP device `device`.  *out receives the handle.  The
 * first context on a device in a process also checks the device's FP32
 * hardware log2 on every FP32 value in [2^-126, 1] (a few milliseconds; see
 * dd_path_level1). */
dd_status dd_create(int device, dd_ctx** out);

/* Level-1 re-decisions of KL walks on dense handles (dd_trace_paths; the
 * steepest-descent rule of Section IV).  A near-tie is first re-decided on
 * row values from FP32 hardware logarithms summed in FP64, each with a
 * stated bound that covers both the exact value and the FP64 evaluation;
 * only when those intervals do not settle the step are the rows computed in
 * FP64.  Either way the step is the one the FP64 values give, so paths do
 * not change; only the cost of a re-decision does.  The bounds assume that
 * the hardware log2 L meets |L(x) - log2 x| <= 2^-22 |log2 x| + 2^-40 on
 * [2^-126, 1], which dd_create checks exhaustively; level 1 is on by default
 * where the check passed.
 *   enable   1 on (DD_EINVAL if the device failed the check), 0 off, -1 query
 *   enabled  host, nullable: the state after the call
 *   ratios   host [2], nullable: the check's largest error over the assumed
 *            bound (<= 1 passes), and its largest relative error
 * Per context; not thread-safe against calls that trace paths. */
dd_status dd_path_level1(dd_ctx* ctx, int enable, int* enabled, double* ratios);

/* Destroy a context.  Every kernel loaded through it must be freed first
 * (DD_ESTATE otherwise, and the context stays valid). */
dd_status dd_destroy(dd_ctx* ctx);

/* Load a dense Poisson-kernel matrix P (N x B, row-major, row stride B).
 *
 * The matrix is the interior block P_IB of eq. (33): row x is the discrete
 * harmonic measure of interior vertex x over the B boundary vertices
 * (Section IV, "The divergence distances").
 *   P           host or device pointer to N*B values, FP32 (p_is_f64 == 0) or
 *               FP64 (p_is_f64 == 1); p_on_device says which memory it is.
 *   adj         nullable; needed by the path entry points.
 *   opts        nullable (defaults: gemm_form DD_FORM_NONE, tau 0, validate 1,
 *               csr_values DD_CSR_F32).
 * Entries must be finite and >= 0; positive entries below the FP32 normal
 * range (1.17549435e-38) are rejected.  With validate, every row sum must be
 * 1 within 1e-5 (FP32 input) or 1e-9 (FP64 input).  All-zero columns are
 * dropped (they contribute nothing to eqs. 34-35).  With opts->tau > 0 the
 * handle holds the truncated matrix only (see dd_load_kernel_csr).
 * The input is copied; the caller may free it on return.  The library owns
 * the device copy until dd_free_kernel.  Synchronous. */
dd_status dd_load_kernel_dense(dd_ctx* ctx, int32_t N, int32_t B, const void* P,
                               int32_t p_is_f64, int32_t p_on_device,
                               const dd_adjacency* adj, const dd_load_opts* opts,
                               dd_kernel** out);

/* Load a truncated (sparsified) Poisson kernel in CSR form (Section V,
 * "Precision": small entries of each row dropped, no renormalisation).
 *   row_ptr   host [N+1] int64; col host [nnz] int32 in [0, B), ascending per
 *             row; val host [nnz] FP32 or FP64 (val_is_f64), all > 0.
 *   row_max   host [N] FP64: max_b P_xb of the untruncated row x.
 *   tau, tau_relative: the threshold the truncation used; the floor of row x
 *             is phi_x = tau * row_max[x] (relative) or tau (absolute).
 * Fields on this handle are the truncated ones:
 *   TV_tau(x) = sum_b |P~_tb - P~_xb|
 *   KL_tau(x) = sum_{b: P~_tb > 0} P~_tb (log P~_tb - log Q_xb),
 *               Q_xb = P~_xb if stored, else phi_x.
 * Copies its inputs.  Synchronous. */
dd_status dd_load_kernel_csr(dd_ctx* ctx, int32_t N, int32_t B, const int64_t* row_ptr,
                             const int32_t* col, const void* val, int32_t val_is_f64,
                             const double* row_max, double tau, int32_t tau_relative,
                             const dd_adjacency* adj, const dd_load_opts* opts,
                             dd_kernel** out);

/* Sizes and device memory held by a handle. */
dd_status dd_kernel_get_info(const dd_kernel* k, dd_kernel_info* info);

/* Device memory resident in a handle (the hbm_bytes of dd_kernel_get_info):
 * admission control of further loads against free memory. */
dd_status dd_kernel_footprint(const dd_kernel* k, size_t* hbm_bytes);

/* Device scratch that one call on this handle allocates while it runs, on top
 * of the resident bytes and of the caller's output buffers: fields_bytes for
 * dd_batch_distance_fields with T targets of `kind`, paths_bytes for
 * dd_trace_paths with T paths (0 without adjacency).  Either output nullable.
 * Admission of a launch against free device memory. */
dd_status dd_call_scratch_bytes(const dd_kernel* k, int32_t T, int32_t kind, size_t* fields_bytes,
                                size_t* paths_bytes);

/* Device bytes a dense load of an N x B matrix with these options would
 * need (admission control before loading). */
dd_status dd_dense_footprint(int32_t N, int32_t B, int32_t p_is_f64, const dd_load_opts* opts,
                             size_t* hbm_bytes);

/* Distance field of one target (eq. 34 or 35, or the truncated forms on a
 * CSR handle) into out_dev[N] (device FP32).  One streaming pass over the
 * kernel rows.  bound: nullable host pointer.  Asynchronous on `stream`. */
dd_status dd_distance_field(dd_kernel* k, int32_t target, int32_t kind, float* out_dev,
                            dd_error_bound* bound, void* stream);

/* The TV field (eq. 34) and the KL field (eq. 35) of one target in one pass
 * over the rows: the values, and the bounds, of two dd_distance_field calls
 * (DD_TV into tv_dev, DD_KL into kl_dev) for the bytes of one.  Dense and
 * truncated handles (on a truncated handle, TV_tau and KL_tau).
 *   tv_dev, kl_dev  device [N] FP32 each, distinct
 *   bounds          host [2] (TV, KL), nullable
 * Asynchronous on `stream`. */
dd_status dd_distance_fields_tv_kl(dd_kernel* k, int32_t target, float* tv_dev, float* kl_dev,
                                   dd_error_bound* bounds, void* stream);

/* Distance fields of T targets into out_dev[T][N] (device FP32, one field
 * contiguous per target).  targets: host [T].  For DD_KL on a dense handle
 * built with a gemm_form the fields come from one contraction,
 *     d(x,t) = H_t - o_x W_t - sum_b P_tb l_xb,
 * with l_xb = log P_xb - o_x, o_x = log max_b P_xb, H_t = sum_b P_tb log P_tb
 * and W_t = sum_b P_tb (eq. 35 expanded).  On a truncated (CSR) handle with
 * T >= 8, TV or KL, the fields come from one pass over the stored rows per
 * group of up to 256 targets, with
 *     TV_tau(x,t) = W_t + Q_x - 2 sum_{b in S_x} min(P~_xb, P~_tb),
 *     KL_tau(x,t) = H_t - log(phi_x) W_t - sum_{b in S_x} P~_tb log(P~_xb / phi_x)
 * (Q_x = sum_{b in S_x} P~_xb; the truncated fields of dd_load_kernel_csr
 * rearranged); a target's field is then bit-identical in every such batch.
 * DD_KL on a truncated handle loaded dense with a gemm_form instead takes the
 * contraction over the floored kernel, for any T:
 *     KL_tau(x,t) = H~_t - o_x W~_t - sum_b P~_tb l~_xb,
 *     l~_xb = log max(P_xb, phi_x) - o_x
 * (P^_xb = max(P_xb, phi_x) is the stored value or the floor; H~_t and W~_t
 * are sums over the truncated target row).
 * Otherwise one streaming pass per target.  bounds: nullable host [T].
 * Asynchronous on `stream`. */
dd_status dd_batch_distance_fields(dd_kernel* k, const int32_t* targets, int32_t T,
                                   int32_t kind, float* out_dev, dd_error_bound* bounds,
                                   void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Same arguments, fields and bounds as dd_batch_distance_fields (the same
 * kernels run, so the fields are bit-identical), but the call's device
 * scratch -- the target operands of the contraction, the target block of the
 * many-target pass, the expanded truncated target rows -- is taken from a
 * fixed buffer of DD_NOALLOC_SCRATCH_BYTES that the library holds on each GPU
 * it runs on until the process ends, and the call allocates and frees nothing.
 * The caller still passes targets, outputs and bounds.
 *   DD_EINVAL   the call would need more scratch than the buffer holds (the
 *               need grows with min(T, 256) and the kept columns; the FP64 rows
 *               of a truncated handle loaded from FP64 values with a gemm_form
 *               are the largest part); nothing has been enqueued.
 * Every call on a GPU, from any context or thread, shares that GPU's buffer,
 * which keeps the last call's contents: calls that overlap on one GPU race
 * and give wrong fields, so a call may start only after the stream of the
 * previous call has reached its end.  No contents need clearing between calls
 * (each call writes, with kernels, every byte it reads; no memset is
 * enqueued).  Asynchronous on `stream`. */
#define DD_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
dd_status dd_batch_distance_fields_noalloc(dd_kernel* k, const int32_t* targets, int32_t T,
                                           int32_t kind, float* out_dev, dd_error_bound* bounds,
                                           void* stream);

/* Trace T steepest-descent paths on precomputed fields (Section IV, edge-based
 * variant): from v = source[i], move to the neighbour with the smallest field
 * value (ties: lowest id) while it is strictly below the current value.
 * Decisions whose FP32 values are within the stated bounds of each other are
 * re-decided in FP64 from the loaded matrix.
 *   fields_dev   device [T][N] FP32 from the field entry points for targets[i]
 *   bounds       host [T], the bounds those calls returned
 *   sources, targets  host [T]
 *   path_dev     device [T][max_steps+1] int32, vertex ids, -1 past the end
 *   len_dev      device [T] int32 path lengths (vertices, source included)
 *   status_dev   device [T] int32 dd_path_status
 *   rechecks_dev device [T] int32 re-decisions (level 1 or FP64, see
 *                dd_path_level1), nullable
 * Needs the adjacency.  Asynchronous on `stream`. */
dd_status dd_trace_paths(dd_kernel* k, int32_t T, const int32_t* sources, const int32_t* targets,
                         int32_t kind, const float* fields_dev, const dd_error_bound* bounds,
                         int32_t max_steps, int32_t* path_dev, int32_t* len_dev,
                         int32_t* status_dev, int32_t* rechecks_dev, void* stream);

/* Paths with distances evaluated on demand (Section V: the CPU evaluates
 * the distances only at the vertices the path needs): no field is given; at
 * each step the distances of the current vertex's neighbours are computed
 * from the resident rows (for DD_KL on a dense handle first as level-1 values,
 * see dd_path_level1, and in FP64 where those do not settle the step) and the
 * walk of dd_trace_paths is taken on them, so the path is the one the exact
 * FP64 field gives.
 *   kind          as for the field entry points (dense: all kinds; CSR: TV, KL
 *                 of the truncated rows)
 *   target_tau    0, or with DD_KL on a dense handle the truncation of the
 *                 target row before the sums (the target-support KL of
 *                 dd_support_kl_field); row-relative if target_tau_relative
 *   sources, targets  host [T]
 *   path_dev, len_dev, status_dev  as for dd_trace_paths
 *   evals_dev     device [T] int32 rows evaluated per path (each row counted
 *                 once, whether at level 1, in FP64 or both), nullable
 * Needs the adjacency.  Asynchronous on `stream`. */
dd_status dd_trace_paths_on_demand(dd_kernel* k, int32_t T, const int32_t* sources,
                                   const int32_t* targets, int32_t kind, double target_tau,
                                   int32_t target_tau_relative, int32_t max_steps,
                                   int32_t* path_dev, int32_t* len_dev, int32_t* status_dev,
                                   int32_t* evals_dev, void* stream);

/* KL summed over the truncated support of the target row, with the rows of
 * x kept exact (the sparse KL of Section V, "Precision"):
 *     d(x) = sum_{b in S_t} P_tb log(P_tb / P_xb),
 *     S_t  = {b : P_tb > 0, P_tb >= thr}, thr = tau * max_b P_tb (tau_relative)
 *            or tau,
 * into out_dev[N] (device FP32).  The support is decided on the FP64 master
 * row when the handle has one.  One streaming pass that reads only the
 * 16-byte row pieces meeting S_t.  tau = 0 gives the DD_KL field bit for bit.
 * Dense handles only.  bound: nullable host pointer (the DD_KL bound, which
 * covers this subset of its terms).  Asynchronous on `stream`. */
dd_status dd_support_kl_field(dd_kernel* k, int32_t target, double tau, int32_t tau_relative,
                              float* out_dev, dd_error_bound* bound, void* stream);

/* Attaches the triangle mesh of the interior for triangle-based paths.
 *   faces  host [n_faces][3] int32 vertex ids in [0, N) (interior-local, as
 *          the rows of the kernel), any orientation (stored counter-clockwise);
 *          only triangles whose three vertices are interior belong here
 *   xy     host [N][2] FP64 vertex coordinates
 * Zero-area faces, repeated vertices, an edge shared by more than two faces
 * or a vertex in more than 64 faces give DD_EINVAL.  Replaces an earlier mesh.
 * Synchronous. */
dd_status dd_attach_mesh(dd_kernel* k, int32_t n_faces, const int32_t* faces, const double* xy);

/* Triangle-based steepest-descent paths on precomputed fields (Section IV,
 * "Gradient-descent path generation", the method of the paper's figures):
 * the field is linear on each triangle; from the source the descent
 * direction of an incident triangle that points into it is followed across
 * triangles; at a vertex with no such triangle the path takes the steepest
 * decreasing incident edge; where the next triangle is missing or its descent
 * direction points back, it slides along the edge to the lower endpoint; an
 * edge incident on the target ends the path at the target.  Geometry in FP64
 * on the given FP32 field values.
 *   fields_dev  device [T][N] FP32
 *   points_dev  device [T][max_steps+1][2] FP64 path points (0 past the end)
 *   where_dev   device [T][max_steps+1][2] int32: (v, -1) for vertex v, (a, b)
 *               with a < b for a point inside edge ab, (-1, -1) past the end
 *   len_dev     device [T] points per path (source included)
 *   status_dev  device [T] dd_path_status
 * Needs the mesh (dd_attach_mesh) and the adjacency.  Asynchronous on
 * `stream`. */
dd_status dd_trace_paths_triangles(dd_kernel* k, int32_t T, const int32_t* sources,
                                   const int32_t* targets, const float* fields_dev,
                                   int32_t max_steps, double* points_dev, int32_t* where_dev,
                                   int32_t* len_dev, int32_t* status_dev, void* stream);

/* dd_trace_paths_triangles on FP64 fields (from dd_exact_distance_fields):
 * every decision of the tracer -- the incident triangle, the exit edge, the
 * slide along an edge, the corner snap -- is then taken on FP64 values, so
 * the path is the one the exact field gives up to the rounding of its FP64
 * sums.  fields_dev: device [T][N] FP64.  Other arguments as for
 * dd_trace_paths_triangles.  Asynchronous on `stream`. */
dd_status dd_trace_paths_triangles_f64(dd_kernel* k, int32_t T, const int32_t* sources,
                                       const int32_t* targets, const double* fields_dev,
                                       int32_t max_steps, double* points_dev, int32_t* where_dev,
                                       int32_t* len_dev, int32_t* status_dev, void* stream);

/* FP64 distance fields of T targets (eqs. 34-35, or the truncated forms on a
 * CSR handle, or the other kinds on a dense handle) into out_dev[T][N]
 * (device FP64): every term and sum in FP64 from the rows as loaded, the
 * evaluation the FP64 re-decisions of the path entry points use (one FP64
 * logarithm per entry for KL, so much slower than the FP32 fields); d(t, t)
 * is 0.  For decisions that need the exact field, such as
 * dd_trace_paths_triangles_f64.  targets: host [T], T <= 65535.
 * Asynchronous on `stream`. */
dd_status dd_exact_distance_fields(dd_kernel* k, const int32_t* targets, int32_t T, int32_t kind,
                                   double* out_dev, void* stream);

/* Spurious local minima of T fields (Section V, "Low resolution
 * discretizations"): a vertex v other than the target is a local minimum when
 * no neighbour u has d(u) < d(v).  Each vertex is classified against the
 * field's stated bound:
 *   0  not a minimum: some neighbour is certainly lower,
 *   1  certainly a minimum: every neighbour is certainly not lower,
 *   2  undecided within the bound (exact ties included).
 *   fields_dev  device [T][N] FP32; bounds host [T]; targets host [T]
 *   class_dev   device [T][N] uint8 classes (nullable)
 *   counts_dev  device [T][2] int32: certain minima, undecided (nullable)
 * Needs the adjacency.  Asynchronous on `stream`. */
dd_status dd_local_minima(dd_kernel* k, int32_t T, const int32_t* targets, const float* fields_dev,
                          const dd_error_bound* bounds, uint8_t* class_dev, int32_t* counts_dev,
                          void* stream);

/* FP64 re-decision of a local-minimum census (Section V, "Low resolution
 * discretizations"): every entry of class 2 (undecided) in class_dev, as
 * dd_local_minima left it for these targets and kind, becomes 1 or 0 from the
 * FP64 distances of the vertex and its neighbours, evaluated from the loaded
 * matrix (1: no neighbour strictly lower, the census rule).  counts_dev
 * (nullable, device [T][2]) is recomputed: minima, and 0 undecided.  Costs
 * (1 + degree) FP64 row evaluations per undecided vertex.  Asynchronous on
 * `stream`. */
dd_status dd_resolve_minima(dd_kernel* k, int32_t T, const int32_t* targets, int32_t kind,
                            uint8_t* class_dev, int32_t* counts_dev, void* stream);

/* Plan one path: the field of `target` (dd_distance_field) followed by the
 * path from `source` (dd_trace_paths).  path_host must hold max_steps+1
 * entries.  rechecks nullable.  Synchronous with respect to `stream`. */
dd_status dd_plan_path(dd_kernel* k, int32_t source, int32_t target, int32_t kind,
                       int32_t max_steps, int32_t* path_host, int32_t* len,
                       int32_t* status, int32_t* rechecks, void* stream);

/* Statistics of dd_grid_poisson_kernel. */
typedef struct {
  int32_t iterations;        /* CG iterations of the slowest column batch */
  int32_t batches;           /* column batches solved */
  int32_t levels;            /* multigrid levels */
  int32_t total_iterations;  /* CG iterations summed over the batches */
  double max_rel_residual;   /* max over columns of ||r|| / ||b|| at exit */
} dd_grid_solve_stats;

/* Poisson kernel P_IB of a grid domain computed on the device (the
 * preprocessing of Section IV, eqs. 32-33): column b is the discrete harmonic
 * function on the interior vertices with boundary values the indicator of
 * boundary vertex b.  On the right-triangle grid the cotangent Laplacian is
 * the five-point stencil, so each column solves
 *   4 u_v - sum_{interior n ~ v} u_n = #{boundary n ~ v : n = b}.
 *   G          vertices per grid side, 3 <= G <= 46340.
 *   node_type  host [G*G] uint8, vertex (i, j) at index j*G + i: 0 = not in
 *              the domain, 1 = interior, 2 = boundary.  Interior vertices
 *              may not lie on the grid's edge, and each of their four axis
 *              neighbours must be interior or boundary.  Rows of P are the
 *              interior vertices and columns the boundary vertices, each in
 *              ascending index order (N and K their counts).
 *   col_begin, ncols  the columns [col_begin, col_begin + ncols) of P_IB to
 *              compute (0 <= col_begin, 1 <= ncols, col_begin + ncols <= K).
 *   P32        nullable device [N][ld32] FP32 (ld32 >= ncols): column
 *              col_begin + c of P_IB is written at position c of each row.
 *   P64        nullable device [N][ld64] FP64, likewise; at least one of the two.
 *              Entries are max(u, 0); other columns of the rows are untouched.
 *   tol        relative residual ||b - A u|| / ||b|| each column must reach.
 *   max_iter   conjugate-gradient iteration cap per column batch (>= 1).
 *   batch      columns solved together (a multiple of 64), or 0 to choose from
 *              free device memory.
 *   stats      nullable host output.
 * Conjugate gradients with a geometric multigrid preconditioner in FP64; the
 * library allocates its workspace (about 5 x 8 x G^2 x batch bytes) for the
 * call and frees it on return.  DD_ENOCONV if a column is above tol at the
 * cap (the outputs then hold the last iterate), DD_ENOMEM if the workspace
 * for 64 columns does not fit.  Synchronous on `stream`. */
dd_status dd_grid_poisson_kernel(dd_ctx* ctx, int32_t G, const uint8_t* node_type,
                                 int32_t col_begin, int32_t ncols, float* P32, int64_t ld32,
                                 double* P64, int64_t ld64, double tol, int32_t max_iter,
                                 int32_t batch, dd_grid_solve_stats* stats, void* stream);

/* The discrete Dirichlet Green's function of a grid domain, the comparison
 * distance D of the paper (Section IV, "The Dirichlet Green's function",
 * eqs. 19-22): for each pole p = poles[c], the column
 *     D_Ip = (-L_II)^{-1} e_p,
 * harmonic at every interior vertex but p, zero on the boundary, positive and
 * largest at p; paths descend -D towards p.  The operator, grid description,
 * solver, tol, max_iter, batch and stats are those of dd_grid_poisson_kernel
 * (on the right-triangle grid -L_II is the five-point stencil, so column c
 * solves 4 u_v - sum_{interior n ~ v} u_n = [v = p]).
 *   poles      host [T] interior-vertex ids in [0, N) (interior vertices in
 *              ascending grid index, as the rows of P_IB)
 *   D32        nullable device [T][ld32] FP32 (ld32 >= N): row c is D_Ip over
 *              the interior vertices
 *   D64        nullable device [T][ld64] FP64, likewise; at least one of the two
 * DD_EINVAL for a pole outside [0, N) or a bad grid; DD_ENOCONV if a column is
 * above tol at the cap.  Synchronous on `stream`. */
dd_status dd_grid_green_function(dd_ctx* ctx, int32_t G, const uint8_t* node_type,
                                 const int32_t* poles, int32_t T, float* D32, int64_t ld32,
                                 double* D64, int64_t ld64, double tol, int32_t max_iter,
                                 int32_t batch, dd_grid_solve_stats* stats, void* stream);

/* Release a handle and its device memory (waits for the device first). */
dd_status dd_free_kernel(dd_kernel* k);

/* Message of the last failure on this thread ("" if none). */
const char* dd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
