/*
 * tci_c.h -- C ABI of the MI355X (gfx950) two-site MPS update library.
 *
 * The calls follow the problem statement of the Tensor Computing Interface
 * (TCI, arXiv:2512.23917): a typed tensor with shape and bond labels,
 * transpose/reshape, label-based contraction, QR, (truncated) SVD, norms.
 * "Spec" below is the paper's appendix that specifies the TCI API; the
 * subsection and function named after it is the passage each call follows.
 *
 * Conventions for every function:
 *   - Return value: tci_status, TCI_OK (0) on success.  On failure the
 *     message of the last error is available from tci_last_error() (per
 *     thread) and outputs of out-of-place calls are left unchanged.
 *   - Tensors are dense and row-major (last index fastest); the reshape
 *     passage of the Spec fixes that reshaping keeps the memory order.
 *   - Element types: TCI_F32, TCI_F64, TCI_C64 (2 x float), TCI_C128
 *     (2 x double, the layout of C99 double complex).
 *   - Device memory: tensor data lives in the context's GPU memory.  A
 *     tensor created by tci_allocate / tci_zeros / tci_copy owns it; one
 *     created by tci_wrap borrows memory the caller keeps alive.
 *   - Output tensors are handles created by the caller (any shape, e.g. by
 *     tci_allocate with order 0); the library sets their shape and, for
 *     owning handles, re-allocates their storage when it is too small.  A
 *     wrapped (borrowing) output must already be large enough, otherwise
 *     TCI_ERR_SHAPE.
 *   - All work is ordered on the context's HIP stream.  Calls that return
 *     host scalars or data-dependent shapes (norm, trunc_svd, qr, close,
 *     the update composites) synchronise that stream before returning.
 *   - Using a handle after it was destroyed is undefined (Spec, context
 *     routines: a destroyed context must not be used again).
 */
#ifndef TCI_C_H
#define TCI_C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tci_status;
#define TCI_OK 0
#define TCI_ERR_INVALID_ARGUMENT 1  /* null handle, bad k_rows, chi_min > chi_max, ... */
#define TCI_ERR_SHAPE 2             /* dimension mismatch, output too small */
#define TCI_ERR_LABEL 3             /* bad label lists in contract */
#define TCI_ERR_DTYPE 4             /* unsupported or mismatched element type */
#define TCI_ERR_OUT_OF_MEMORY 5     /* device allocation failed */
#define TCI_ERR_DEVICE 6            /* any HIP runtime error (message has hipGetErrorString) */
#define TCI_ERR_NOT_CONVERGED 7
#define TCI_ERR_NUMERIC 8           /* NaN / Inf where a finite value is required */
#define TCI_ERR_UNSUPPORTED 9
#define TCI_ERR_INTERNAL 10         /* an unexpected C++ exception inside the library (never escapes) */

typedef enum { TCI_F32 = 0, TCI_F64 = 1, TCI_C64 = 2, TCI_C128 = 3 } tci_dtype;

/* Arithmetic of contractions: FP64 matrix cores; FP32 matrix cores with FP32
 * accumulation; split-BF16 x3 (x = hi + lo, three bf16 products, FP32
 * accumulation).  FP64 requires F64/C128 tensors, the others F32/C64. */
typedef enum { TCI_PREC_FP64 = 0, TCI_PREC_FP32 = 1, TCI_PREC_BF16X3 = 2 } tci_precision;

/* Truncated-SVD method inside the update composites. */
typedef enum {
  TCI_SVD_PLAIN = 0,       /* Gram matrix + Householder tridiagonal eigensolver, all FP64 */
  TCI_SVD_RANDOMIZED = 1,  /* sketch of rank params.sketch_rank, plain SVD as fallback */
  TCI_SVD_LEARNED = 2      /* sketch rank predicted by a tci_sketch_model, plain as fallback */
} tci_svd_mode;

/* Write-back of the factors after the two-site update. */
typedef enum {
  TCI_DIR_LEFT = 0,   /* A' = U,            B' = diag(s) V^dagger  (centre moves right) */
  TCI_DIR_RIGHT = 1,  /* A' = U diag(s),    B' = V^dagger          (centre moves left)  */
  TCI_DIR_VIDAL = 2   /* A' = diag(1/lambda_l) U,  B' = V^dagger diag(1/lambda_r): the Gamma
                         tensors of the Vidal form (App. A); s is the new Lambda */
} tci_direction;

typedef struct tci_context_s* tci_context;
typedef struct tci_tensor_s* tci_tensor;
typedef struct tci_sketch_model_s* tci_sketch_model;

/* ------------------------------------------------------------------ */
/* Version and errors (Spec, miscellaneous routines: version)          */
/* ------------------------------------------------------------------ */

/* Returns the interface version "1.0" (static string, never NULL). */
const char* tci_version(void);

/* Message of the last failed call on this thread ("" if none).  Static
 * per-thread storage, valid until the next failing call on the thread. */
const char* tci_last_error(void);

/* ------------------------------------------------------------------ */
/* Context (Spec, miscellaneous routines: create_context,               */
/* destroy_context)                                                     */
/* ------------------------------------------------------------------ */

/* Device-memory allocator of a context.  Every device buffer the library
 * allocates for the context (tensor storage, block-sparse storage, sketch
 * models, workspace chunks) comes from alloc and goes back through free with
 * the same size; hip_stream is the context's stream at that moment.  alloc
 * returns NULL on failure, and the call that needed the memory then fails
 * with TCI_ERR_OUT_OF_MEMORY.  Workspace is requested in chunks of at least
 * 256 MiB and kept until the context is destroyed.  alloc and free are both
 * set or both NULL (NULL: hipMalloc / hipFree). */
typedef struct {
  void* (*alloc)(size_t bytes, void* hip_stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* hip_stream, void* user);
  void* user;
} tci_allocator;

/* Implementation-defined parameters of create_context (Spec, miscellaneous
 * routines: create_context names allocators and logging flags as examples). */
typedef struct {
  tci_allocator allocator;
  int32_t precision;          /* tci_precision of F32 / C64 contractions; -1: TCI_PREC_FP32 */
  int32_t svd_mode;           /* tci_svd_mode of tci_trunc_svd and of the update composites called
                                 with params NULL: TCI_SVD_PLAIN, or TCI_SVD_RANDOMIZED (a sketch of
                                 rank chi_max + 64 rounded up to 32, two power iterations, kept only
                                 when the discarded weight meets a positive target and the residual
                                 certificate holds; the plain SVD otherwise).  TCI_SVD_LEARNED needs
                                 per-call spectra and a model, so it is set in tci_update_params */
  const char* autotune_cache; /* file of tuned grouped-GEMM tile shapes: read when the context is
                                 created (a missing file is not an error), rewritten when it is
                                 destroyed; NULL: no file.  The string is copied. */
  int32_t verbosity;          /* 0, 1, 2 as TCI_VERBOSE; -1: from the environment */
} tci_context_opts;

/* Defaults: no allocator, precision -1, TCI_SVD_PLAIN, no cache, verbosity -1. */
void tci_context_opts_default(tci_context_opts* opts);

/* Create a context on HIP device `device_id` whose work is ordered on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  The
 * stream is borrowed.  opts may be NULL (the defaults above).  The
 * environment variable TCI_VERBOSE (0, 1, 2; Spec, environment variables)
 * selects per-call logging to stderr unless opts->verbosity >= 0; level 2
 * adds wall time and synchronises after each call.
 * Errors: TCI_ERR_INVALID_ARGUMENT (out NULL, only one of alloc / free set,
 * bad precision, svd mode or verbosity), TCI_ERR_DEVICE. */
tci_status tci_create_context(tci_context* out, int device_id, void* hip_stream, const tci_context_opts* opts);

/* Release the context, its workspace and every cached resource.  Tensors
 * must be destroyed before their context. */
tci_status tci_destroy_context(tci_context ctx);

/* Change the stream used by later calls (borrowed). */
tci_status tci_set_stream(tci_context ctx, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Tensor life (Spec, construction and destruction: allocate, zeros,    */
/* copy, move, clear)                                                   */
/* ------------------------------------------------------------------ */

/* New owning tensor of the given shape, contents uninitialised.
 * order in [0, 8]; shape[i] >= 0 (order 0 is a scalar with one element).
 * Errors: TCI_ERR_INVALID_ARGUMENT, TCI_ERR_DTYPE, TCI_ERR_OUT_OF_MEMORY. */
tci_status tci_allocate(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape,
                        tci_tensor* out);

/* As tci_allocate, zero-filled. */
tci_status tci_zeros(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape,
                     tci_tensor* out);

/* Borrowing tensor over caller-owned device memory `dev_ptr`, which must
 * hold prod(shape) elements of `dtype` and outlive the handle. */
tci_status tci_wrap(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape,
                    void* dev_ptr, tci_tensor* out);

/* Spec, construction: fill.  New owning tensor of the given shape with every
 * element equal to *value (one host scalar of `dtype`).  Asynchronous on the
 * context stream.  Errors as tci_allocate; TCI_ERR_INVALID_ARGUMENT for a
 * NULL value. */
tci_status tci_fill(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape, const void* value,
                    tci_tensor* out);

/* Spec, construction: eye.  New owning n x n tensor (order 2) with ones on
 * the main diagonal and zeros elsewhere.  Errors: TCI_ERR_INVALID_ARGUMENT
 * (n < 0), TCI_ERR_DTYPE, TCI_ERR_OUT_OF_MEMORY. */
tci_status tci_eye(tci_context ctx, tci_dtype dtype, int64_t n, tci_tensor* out);

/* Deep copy into a new owning tensor. */
tci_status tci_copy(tci_context ctx, tci_tensor in, tci_tensor* out);

/* Transfer contents and ownership of *from into a new handle *out; *from
 * becomes an empty (order 0, no storage) handle that must still be
 * destroyed. */
tci_status tci_move(tci_context ctx, tci_tensor* from, tci_tensor* out);

/* Release a tensor handle (and its storage if owning).  NULL is allowed. */
tci_status tci_destroy(tci_context ctx, tci_tensor t);

/* ------------------------------------------------------------------ */
/* Read-only queries (Spec, read-only queries: order, shape, size,      */
/* size_bytes, get_elem)                                                */
/* ------------------------------------------------------------------ */
tci_status tci_order(tci_context ctx, tci_tensor t, int* out);
/* Writes min(order, cap) dimensions. */
tci_status tci_shape(tci_context ctx, tci_tensor t, int64_t* shape_out, int cap);
tci_status tci_size(tci_context ctx, tci_tensor t, int64_t* out);
/* Bytes of the elements, e.g. 96 for a {3,4,2} F32 tensor (Spec, size_bytes example). */
tci_status tci_size_bytes(tci_context ctx, tci_tensor t, int64_t* out);
tci_status tci_dtype_of(tci_context ctx, tci_tensor t, tci_dtype* out);
/* Device address of element 0 (NULL for an empty handle). */
tci_status tci_data_ptr(tci_context ctx, tci_tensor t, void** out);

/* One element at coordinates `coors` (order entries) copied to host `out`
 * (elem_bytes of dtype).  Synchronous.  Errors: TCI_ERR_SHAPE (out of range). */
tci_status tci_get_elem(tci_context ctx, tci_tensor t, const int64_t* coors, void* out);
/* Spec, manipulation: set_elem.  Synchronous. */
tci_status tci_set_elem(tci_context ctx, tci_tensor t, const int64_t* coors, const void* val);

/* Bond labels (optional metadata used by tci_contract_labeled). */
tci_status tci_set_labels(tci_context ctx, tci_tensor t, const int32_t* labels, int n);
tci_status tci_get_labels(tci_context ctx, tci_tensor t, int32_t* labels, int cap);

/* ------------------------------------------------------------------ */
/* Host I/O (Spec: assign_from_range / to_range with the row-major      */
/* coordinate map; convert)                                             */
/* ------------------------------------------------------------------ */

/* Copy `bytes` (must equal size_bytes) from host memory, row-major. */
tci_status tci_from_host(tci_context ctx, tci_tensor t, const void* host, size_t bytes);
/* Copy the tensor to host memory (row-major), synchronous. */
tci_status tci_to_host(tci_context ctx, tci_tensor t, void* host, size_t bytes);
/* Spec, miscellaneous: convert.  New owning tensor `out` with element type
 * `dtype` (C128 <-> C64, F64 <-> F32, real -> complex). */
tci_status tci_convert(tci_context ctx, tci_tensor in, tci_dtype dtype, tci_tensor* out);

/* Spec, construction: save / load.  Back-end file format: 8 bytes
 * "TCIMI355", int32 format version (1), int32 dtype, int32 order, int32 0,
 * int64 shape[order], then the elements row-major in the host's
 * little-endian byte order.  save copies the tensor to the host
 * (synchronous); load returns a new owning tensor.  Errors:
 * TCI_ERR_INVALID_ARGUMENT (file cannot be opened, written, or is not such
 * a file, or is truncated). */
tci_status tci_save(tci_context ctx, tci_tensor t, const char* path);
tci_status tci_load(tci_context ctx, const char* path, tci_tensor* out);

/* Spec, miscellaneous: show.  Print dtype, shape and every element with
 * its coordinates to standard output (synchronous). */
tci_status tci_show(tci_context ctx, tci_tensor t);

/* ------------------------------------------------------------------ */
/* Manipulation (Spec, manipulation: reshape, transpose, cplx_conj,      */
/* scale; linear algebra: linear_combine)                               */
/* ------------------------------------------------------------------ */

/* Metadata only; memory order kept.  out == in reshapes in place,
 * otherwise `out` receives a copy.  Errors: TCI_ERR_SHAPE (size differs). */
tci_status tci_reshape(tci_context ctx, tci_tensor in, int order, const int64_t* shape,
                       tci_tensor out);

/* Sec. II.B transpose: out.shape[b] = in.shape[perm[b]],
 * out[c] = in[c'] with c'[perm[b]] = c[b] (numpy transpose).  out == in
 * is allowed (a temporary is used). */
tci_status tci_transpose(tci_context ctx, tci_tensor in, const int32_t* perm, tci_tensor out);

/* Spec, manipulation: diag.  A first-order input of length n gives the
 * n x n matrix with it on the main diagonal and zeros elsewhere; a
 * second-order input gives its main diagonal (length min(d0, d1)).  `out`
 * may be `in`.  Errors: TCI_ERR_SHAPE (order not 1 or 2). */
tci_status tci_diag(tci_context ctx, tci_tensor in, tci_tensor out);

/* Spec, manipulation: to_cplx, real, imag.  `out` (an existing handle; may
 * be `in`) receives, elementwise: to_cplx the complex embedding (F32 -> C64,
 * F64 -> C128, a copy for complex types); real the real part (F32/F64; a
 * copy for real types); imag the imaginary part (zeros for real types). */
tci_status tci_to_cplx(tci_context ctx, tci_tensor in, tci_tensor out);
tci_status tci_real(tci_context ctx, tci_tensor in, tci_tensor out);
tci_status tci_imag(tci_context ctx, tci_tensor in, tci_tensor out);

/* Elementwise complex conjugate (identity copy for real types). */
tci_status tci_cplx_conj(tci_context ctx, tci_tensor in, tci_tensor out);

/* inout *= s.  `s` points to one host scalar of the tensor's dtype. */
tci_status tci_scale(tci_context ctx, tci_tensor inout, const void* s);

/* out = sum_i coefs[i] * ins[i] (coefs: n host scalars of the dtype, NULL =
 * all ones).  All inputs same shape and dtype; out may alias one input. */
tci_status tci_linear_combine(tci_context ctx, int n, const tci_tensor* ins, const void* coefs,
                              tci_tensor out);

/* Sub-tensors (Spec, manipulation: extract_sub, shrink, expand,
 * replace_sub, concatenate, stack).  All are asynchronous on the context
 * stream; `out` is an existing handle whose shape and dtype are set by the
 * call (an owning handle is resized, a borrowed one must have room).
 * Coordinates are element coordinates, bond 0 slowest (row-major). */

/* out = in[first[0]:last[0], ..., first[r-1]:last[r-1]] (half-open ranges,
 * one per bond, 0 <= first <= last <= dim).  out == in works in place.
 * Errors: TCI_ERR_INVALID_ARGUMENT (range outside a bond, NULL). */
tci_status tci_extract_sub(tci_context ctx, tci_tensor in, const int64_t* first, const int64_t* last,
                           tci_tensor out);

/* As tci_extract_sub for the n listed bonds bonds[i] (each at most once),
 * cut to [first[i], last[i]); unlisted bonds keep their full range. */
tci_status tci_shrink(tci_context ctx, tci_tensor in, int n, const int32_t* bonds, const int64_t* first,
                      const int64_t* last, tci_tensor out);

/* Bond bonds[i] grows by increments[i] >= 0 (appended at the end); elements
 * inside the old bounds keep their values, every other element is zero.
 * out == in works in place (owning handles). */
tci_status tci_expand(tci_context ctx, tci_tensor in, int n, const int32_t* bonds, const int64_t* increments,
                      tci_tensor out);

/* out = in with the box of `sub` (same order and dtype) written so that its
 * origin lands at coordinate begin[].  out == in works in place; out must
 * not alias sub otherwise.  Errors: TCI_ERR_SHAPE (order/dtype),
 * TCI_ERR_INVALID_ARGUMENT (sub does not fit at begin). */
tci_status tci_replace_sub(tci_context ctx, tci_tensor in, tci_tensor sub, const int64_t* begin,
                           tci_tensor out);

/* The n >= 1 inputs (same order and dtype, equal dimensions on every bond
 * but `bond`) follow one another along `bond`; the output dimension there is
 * the sum of the input dimensions.  out must not alias an input. */
tci_status tci_concatenate(tci_context ctx, int n, const tci_tensor* ins, int bond, tci_tensor out);

/* The n >= 1 inputs (identical shapes) along a new bond of dimension n
 * inserted at position `bond` (0 <= bond <= order): out[.., k, ..] = ins[k].
 * out must not alias an input.  Errors: TCI_ERR_UNSUPPORTED when the result
 * order exceeds the maximum. */
tci_status tci_stack(tci_context ctx, int n, const tci_tensor* ins, int bond, tci_tensor out);

/* Spec, linear algebra: trace.  Partial trace over npairs bond pairs
 * (pairs[2p], pairs[2p+1]; equal dimensions, every bond in at most one
 * pair): out[kept] = sum_t in[kept, t, t]; the kept bonds keep their order;
 * all bonds paired gives order 0.  FP64 accumulation.  out == in works in
 * place.  Errors: TCI_ERR_INVALID_ARGUMENT, TCI_ERR_SHAPE. */
tci_status tci_trace(tci_context ctx, tci_tensor in, int npairs, const int32_t* pairs, tci_tensor out);

/* Spec, linear algebra: exp.  Matricise with the first k_rows bonds as rows
 * (rows must equal columns), take the matrix exponential, fold back to the
 * input shape.  Scaling and squaring in FP64 for every dtype (F32/C64 are
 * promoted and the result rounded back): A / 2^s with ||A / 2^s||_F <= 1/2,
 * Taylor polynomial of degree 18 by Horner's rule, s squarings, the
 * products as FP64 GEMMs on the matrix cores.  out == in works in place.
 * Synchronous.  Errors:
 * TCI_ERR_SHAPE (not square), TCI_ERR_NUMERIC (non-finite input). */
tci_status tci_exp(tci_context ctx, tci_tensor in, int k_rows, tci_tensor out);

/* ------------------------------------------------------------------ */
/* Reductions (Spec, linear algebra: norm, normalize)                   */
/* ------------------------------------------------------------------ */

/* Frobenius norm (square root of the sum of squared moduli, FP64
 * accumulation).  Synchronous. */
tci_status tci_norm(tci_context ctx, tci_tensor t, double* out);
/* Scale to unit Frobenius norm in place; *old_norm receives the norm
 * before scaling (may be NULL).  A zero tensor is left unchanged. */
tci_status tci_normalize(tci_context ctx, tci_tensor inout, double* old_norm);

/* ------------------------------------------------------------------ */
/* Contraction (Sec. II.B contraction equations; Spec, linear algebra:   */
/* contract)                                                            */
/* ------------------------------------------------------------------ */

/* Labels shared by a (la, na entries) and b (lb, nb) and absent from c (lc,
 * nc) are summed; lc fixes the bonds of c and their order; nc == 0 gives a
 * scalar (order 0).  c may alias a and/or b.  A label repeated inside one
 * list, a label of c found in neither or both operands, and a label found
 * in one operand only but not in c give TCI_ERR_LABEL; dimensions of equal
 * labels must agree (TCI_ERR_SHAPE); a and b must have the same dtype.
 * Runs as transpose + one GEMM on the matrix cores in the context's
 * precision for that dtype (tci_set_precision). */
tci_status tci_contract(tci_context ctx, tci_tensor a, const int32_t* la, int na, tci_tensor b,
                        const int32_t* lb, int nb, tci_tensor c, const int32_t* lc, int nc);

/* String form: every character is one label ("ijk"). */
tci_status tci_contract_str(tci_context ctx, tci_tensor a, const char* la, tci_tensor b,
                            const char* lb, tci_tensor c, const char* lc);

/* Precision used by contractions on F32/C64 tensors (default TCI_PREC_FP32). */
tci_status tci_set_precision(tci_context ctx, tci_precision prec);

/* ------------------------------------------------------------------ */
/* Decompositions (Spec, linear algebra: svd, trunc_svd, qr, eigh)      */
/* ------------------------------------------------------------------ */

/* Matricise `a` with its first k_rows bonds as rows (1 <= k_rows < order)
 * and compute a thin SVD: u {d_0..d_{k-1}, kappa}, s {kappa} (real, FP64 for
 * double types, non-increasing, >= 0), vdag {kappa, d_k..}.  Gauge: each
 * column of u has its largest-modulus entry (first on ties) real positive.
 * Implemented as trunc_svd keeping every value.  Synchronous. */
tci_status tci_svd(tci_context ctx, tci_tensor a, int k_rows, tci_tensor u, tci_tensor s,
                   tci_tensor vdag);

/* Spec, trunc_svd form (2): discard s_i < s_min; keep at least chi_min (or
 * all that survive when fewer); grow chi until the relative truncation
 * error eps = sum_{i>=chi} s_i^2 / sum_i s_i^2 <= target_trunc_err or chi
 * = chi_max.  chi >= 1.  Form (1) is chi_min = 1, target 0.  The kept s is
 * NOT renormalised.  *trunc_err (may be NULL) receives eps.
 * Errors: TCI_ERR_INVALID_ARGUMENT (k_rows, chi_min < 1, chi_min > chi_max). */
tci_status tci_trunc_svd(tci_context ctx, tci_tensor a, int k_rows, tci_tensor u, tci_tensor s,
                         tci_tensor vdag, double* trunc_err, int64_t chi_min, int64_t chi_max,
                         double target_trunc_err, double s_min);

/* Spec, qr: thin QR of the matricised tensor, q {d_0..d_{k-1}, rho},
 * r {rho, d_k..}, rho = min(I, J); r upper triangular with a real positive
 * diagonal.  Cholesky-QR2 in FP64; a rank-deficient column gives a zero
 * column of q and a zero row of r.  Synchronous. */
tci_status tci_qr(tci_context ctx, tci_tensor a, int k_rows, tci_tensor q, tci_tensor r);

/* Spec, linear algebra: inverse.  Matricise with the first k_rows bonds as
 * rows (rows must equal columns, at most 65536), invert, fold back to the
 * input shape.  Gauss-Jordan elimination with partial pivoting on [A | I]
 * in FP64 for every dtype (single types promoted, the result rounded back).
 * out == in works in place.  Synchronous.  Errors: TCI_ERR_SHAPE (not
 * square), TCI_ERR_NUMERIC (an exactly zero pivot column, i.e. singular, or
 * non-finite entries), TCI_ERR_UNSUPPORTED (too large). */
tci_status tci_inverse(tci_context ctx, tci_tensor in, int k_rows, tci_tensor out);

/* Spec, lq: thin LQ of the matricised tensor, l {d_0..d_{k-1}, rho},
 * q {rho, d_k..}, rho = min(I, J); l lower triangular with a real
 * non-negative diagonal, q with orthonormal rows.  Computed as the
 * Cholesky-QR2 of the conjugate transpose.  Wide or square matrices only
 * (I <= J; TCI_ERR_UNSUPPORTED otherwise).  Synchronous. */
tci_status tci_lq(tci_context ctx, tci_tensor a, int k_rows, tci_tensor l, tci_tensor q);

/* Spec, eigh: the tensor matricised with its first k_rows bonds as rows
 * (1 <= k_rows < order; I = prod d_0..d_{k-1} must equal J = prod d_k..) is
 * read as a Hermitian matrix (as given, no symmetrisation)
 * -> w (I eigenvalues ascending, real: F64 for F64/C128, F32 for F32/C64)
 * and v {d_0, .., d_{k-1}, I} in a's dtype whose last bond indexes the
 * eigenvectors (gauge as in tci_svd).  Single-precision inputs are solved in
 * FP64 and rounded.  FP64 Householder tridiagonalisation, bisection, inverse
 * iteration and back-transformation on the GPU.  Synchronous.
 * Errors: TCI_ERR_INVALID_ARGUMENT (k_rows), TCI_ERR_SHAPE (I != J). */
tci_status tci_eigh(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v);

/* Spec, eigvalsh: the eigenvalues of tci_eigh only (no vectors are formed). */
tci_status tci_eigvalsh(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w);

/* Spec, eig: right eigendecomposition A'V = V diag(w) of the matricised
 * tensor (first k_rows bonds as rows; I == J required, I <= 1024).
 * - w: first-order complex tensor of I eigenvalues, sorted by ascending real
 *   part, then ascending imaginary part, compared as returned (after
 *   rounding to C64 for single-precision input); the paper fixes no order.
 * - v: shape {d_0, ..., d_{k-1}, I}; column k (the last bond) is the right
 *   eigenvector of w[k], scaled to unit 2-norm with its largest-modulus
 *   entry (the first on exact ties) real and positive.
 * - w and v are C128 for F64 / C128 input and C64 for F32 / C64 input; the
 *   arithmetic is complex128 throughout: Householder reduction to Hessenberg
 *   form, single-shift QR iteration (Wilkinson shifts) to the complex Schur
 *   form, back substitution for the eigenvectors of the triangular factor.
 *   The Hessenberg and QR steps run in one workgroup per matrix.
 * - Synchronous.  Errors: TCI_ERR_INVALID_ARGUMENT (k_rows), TCI_ERR_SHAPE
 *   (I != J), TCI_ERR_UNSUPPORTED (I > 1024), TCI_ERR_NOT_CONVERGED (more
 *   than 60 QR sweeps for one eigenvalue), TCI_ERR_NUMERIC (non-finite input). */
tci_status tci_eig(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v);

/* Spec, eigvals: the eigenvalues of tci_eig only (no vectors are formed). */
tci_status tci_eigvals(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w);

/* Spec, close: *result = 1 iff max |a - b| <= eps elementwise (same shape
 * and dtype), else 0.  Synchronous. */
tci_status tci_close(tci_context ctx, tci_tensor a, tci_tensor b, double eps, int* result);

/* ------------------------------------------------------------------ */
/* Two-site update composites (the hot path of the paper's applications, */
/* Application A listing: theta = contract(A, B), gate, trunc_svd,       */
/* normalize)                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t chi_min;          /* trunc_svd form (2) parameters */
  int64_t chi_max;
  double target_trunc_err;
  double s_min;
  int32_t direction;        /* tci_direction */
  int32_t precision;        /* tci_precision of the contractions */
  int32_t svd_mode;         /* tci_svd_mode */
  int32_t sketch_rank;      /* TCI_SVD_RANDOMIZED: sketch columns k (0: chi_max + 64) */
  int32_t power_iters;      /* randomized: power iterations q (default 2 when < 0) */
  int32_t max_batch;        /* problems per internal launch (0: all) */
  uint64_t seed;            /* Philox key of the sketch */
  double cert_tol;          /* randomized acceptance: max residual <= cert_tol * s_1 (0: 1e-7) */
  void* sketch_model;       /* tci_sketch_model for TCI_SVD_LEARNED */
  const tci_tensor* prev_spectra; /* TCI_SVD_LEARNED: per update, the bond's spectrum before the
                                     update (F64 vector, descending); indexed like A / theta */
  const tci_tensor* lambda_left;  /* TCI_DIR_VIDAL: per update, the outer bond weights on the left
                                     (F64 vector of chi_l entries, all > 0); indexed like A */
  const tci_tensor* lambda_right; /* TCI_DIR_VIDAL: the same on the right (chi_r entries) */
} tci_update_params;

typedef struct {
  int64_t chi;              /* kept bond dimension */
  double trunc_err;         /* relative truncation error eps */
  double discarded_abs;     /* sum of the squares of the cut values (eps * ||theta||_F^2) */
  double norm2;             /* ||theta||_F^2 after the gate */
  int32_t used_fallback;    /* randomized/learned: 1 if the plain SVD decided */
  int32_t sketch_rank;      /* sketch columns used (0 for plain) */
  double max_residual;      /* randomized: max ||theta v_i - s_i u_i|| / s_1 of the kept i */
} tci_update_info;

/* Fill `p` with defaults: chi_min 1, chi_max INT64_MAX, target 0, s_min 0,
 * RIGHT, FP64, PLAIN, sketch 0, q 2, max_batch 0, seed 0, cert 1e-7, no
 * model, spectra or Vidal weights. */
void tci_update_params_default(tci_update_params* p);

/* n independent two-site updates.  A[i] has shape (chi_l, d, chi_m), B[i]
 * (chi_m, d, chi_r), all i the same shapes and dtype (C128/F64 for FP64,
 * C64/F32 for the mixed precisions).  gates (nullable; entries nullable)
 * are (d*d, d*d) or (d, d, d, d) with rows = outgoing (s1', s2'):
 * theta'(a,s1',s2',b) = sum G[(s1' s2'),(s1 s2)] theta(a,s1,s2,b).
 * Then trunc_svd of theta' with k_rows = 2 under params, s renormalised
 * to unit 2-norm, and the write-back chosen by params->direction:
 * A_out[i] (chi_l, d, chi_i), s_out[i] (chi_i) real FP64, B_out[i]
 * (chi_i, d, chi_r).  infos (nullable) receives per-update results.
 * Supports d = 2.  Synchronous. */
tci_status tci_two_site_update_batched(tci_context ctx, int n, const tci_tensor* A,
                                       const tci_tensor* B, const tci_tensor* gates,
                                       const tci_update_params* params, tci_tensor* A_out,
                                       tci_tensor* s_out, tci_tensor* B_out,
                                       tci_update_info* infos);

/* One two-site update (the Application A listing: theta = contract(A, B),
 * gate, trunc_svd, normalize, then the write-back of params->direction):
 * tci_two_site_update_batched with n = 1.  gate and info are nullable;
 * params NULL means tci_update_params_default with the context's svd mode
 * and precision (FP64 for F64/C128 tensors).  Synchronous. */
tci_status tci_two_site_update(tci_context ctx, tci_tensor A, tci_tensor B, tci_tensor gate,
                               const tci_update_params* params, tci_tensor A_out, tci_tensor s_out,
                               tci_tensor B_out, tci_update_info* info);

/* The second half of the update for given two-site tensors: theta[i] of
 * shape (chi_l, d, d, chi_r) (all i the same shape and dtype) is split by
 * trunc_svd with k_rows = 2 under params (plain SVD), s renormalised and
 * written back as in tci_two_site_update_batched.  Used after the Lanczos
 * step of a DMRG update.  Synchronous. */
tci_status tci_split_batched(tci_context ctx, int n, const tci_tensor* theta,
                             const tci_update_params* params, tci_tensor* A_out,
                             tci_tensor* s_out, tci_tensor* B_out, tci_update_info* infos);

/* Effective-Hamiltonian matvec of the two-site DMRG update:
 * y[a,s1,s2,b] = sum L[a,w,a'] W1[w,w',s1,s1'] W2[w',w'',s2,s2'] R[b,w'',b']
 *                    x[a',s1',s2',b'].
 * L (chi_l, w, chi_l), W1 (w, w, d, d), W2 (w, w, d, d), R (chi_r, w, chi_r),
 * x, y (chi_l, d, d, chi_r); all one dtype.  y must not alias x. */
tci_status tci_heff_matvec(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2,
                           tci_tensor R, tci_tensor x, tci_tensor y);

/* tci_heff_matvec for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same operation, operands, precision and kernels as tci_heff_matvec, but
 * its workspace (the MPO pair W12, the intermediates X1 and X2 and, in the
 * split-BF16x3 precision, the operand planes) lives in a fixed device array
 * of 64 MiB per device, held from library load until the process ends; the
 * call itself makes no device allocation and no free.
 * - y must already own or wrap storage for chi_l*d*d*chi_r elements of the
 *   operands' dtype (TCI_ERR_INVALID_ARGUMENT / TCI_ERR_DTYPE otherwise); its
 *   shape is set to (chi_l, d, d, chi_r).
 * - Shapes whose workspace exceeds 64 MiB are rejected with
 *   TCI_ERR_INVALID_ARGUMENT before any work is queued (for w = 5, d = 2
 *   and chi_l = chi_r = chi: complex64 in split-BF16x3 and complex128 both
 *   fit up to chi = 320).
 * - Every call on one device shares that device's array and leaves its
 *   contents behind; whatever must start at zero is cleared by a kernel on
 *   the context stream.  Calls on the same stream are ordered; calls that
 *   overlap on one device (other streams, other contexts, other threads)
 *   race on the array and give undefined results.
 * - Stream-ordered on the context stream; does not synchronise. */
tci_status tci_heff_matvec_noalloc(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2,
                                   tci_tensor R, tci_tensor x, tci_tensor y);

/* Lowest Ritz pair after at most n_matvec matvecs of Lanczos with full
 * re-orthogonalisation (FP64 scalars and vector arithmetic): after the
 * three-term recurrence, one classical Gram-Schmidt pass against the whole
 * basis, and a second pass when the first removed more than half of the
 * residual's norm.  Started at theta_inout, which receives the normalised
 * Ritz vector (phase: <theta_in, psi> real positive).  *energy receives the
 * Ritz value.  For F32/C64 operands the matvecs run in the context's mixed
 * precision.  The Krylov vectors are stored in FP64 (complex128), except for
 * C64 operands, where they are stored in complex64 (the operand precision of
 * their matvec) and combined in FP64.  The Krylov scalars, the second-pass
 * decision and the breakdown test (beta <= 1e-13 max|T|, after which the
 * remaining steps do no work) stay on the device; the call waits for the
 * device once, at its end, to return the energy.  TCI_ERR_NUMERIC when
 * theta_inout has a zero or non-finite norm or the Ritz vector is not finite;
 * theta_inout is then left unchanged.  At verbosity >= 1 the call's log line
 * gives the order of T (krylov=), the number of second Gram-Schmidt passes
 * (reorth=) and its host synchronisations (host_syncs=).  Synchronous. */
tci_status tci_lanczos_ground(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2,
                              tci_tensor R, tci_tensor theta_inout, int n_matvec, double* energy);

/* ------------------------------------------------------------------ */
/* U(1) block-sparse two-site update                                    */
/* ------------------------------------------------------------------ */
/* A site tensor of an MPS with a conserved U(1) charge (2 S^z for spin 1/2),
 * the symmetric-tensor form that the paper names as the extension of its
 * dense interface (Sec. V, future work).  Its left and right bonds are lists
 * of sectors (charge q, dimension D); the physical index has d = 2 with
 * charges +1 (index 0) and -1 (index 1).  Block (a, s, b) is non-zero only
 * when q_right[b] = q_left[a] + charge(s); each allowed block is a
 * D_left[a] x D_right[b] row-major matrix, and the blocks are stored back to
 * back in one device buffer in the order of (a, s) ascending.  The handle
 * owns the buffer. */
typedef struct tci_bs_tensor_s* tci_bs_tensor;

/* Create a block-sparse site tensor (F32 or F64; storage uninitialised).
 * Charges within a bond must be distinct; dimensions >= 0.  n_left = n_right
 * = 0 gives an empty placeholder for an output argument. */
tci_status tci_bs_create(tci_context ctx, tci_dtype dtype, int n_left, const int32_t* q_left,
                         const int64_t* d_left, int n_right, const int32_t* q_right,
                         const int64_t* d_right, tci_bs_tensor* out);
tci_status tci_bs_destroy(tci_context ctx, tci_bs_tensor t);
/* Sector counts of the two bonds and the number of stored blocks. */
tci_status tci_bs_dims(tci_context ctx, tci_bs_tensor t, int* n_left, int* n_right, int* n_blocks,
                       int64_t* n_elems);
/* Charges and dimensions of the bonds (arrays of n_left / n_right entries). */
tci_status tci_bs_bonds(tci_context ctx, tci_bs_tensor t, int32_t* q_left, int64_t* d_left,
                        int32_t* q_right, int64_t* d_right);
/* Block i: sector indices (a, s, b) and its element offset in the buffer. */
tci_status tci_bs_block_info(tci_context ctx, tci_bs_tensor t, int i, int* a, int* s, int* b,
                             int64_t* offset);
/* Whole-buffer host copies (bytes = n_elems * element size); synchronous. */
tci_status tci_bs_from_host(tci_context ctx, tci_bs_tensor t, const void* host, size_t bytes);
tci_status tci_bs_to_host(tci_context ctx, tci_bs_tensor t, void* host, size_t bytes);

/* n independent U(1) two-site updates (the block form of
 * tci_two_site_update_batched; Sec. II.B contraction and decomposition
 * equations applied sector by sector).  For update i, A[i]'s right bond must
 * equal B[i]'s left bond.  gates[i] (nullable array or entries) is a 4 x 4
 * (or 2,2,2,2) charge-conserving gate with rows = outgoing pair, in any real
 * dtype; off-sector entries are ignored.  Per update:
 *   theta'(a, s1', s2', b) = sum G[(s1' s2'), (s1 s2)] A[a, s1, m] B[m, s2, b]
 * built directly into the sector matrices of the new bond (sector Q: rows
 * (a, s1') with q_a + charge(s1') = Q, columns (s2', b)) by grouped FP32
 * GEMMs in one launch per accumulation phase for all updates; each sector is
 * split by the plain FP64 truncated SVD (Gram, tridiagonal eigensolve); the
 * singular values of all sectors of the update are merged in descending
 * order (ties: sector charge ascending, then in-sector index) and cut once by
 * the trunc_svd rule under params (chi_min, chi_max, target, s_min) with the
 * total weight ||theta'||_F^2; s is renormalised over the kept set.
 * Outputs: A_out[i] (bonds: A's left, new bond), B_out[i] (new bond, B's
 * right) re-created by the library in the input dtype, written as in
 * params.direction; the new bond holds the sectors with a kept value, in
 * ascending charge.  s_out[i]: F64 vector of the kept values in bond order
 * (sector by sector, descending within a sector).  chi_max_each (nullable):
 * per-update caps that replace params->chi_max.  infos (nullable) as for
 * the dense update.  The tile shape of the grouped GEMM is autotuned per
 * problem-size signature on first use.  The first half of the update
 * (products, padding, Gram matrices, eigenvalue stage) is recorded as a HIP
 * graph the second time a problem structure is seen and replayed from then
 * on (not while tci_profile_enable is on, nor with TCI_NO_GRAPHS set).
 * Synchronous. */
tci_status tci_bs_two_site_update_batched(tci_context ctx, int n, const tci_bs_tensor* A,
                                          const tci_bs_tensor* B, const tci_tensor* gates,
                                          const tci_update_params* params, const int64_t* chi_max_each,
                                          tci_bs_tensor* A_out, tci_tensor* s_out, tci_bs_tensor* B_out,
                                          tci_update_info* infos);

/* ------------------------------------------------------------------ */
/* Sketch-rank model for TCI_SVD_LEARNED                                */
/* ------------------------------------------------------------------ */
/* A perceptron 35 -> 128 -> 128 -> 1 with exact GELU that predicts
 * y = log2 chi*(eps) of a bond from its features
 *   [log2(chi_max)/11, d/4, -log10(eps)/16, 32 clamped log10 quantiles
 *    q_t = clamp(log10(s_j/s_0)/16, -1, 0), j = floor((t+1/2)/32 (len-1))]
 * of the bond's previous spectrum s.  The update uses the sketch rank
 * k = 32 ceil((1.5 * 2^y + 32)/32) and the plain truncated SVD when
 * y > log2(chi_max) or k > min(m, n) / 4 (the range finder's FP64
 * orthonormalisations cost O(n k^2): at k = n / 3 a sketch of a 2048 x 2048
 * complex bond costs about as much as the plain SVD).  Parameters are FP32, flat: W1 (128x35), b1, W2
 * (128x128), b2, W3 (1x128), b3.  All data pointers below are device
 * pointers unless marked host. */

/* New model with He-uniform weights from Philox4x32-10 (key seed, stream 7),
 * zero biases and zero Adam state. */
tci_status tci_sketch_model_create(tci_context ctx, uint64_t seed, tci_sketch_model* out);
tci_status tci_sketch_model_destroy(tci_context ctx, tci_sketch_model m);
/* Number of parameters (21249). */
int64_t tci_sketch_model_nparams(void);
/* Copy the flat parameters to / from host memory (n must equal nparams). */
tci_status tci_sketch_model_get_params(tci_context ctx, tci_sketch_model m, float* host, int64_t n);
tci_status tci_sketch_model_set_params(tci_context ctx, tci_sketch_model m, const float* host, int64_t n);
/* Raw binary file: "TCISKM1\0", int32 count, count float32 parameters. */
tci_status tci_sketch_model_save(tci_context ctx, tci_sketch_model m, const char* path);
tci_status tci_sketch_model_load(tci_context ctx, const char* path, tci_sketch_model* out);
/* y[i] = model(X[i, 0:35]) for i < n (X row-major n x 35).  Asynchronous. */
tci_status tci_sketch_predict(tci_context ctx, tci_sketch_model m, const float* X, int n, float* y);
/* Gradient of the mean pinball loss (tau = 0.9, targets T) w.r.t. the flat
 * parameters into grad (device, nparams); *loss (host, may be NULL). */
tci_status tci_sketch_grads(tci_context ctx, tci_sketch_model m, const float* X, const float* T, int n,
                            float* grad, float* loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on a batch. */
tci_status tci_sketch_train_step(tci_context ctx, tci_sketch_model m, const float* X, const float* T,
                                 int n, float lr, float* loss);
/* Features of n bonds: spectra s (row i at s + i*ss, length len[i]). */
tci_status tci_sketch_features(tci_context ctx, const double* s, int64_t ss, const int32_t* len, int n,
                               int chi_max, int d, double eps, float* X);

/* Raw Philox4x32-10 blocks (key seed, counter (first + i, stream, 0)) into
 * out[4i .. 4i+3] (device), for checking the generator against published
 * vectors. */
tci_status tci_philox_blocks(tci_context ctx, uint64_t seed, uint32_t stream, uint64_t first, int64_t n,
                             uint32_t* out);

/* ------------------------------------------------------------------ */
/* Kernel timing (instrumentation; not part of the paper's API)         */
/* ------------------------------------------------------------------ */

/* Start (enable != 0) or stop recording a HIP event pair around every
 * matrix-core GEMM and tridiagonal matrix-vector launch, on the stream the
 * kernel runs on.  Either call clears the records.  Process-wide. */
tci_status tci_profile_enable(tci_context ctx, int enable);

/* Sum over the recorded launches with tag `tag` ("<call site>:<class>",
 * e.g. "heff_L:c64_bf16x3", "gemm:c128_fp64", "gemm:hemv"): number of
 * launches, total event time in ms and total algorithmic work (flops for
 * GEMMs, bytes for the matrix-vector product).  Synchronises the stream. */
tci_status tci_profile_query(tci_context ctx, const char* tag, int64_t* count, double* total_ms,
                             double* work);

/* Distinct recorded tags separated by newlines, NUL-terminated in buf. */
tci_status tci_profile_tags(tci_context ctx, char* buf, int cap);

#ifdef __cplusplus
}
#endif

#endif /* TCI_C_H */
