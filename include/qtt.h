/*
 * qtt.h -- C ABI of libqtt, the MI355X (gfx950) quantics-MPS Fresnel path.
 *
 * What the library computes (paper: "Tensor network methods for
 * quantum-inspired image processing and classical optics"):
 *   - tt_encode:    a 2^n x 2^n image/field -> quantics MPS (bit-interleaved
 *                   coordinates, Sec. 3) by sequential SVD (Sec. 4, App. A);
 *   - mpo_apply:    MPO x MPS (Sec. 5; the Fresnel propagator of Sec. 6.1 is
 *                   one MPO per axis) by zip-up, then an SVD truncation sweep;
 *   - tt_truncate:  recompression of an MPS (QR sweep + SVD sweep);
 *   - tt_to_dense:  decompression back to the N x N grid (Sec. 3, Fig. 6);
 *   - mpo_apply_backward: adjoint of mpo_apply for gradient-based inverse
 *                   problems (phase retrieval, listed as future work in Sec. 7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sites.  An N x N grid, N = 2^n, has m = 2n sites of dimension 2.  Site
 *   2p-1 (1-based) is bit p of the row index a, site 2p bit p of the column
 *   index b, most significant bit first (reading of Sec. 3).
 * MPS storage (qtt_mps).  Device memory, caller-owned.  Core k (0-based) sits
 *   at element offset k * chi_cap * 2 * chi_cap and is laid out
 *   [r_k][s][r_(k+1)] row-major with row stride 2*chi_cap and physical stride
 *   chi_cap (capacity layout: entries outside the actual bonds are ignored
 *   and may hold anything).  The actual bond dimensions live on the DEVICE in
 *   bonds[0..m] (bonds[0] = bonds[m] = 1) and are written by the library, so
 *   no call ever synchronises with the host.  Element type is complex64
 *   (QTT_C64, interleaved re/im floats) or complex128 (QTT_C128).
 * MPO storage (qtt_mpo).  Device cores [D_k][t][s][D_(k+1)] row-major with
 *   actual bonds (host array d_bonds[0..m]) -- operator bonds are static --
 *   core k at element offset k * d_cap * 4 * d_cap; t is the output bit and s
 *   the input bit.  site_kind[k] = 1 marks an identity site whose bond is
 *   passed through (D_k == D_(k+1), core not read); site_kind[k] = 2 a
 *   diagonal site (W[.][t][s][.] = 0 for t != s: an operator diagonal in the
 *   computational basis there, such as the transfer function between the two
 *   Fourier transforms of Sec. 6.1 or an element-wise product, Sec. 5), whose
 *   forward contraction reads only the t = s blocks (the zero blocks must
 *   still be stored: the adjoint and the fitting sweep read the full core);
 *   NULL means all general.
 * Truncation (qtt_opts).  At every bond, with lam_i the squared singular
 *   values in descending order, keep
 *       k = min(cap, k_eps, #{lam_i > tau * lam_1}), at least 1,
 *   k_eps = smallest k with sum_{i>k} lam_i <= cutoff * sum_i lam_i
 *   (cutoff = 0 disables it).  The zip-up uses cap = chi_zip (0 -> chi_max),
 *   the sweep cap = chi_max.  tau <= 0 selects the default 1e-13.
 * Precision.  QTT_PREC_FP32: complex64 operands, FP32 MFMA contractions;
 *   Gram matrices accumulated and eigen-decomposed in FP64.  QTT_PREC_FP64:
 *   complex128 throughout.  QTT_PREC_BF16 (complex64 storage): contraction
 *   operands rounded to bfloat16 on the way into the matrix cores, FP32
 *   accumulation, FP64 Gram/eigen; usually combined with opts.refine = 1.
 *   QTT_PREC_BF16X3 (complex64 storage): every operand split into two
 *   bfloat16 terms hi + lo and each product formed as hi.hi + hi.lo + lo.hi
 *   on the bfloat16 matrix cores with FP32 accumulation (close to FP32
 *   accuracy).
 * Ownership.  The library never allocates device memory.  Every call takes a
 *   caller-owned device workspace `ws` of at least tt_workspace_size(...)
 *   bytes; its first 256 bytes hold the device status word.
 * Streams.  Every call is enqueued on `stream` (a hipStream_t; NULL = the
 *   default stream) and returns without synchronising.  Calls on one stream
 *   may share a workspace (they run in stream order); calls that may run at
 *   the same time on different streams need disjoint workspaces and disjoint
 *   outputs, since the workspace holds the call's scratch and status word.
 *   The library keeps no device state of its own between calls (the
 *   autotuned tile table and the profiling hooks are host-side), so calls on
 *   different streams with their own workspaces do not interact.
 * Errors.  Argument errors are detected on the host before anything is
 *   enqueued and returned as negative codes.  Numerical failures (non-finite
 *   values reaching an eigensolver) are recorded in the device status word
 *   and reported by tt_check_status after it synchronises the stream.  No
 *   call aborts the process and no C++ exception crosses this boundary.
 *   tt_last_error() returns a message for the last failing call on the
 *   calling thread.
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum qtt_status {
  QTT_OK = 0,
  QTT_ERR_ARG = -1,        /* NULL pointer or invalid parameter              */
  QTT_ERR_SHAPE = -2,      /* side not a power of two, m mismatch, n < 1     */
  QTT_ERR_DTYPE = -3,      /* unsupported or mismatched element type         */
  QTT_ERR_WORKSPACE = -4,  /* workspace (or saved buffer) too small          */
  QTT_ERR_CAPACITY = -5,   /* chi_max > chi_cap, or bonds exceed capacity    */
  QTT_ERR_HIP = -6,        /* a HIP runtime call failed                      */
  QTT_ERR_NONFINITE = -7,  /* device: NaN/Inf reached a Gram/eigensolver     */
  QTT_ERR_NOCONVERGE = -8  /* device: eigenvalue iteration cap reached       */
};

enum qtt_dtype { QTT_C64 = 1, QTT_C128 = 2, QTT_F32 = 3, QTT_F64 = 4 };
enum qtt_prec { QTT_PREC_FP32 = 0, QTT_PREC_BF16 = 1, QTT_PREC_FP64 = 2, QTT_PREC_BF16X3 = 3 };
enum qtt_op {
  QTT_OP_ENCODE = 1, QTT_OP_APPLY = 2, QTT_OP_TRUNCATE = 3,
  QTT_OP_TO_DENSE = 4, QTT_OP_APPLY_BACKWARD = 5, QTT_OP_TO_DENSE_BACKWARD = 6,
  QTT_OP_LOSS = 7
};

typedef struct {
  int32_t n_sites;   /* m = 2n                                             */
  int32_t chi_cap;   /* capacity bond dimension of the storage             */
  int32_t dtype;     /* QTT_C64 or QTT_C128                                */
  void* cores;       /* device, n_sites * chi_cap * 2 * chi_cap elements   */
  int32_t* bonds;    /* device, n_sites + 1 ints                           */
  double* norm;      /* device FP64 scalar ||psi||_2 written by the library, or NULL */
} qtt_mps;

typedef struct {
  int32_t n_sites;
  int32_t d_cap;
  int32_t dtype;              /* QTT_C64 or QTT_C128 (matching the MPS)    */
  const void* cores;          /* device, n_sites * d_cap * 4 * d_cap       */
  const int32_t* d_bonds;     /* HOST, n_sites + 1 ints, d_bonds[0] = d_bonds[m] = 1 */
  const int32_t* site_kind;   /* HOST, n_sites ints or NULL (0 general, 1 identity, 2 diagonal) */
} qtt_mpo;

/* A batch of `count` MPS of identical shape in one allocation: field f's
 * core k at element offset (f * n_sites + k) * chi_cap * 2 * chi_cap, its
 * bonds at bonds[f * (n_sites + 1) + k], its norm at norms[f]. */
typedef struct {
  int32_t count;
  int32_t n_sites;
  int32_t chi_cap;
  int32_t dtype;
  void* cores;
  int32_t* bonds;    /* device, count * (n_sites + 1) */
  double* norms;     /* device, count, or NULL */
} qtt_mps_batch;

/* A batch of `count` MPOs sharing one bond profile (pad cores with zeros to
 * make profiles equal): field f's core k at element offset
 * (f * n_sites + k) * d_cap * 4 * d_cap, dense [D_k][t][s][D_(k+1)]. */
typedef struct {
  int32_t count;
  int32_t n_sites;
  int32_t d_cap;
  int32_t dtype;
  const void* cores;
  const int32_t* d_bonds;     /* HOST, n_sites + 1 ints shared by the batch */
  const int32_t* site_kind;   /* HOST, n_sites ints or NULL */
} qtt_mpo_batch;

typedef struct {
  int32_t chi_max;   /* final bond cap                                     */
  int32_t chi_zip;   /* zip-up bond cap, 0 -> chi_max                      */
  double cutoff;     /* relative discarded-weight target (0 = off)         */
  double tau;        /* numerical-zero threshold on lam_i / lam_1 (<=0: 1e-13) */
  int32_t prec;      /* qtt_prec                                           */
  int32_t refine;    /* 0: plain truncation sweep after the zip-up;
                        1: one two-site variational fitting sweep instead
                        (left to right, initialised from the right-canonical
                        zip-up output, contractions in FP32 -- FP64 for
                        complex128 -- whatever prec is; the refinement pass
                        that follows a BF16 zip-up).  The adjoint covers
                        refine = 0 only. */
} qtt_opts;

/* Bytes of device workspace needed by an operation on MPS of n_sites sites
 * stored at capacity chi_cap, with MPO capacity d_cap (ignored by ops that
 * take no MPO).  Returns 0 on invalid arguments. */
size_t tt_workspace_size(int op, int n_sites, int chi_cap, int d_cap, int prec);

/* Workspace of the batched calls below for `count` fields (capacity sizes
 * as for tt_workspace_size). */
size_t tt_workspace_size_batched(int op, int count, int n_sites, int chi_cap, int d_cap, int prec);

/* Encode an N x N image into a quantics MPS by sequential SVD (Sec. 3, Sec. 4,
 * App. A).  img: device, row-major N x N of img_dtype (F32/F64 real or
 * C64/C128 complex); N = 2^log2_side, log2_side >= 1; out->n_sites must be
 * 2*log2_side; opts->chi_max <= out->chi_cap.  The output is left-canonical
 * with the norm in the last core; *out->norm receives ||img||_2 of the kept
 * approximation.  opts->prec selects FP32 (out C64) or FP64 (out C128). */
int tt_encode(const void* img, int img_dtype, int log2_side, const qtt_opts* opts,
              qtt_mps* out, void* ws, size_t ws_bytes, void* stream);

/* out = W . in by zip-up (right to left, cap chi_zip) followed by an SVD
 * truncation sweep (left to right, cap chi_max): the MPO x MPS product of
 * Sec. 5 with truncation.  `in` should be left-canonical (as produced by
 * tt_encode, tt_truncate and mpo_apply).  out is left-canonical, *out->norm =
 * ||out||.  in and out must not alias.  saved: if non-NULL, a device buffer of
 * at least tt_saved_size(...) bytes that receives what mpo_apply_backward needs
 * (per-site carries and centres, every truncation's full eigen-decomposition);
 * NULL skips it. */
int mpo_apply(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts,
              qtt_mps* out, void* saved, size_t saved_bytes,
              void* ws, size_t ws_bytes, void* stream);

/* Batched forms: every field advances site by site in lockstep, one launch
 * per kernel covering the whole batch, so the per-bond eigen-decompositions
 * of different fields run concurrently.  img: count row-major N x N images
 * back to back; chi_dev: NULL or device ints (one per field) that lower the
 * bond cap of individual fields below opts->chi_max (uneven chi in one
 * batch).  Fields of different side length are batched by zero-padding them
 * to a common side with identity MPO sites on the padded bits. */
int tt_encode_batched(const void* img, int img_dtype, int log2_side, const qtt_opts* opts, const int32_t* chi_dev,
                      qtt_mps_batch* out, void* ws, size_t ws_bytes, void* stream);
int mpo_apply_batched(const qtt_mps_batch* in, const qtt_mpo_batch* W, const qtt_opts* opts, const int32_t* chi_dev,
                      qtt_mps_batch* out, void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, void* stream);
int tt_to_dense_batched(const qtt_mps_batch* in, void* out, int out_dtype, void* ws, size_t ws_bytes, void* stream);

/* Element-wise (Hadamard) product of two fields in MPS form, out = a (.) b,
 * or conj(a) (.) b if conj_a (Sec. 5: the local contraction of physical
 * indices that maps the focal-plane field to the PSF, |phi> (.) |phi>^dag,
 * and the product of the two spectra in the image-formation equation).  It is
 * computed as the application of the diagonal operator of a (cores
 * delta_ts A_k, built on the device from a's cores and device bonds; bonds
 * bounded by a->chi_cap) to b: zip-up with the diagonal-site contraction,
 * cap opts->chi_zip, then the truncation sweep to opts->chi_max, exactly as
 * mpo_apply.  a and b: same n_sites and dtype; out must not alias either.
 * out is left-canonical, *out->norm = ||out||.  Workspace:
 * tt_hadamard_workspace_size(n_sites, a->chi_cap, max capacity of b / out /
 * chi_zip, prec). */
size_t tt_hadamard_workspace_size(int n_sites, int chi_cap_a, int chi_cap, int prec);
int tt_hadamard(const qtt_mps* a, int conj_a, const qtt_mps* b, const qtt_opts* opts, qtt_mps* out, void* ws,
                size_t ws_bytes, void* stream);

/* Recompress an MPS in place (the truncation of Sec. 4 and App. A applied to
 * an existing MPS: every bond is a Schmidt cut whose singular values decide
 * what is kept): orthogonalisation right to left, then an SVD truncation
 * sweep left to right with cap opts->chi_max and the keep rule above
 * (TT-rounding).  The input may be any MPS whose inner bonds fit its
 * capacity (not necessarily canonical, bonds not limited to 2^k: a sum of
 * MPS is one).  Output left-canonical, *inout->norm = ||result||.  The
 * bonds are rewritten on the device; cores outside them are left as they
 * were.  Workspace: tt_workspace_size(QTT_OP_TRUNCATE, ...). */
int tt_truncate(qtt_mps* inout, const qtt_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* Decompress: out[a][b] (row-major N x N, out_dtype C64 or C128) = the field
 * the MPS represents (Sec. 3, decompression in Fig. 6). */
int tt_to_dense(const qtt_mps* in, void* out, int out_dtype, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the `saved` buffer mpo_apply / mpo_apply_batched need for a later
 * backward call (capacity bound for chi_zip <= chi_cap; the call itself
 * checks the exact requirement).  The buffer receives the bonds chosen by the
 * forward call, the zip-up cores, the carry entering each zip-up site and the
 * site matrix M formed there, the centre entering each sweep step, and the
 * full eigen-decomposition of every truncation's Gram matrix, computed by the
 * forward beside its keep rule (all n eigenvectors as an L x L matrix in the
 * working precision plus L FP64 eigenvalues per truncation and field, L =
 * twice the largest bond a truncation splits; two truncations per site), so
 * that the backward call differentiates the very factorisations the forward
 * truncated with and runs no eigensolver and no site product of its own. */
size_t tt_saved_size(int n_sites, int chi_cap, int d_cap, int prec);
size_t tt_saved_size_batched(int count, int n_sites, int chi_cap, int d_cap, int prec);

/* Adjoint of mpo_apply (vector-Jacobian product), for gradient-based inverse
 * problems such as phase retrieval (the paper's outlook, Sec. 7).  Given the
 * forward input `in`, the operator W, the options used forward, the `saved`
 * buffer the forward call filled, the forward output `out` (cores and bonds)
 * and grad_out (same shape as out; PyTorch convention for a real loss L:
 * dL/dRe + i dL/dIm), writes grad_in (same shape as in; padding zeroed,
 * bonds = the forward input bonds).  Each truncation is differentiated at the
 * forward's kept ranks through the full FP64 eigen-decomposition of its Gram
 * matrix that the forward computed and kept in `saved` (the buffer is read,
 * not modified); the contribution of
 * rotations inside a kept block is omitted (it vanishes for every function of
 * the decompressed field).  Valid for cotangents of such functions (e.g. the
 * output of tt_to_dense_backward).  Workspace: tt_workspace_size(
 * QTT_OP_APPLY_BACKWARD, ...).  The adjoint eigenproblems are at most
 * 2*chi in size and must not exceed 512. */
int mpo_apply_backward(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts,
                       const void* saved, size_t saved_bytes,
                       const qtt_mps* out, const qtt_mps* grad_out, qtt_mps* grad_in,
                       void* ws, size_t ws_bytes, void* stream);
int mpo_apply_backward_batched(const qtt_mps_batch* in, const qtt_mpo_batch* W, const qtt_opts* opts,
                               const void* saved, size_t saved_bytes,
                               const qtt_mps_batch* out, const qtt_mps_batch* grad_out,
                               qtt_mps_batch* grad_in, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of tt_to_dense: grad_dense (device row-major N x N complex, same
 * dtype as the MPS; count fields back to back for the batched form) -> grad
 * (same shape as in; padding zeroed, bonds = the input bonds).  Workspace:
 * tt_workspace_size(QTT_OP_TO_DENSE_BACKWARD, ...). */
int tt_to_dense_backward(const qtt_mps* in, const void* grad_dense, qtt_mps* grad,
                         void* ws, size_t ws_bytes, void* stream);
int tt_to_dense_backward_batched(const qtt_mps_batch* in, const void* grad_dense, qtt_mps_batch* grad,
                                 void* ws, size_t ws_bytes, void* stream);

/* Intensity loss of the phase-retrieval objective, per field f of `count`
 * N x N fields (N = 2^log2_side) stored back to back:
 *     loss[f] = sum_px (|E|^2 - I_target)^2      (device doubles),
 * and, if grad is non-NULL, grad = dL/dRe + i dL/dIm = 4 (|E|^2 - I) E in the
 * field's layout.  dtype QTT_C64 (target float) or QTT_C128 (target double).
 * Workspace: tt_workspace_size_batched(QTT_OP_LOSS, count, ...) bytes (only
 * the count matters); fixed-order reduction, so results are reproducible. */
int tt_intensity_loss(const void* field, const void* target, int dtype, int log2_side, int count,
                      double* loss, void* grad, void* ws, size_t ws_bytes, void* stream);

/* ---- fields too large to densify ----
 * tt_encode_separable: E0[a][b] = vec_a[a] * vec_b[b] on a 2^n x 2^n grid
 * (n = log2_side, even) without forming the 2-D array: each vector is
 * encoded as a 1-D MPS of n sites by sequential SVD (cap c1 = the largest
 * integer with c1^2 <= out->chi_cap, keep rule with tau = 1e-13) and the two
 * are interleaved in quantics order (Sec. 3): the site of bit p of a carries
 * core_a(p) x identity, the site of bit p of b identity x core_b(p), so every
 * bond is a product of the factors' bonds.  vec_dtype F32/F64/C64/C128 (the
 * MPS dtype decides the compute precision).  out->norm is not written and
 * the result is left-orthonormal except for its last two cores.  Workspace:
 * tt_encode_separable_workspace_size(log2_side, chi_cap, prec).
 * tt_eval_points: out[p] = the field at pixel (rows[p], cols[p]) for count
 * points (device int arrays; device output of the MPS dtype), all points
 * contracted site by site together.  Workspace: tt_eval_points_workspace_size.
 * tt_to_dense_block: the aligned 2^log2_block square block (block_row,
 * block_col) of the field (row-major, out_dtype C64/C128): the high bits are
 * contracted into a boundary vector, the remaining sites decompressed.
 * Workspace: tt_to_dense_block_workspace_size. */
size_t tt_encode_separable_workspace_size(int log2_side, int chi_cap, int prec);
int tt_encode_separable(const void* vec_a, const void* vec_b, int vec_dtype, int log2_side, qtt_mps* out,
                        void* ws, size_t ws_bytes, void* stream);
/* tt_encode_low_rank: E0[a][b] = sum_r vecs_a[r][a] * vecs_b[r][b], r < rank,
 * on a 2^n x 2^n grid (n = log2_side, even) without forming the 2-D array.
 * The sequential SVD of a dense field costs exponentially in the number of
 * sites (Sec. 4); a field of low separation rank is built instead from its
 * factors: every term is encoded as by tt_encode_separable with bond cap
 * term_cap, the rank terms are summed as MPS (bonds add: first core side by
 * side, last core stacked, the rest block-diagonal), and the sum is
 * recompressed by TT-rounding (as tt_truncate, keep rule of opts: Sec. 4).
 * vecs_a, vecs_b: device, rank x 2^n elements each, row r = term r, dtype
 * vec_dtype (F32/F64/C64/C128; the MPS dtype decides the precision).
 * rank in [1, 16]; rank * term_cap <= out->chi_cap <= 256 (the sum's bonds
 * must fit before rounding).  out: left-canonical, bonds <= opts->chi_max,
 * *out->norm written when not NULL.  Workspace:
 * tt_encode_low_rank_workspace_size(log2_side, rank, term_cap, out->chi_cap,
 * prec), its first bytes the status word of every step. */
size_t tt_encode_low_rank_workspace_size(int log2_side, int rank, int term_cap, int chi_cap, int prec);
int tt_encode_low_rank(const void* vecs_a, const void* vecs_b, int vec_dtype, int log2_side, int rank, int term_cap,
                       qtt_mps* out, const qtt_opts* opts, void* ws, size_t ws_bytes, void* stream);
/* tt_sample: perfect sampling of photon detection events (Sec. 5: samples
 * drawn from |E(a, b)|^2 / ||E||^2 directly from an orthogonalised MPS, with
 * O(chi^2) work per site and sample, the distribution never formed).  in must
 * be left-canonical (the output of tt_encode, mpo_apply, tt_truncate; the
 * norm may sit in the last core): sites are visited from the last to the
 * first, and with the sites left of k an isometry the probability of bit s
 * at site k given the bits drawn right of it is |A_k[s] R|^2 over the sum of
 * both, R the boundary vector of the drawn bits (renormalised each site).
 * uniforms: device, count x n_sites doubles in [0, 1): sample p takes bit 0
 * at site k when uniforms[p * n_sites + k] * (p0 + p1) < p0.  rows, cols:
 * device int32 outputs (pixel coordinates, most significant bit at the first
 * site).  Products in the MPS precision, probabilities summed in FP64.
 * Workspace: tt_sample_workspace_size(n_sites, chi_cap, count, prec). */
size_t tt_sample_workspace_size(int n_sites, int chi_cap, int count, int prec);
int tt_sample(const qtt_mps* in, const double* uniforms, int count, int32_t* rows, int32_t* cols, void* ws,
              size_t ws_bytes, void* stream);
size_t tt_eval_points_workspace_size(int n_sites, int chi_cap, int count, int prec);
int tt_eval_points(const qtt_mps* in, const int32_t* rows, const int32_t* cols, int count, void* out,
                   void* ws, size_t ws_bytes, void* stream);
size_t tt_to_dense_block_workspace_size(int n_sites, int chi_cap, int log2_block, int prec);
int tt_to_dense_block(const qtt_mps* in, int log2_block, int block_row, int block_col, void* out, int out_dtype,
                      void* ws, size_t ws_bytes, void* stream);

/* Decompression of a window (Sec. 3, decompression in Fig. 6): out[i][j]
 * (row-major rows x cols, out_dtype C64/C128, device) = the field at pixel
 * (row0 + i, col0 + j), for any window inside the N x N field.  It is
 * assembled from the aligned 2^log2_block blocks that cover it (log2_block
 * <= 0: half the window's longer side rounded up to a power of two, so at
 * most 3 x 3 blocks), each decompressed by tt_to_dense_block into a scratch
 * block in ws and its part of the window copied out; nothing else of the
 * field is formed.  Errors: QTT_ERR_SHAPE for a window outside the field or a
 * block size outside [1, n].  Workspace:
 * tt_to_dense_window_workspace_size(n_sites, chi_cap, rows, cols, log2_block,
 * prec). */
size_t tt_to_dense_window_workspace_size(int n_sites, int chi_cap, int rows, int cols, int log2_block, int prec);
int tt_to_dense_window(const qtt_mps* in, int row0, int col0, int rows, int cols, int log2_block, void* out,
                       int out_dtype, void* ws, size_t ws_bytes, void* stream);

/* ---- auxiliary entry points (the building blocks of the calls above) ---- */

/* C = op(A) . op(B) for dense row-major complex matrices through the MFMA
 * contraction kernel used by every step above.  A is M x K (lda), B is K x N
 * (ldb), C is M x N (ldc), all device pointers; conj_a / conj_b conjugate the
 * operand elements.  prec QTT_PREC_FP32 (complex64), QTT_PREC_BF16 /
 * QTT_PREC_BF16X3 (complex64 in memory, bfloat16 matrix cores, FP32
 * accumulation) or QTT_PREC_FP64 (complex128).  Asynchronous on `stream`. */
int tt_cgemm(int M, int N, int K, const void* A, int lda, int conj_a, const void* B, int ldb, int conj_b,
             void* C, int ldc, int prec, void* stream);

/* Batched Hermitian eigen-decomposition with the keep rule of the truncation
 * steps (Sec. 4: squared singular values of a bond cut are the eigenvalues of
 * its Gram matrix).  G: device, batch x n x n complex128 row-major Hermitian;
 * only the lower triangle (with the diagonal) is referenced; the upper
 * triangle is overwritten.  Writes, per matrix b: kept[b] (device int) from the keep
 * rule with cap kcap / cutoff / tau, evals[b*kcap + i] (device double, the
 * kept eigenvalues in descending order, zero beyond kept[b]) and
 * evecs[b*n*kcap + p*kcap + i] (device complex128, eigenvector i).  n <= 512.
 * ws: tt_heev_workspace_size(n, kcap, batch) bytes. */
size_t tt_heev_workspace_size(int n, int kcap, int batch);
int tt_heev(void* G, int n, int batch, int kcap, double cutoff, double tau, int* kept, double* evals,
            void* evecs, void* ws, size_t ws_bytes, void* stream);

/* ---- diagnostics: per-launch timing of one kernel class ----
 * tt_prof_begin(what, nlog, max_entries, max_launches): from now on, every
 * launch of kernel class `what` (1 = the multi-workgroup or streaming
 * Householder tridiagonalisation of Gram matrices larger than 128, which
 * takes their first n - 128 steps; 2 = the LDS-resident one, which reduces
 * matrices up to 128 and the trailing 128 x 128 block of larger ones) is
 * bracketed by HIP events on its stream and writes the size n of the matrix
 * (class 1) or of the block it reduces (class 2) to the device int array
 * nlog (one entry per matrix).
 * tt_prof_end(launches, entries, total_ms): synchronise, return the number of
 * launches, of nlog entries written, and the summed event time in ms; stops
 * recording.  Not thread-safe; intended for benchmarks. */
int tt_prof_begin(int what, int* nlog, int max_entries, int max_launches);
int tt_prof_end(int* launches, int* entries, double* total_ms);
/* tt_prof_begin_flops(flog, max_launches): from now on every contraction the
 * library enqueues (products and Gram matrices, with their K-split reductions)
 * is bracketed by HIP events on its stream, and after the closing event a
 * one-thread kernel adds the product's algorithmic flops -- 8 M N K per
 * complex product, 4 n^2 K per Hermitian Gram (its lower half), from the
 * device-side sizes summed over fields -- to flog[2 i] (FP32-MFMA products)
 * or flog[2 i + 1] (FP64-accumulating ones) for launch i.  flog: device
 * doubles, 2 * max_launches, zeroed by the caller.  Ends with tt_prof_end
 * (entries is then 0).  tt_prof_times(ms, max): after tt_prof_end, the event
 * time of each recorded launch (host floats, ms); returns how many were
 * written or a negative qtt_status.  Diagnostics only: not thread-safe, and
 * the extra kernels make a profiled run slower. */
int tt_prof_begin_flops(double* flog, int max_launches);
int tt_prof_times(float* ms, int max);

/* ---- tile autotuner of the contraction kernel ----
 * The contraction kernel has several output-tile variants (64x64, 32x64,
 * 32x32 complex per workgroup; for FP32 operands with FP32 accumulation also
 * 128x64 and 128x128, variants 3 and 4).  tt_autotune_record(1) starts
 * collecting the call shapes (element types, host bounds of the output, grid
 * depth, operand access pattern) of every contraction enqueued afterwards,
 * each with the largest contraction depth one workgroup reduces over; (0)
 * stops.  tt_autotune_run times every variant on synthetic operands of each
 * recorded shape at that depth (clamped to 16..1024) on `stream`
 * (synchronises; needs tt_autotune_workspace_size() bytes of device memory)
 * and from then on every contraction of that shape uses the fastest (outputs
 * larger than 4096 x 4096 keep the 64x64 tile).
 * Variants differ only in how the output is partitioned, so results are
 * bit-identical whatever is chosen.  tt_autotune_export writes
 * up to max_entries 6-int entries (types, m, n, depth, pattern, variant) and
 * returns the table size; tt_autotune_import loads such entries (invalid
 * ones are skipped and reported).  Host state, not thread-safe; choices are
 * read when a call is enqueued, so capture graphs after tuning. */
int tt_autotune_record(int on);
size_t tt_autotune_workspace_size(void);
int tt_autotune_run(void* ws, size_t ws_bytes, void* stream, int* n_tuned);
int tt_autotune_export(int32_t* entries, int max_entries);
int tt_autotune_import(const int32_t* entries, int n);
int tt_autotune_clear(void);

/* ---- allocation-free application ----
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same computation, kernels and results as mpo_apply (no saved
 * buffer), with the workspace taken from a static device array of
 * QTT_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (address looked up once per device; the stream's
 * device must be the current device).  Nothing is allocated by the call.
 * Problems whose workspace (tt_workspace_size for these exact sizes) exceeds
 * the array are rejected with QTT_ERR_WORKSPACE before anything is enqueued.
 * The array's status word is cleared at the start of every call and, if
 * status_out (device int) is non-NULL, copied there at the end (QTT_OK or a
 * negative qtt_status), in stream order.  Every call on one GPU shares the
 * array and it keeps the last call's contents: calls that may overlap on one
 * GPU (different streams, or several host threads) race and must be
 * serialised by the caller. */
#define QTT_NOALLOC_SCRATCH_BYTES (64u << 20)
int mpo_apply_noalloc(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts, qtt_mps* out,
                      int32_t* status_out, void* stream);

/* Synchronise `stream`, read the device status word in ws, reset it to 0 and
 * return it (QTT_OK or a negative qtt_status). */
int tt_check_status(void* ws, void* stream);

/* Message for the last failing call on this thread ("" if none). */
const char* tt_last_error(void);

/* Library version string. */
const char* tt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QTT_H */
