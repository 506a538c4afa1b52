// Host-side launch interface of the libqtt kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace qtt {

// GEMM_BF16: complex64 operands rounded to bfloat16, FP32 accumulation.
// GEMM_BF16X3: operands split into two bfloat16 terms (hi + lo), products
// hi.hi + hi.lo + lo.hi on the bfloat16 matrix cores, FP32 accumulation.
enum GemmTypes { GEMM_F32 = 0, GEMM_F32_GRAM64 = 1, GEMM_F64 = 2, GEMM_BF16 = 3, GEMM_BF16X3 = 4 };

// C(M,N) = op(A)(M,K) . op(B)(K,N), batched.  Sizes are device expressions;
// *_bound are host upper bounds used only to size the launch grid.
struct GemmSpec {
  DimExpr M, N, K, batch;
  int mlo, nlo, klo;            // low extents of the split indices (1 = unsplit)
  int m_bound, n_bound, batch_bound;
  int k_bound = 1 << 30;
  int nfield = 1;               // outer batch: fields (Operand.sb strides)
  Operand A, B, C;
  int accumulate = 0;
  int lower = 0;                // Hermitian result: only tiles touching the lower triangle
  int ksplit = 1;
  long long csplit = 0;
  int types = GEMM_F32;
};

FastDiv make_fastdiv(uint32_t d);
hipError_t gemm_launch(const GemmSpec& sp, hipStream_t s);
// Algorithmic flops of the product sp describes, from its device-side sizes
// (clamped to the host bounds, summed over fields and inner batch): scale *
// M * N * K, added to out[0] for FP32-MFMA types and to out[1] for the
// FP64-accumulating ones.  One thread; for the diagnostics pass only.
hipError_t gemm_flops(const GemmSpec& sp, double scale, double* out, hipStream_t s);
// Tile autotuner (host state, not thread-safe): record the call shapes of a
// run, time every tile variant on synthetic operands of each shape, use the
// fastest from then on; export / import the table as 6-int entries.
void autotune_record(bool on);
size_t autotune_ws_bytes();
hipError_t autotune_run(void* ws, size_t ws_bytes, hipStream_t s, int* n_tuned);
int autotune_export(int* out, int max_entries);
int autotune_import(const int* entries, int n);
void autotune_clear();
// Sum K-chunk partials (leading dimension ldp) into out (ld; only j <= i when lower).
hipError_t ksplit_reduce(const void* part, long long cstride, int nsplit, int ldp, void* out, int ld,
                         DimExpr nrows, DimExpr ncols, int rows_bound, int cols_bound,
                         long long bstride_part, long long bstride_out, int batch_bound, int lower,
                         hipStream_t s);
// Lower-triangle partial Gram matrices X X^H of an operand with at most
// GRAM_SKINNY_N rows (sp.A = X, sp.M its rows, sp.K its columns; sp.B is
// not read): nsplit K chunks per field, partial (f, c) at
// part + (f * nsplit + c) * ldp * ldp.  FP64 accumulation.
constexpr int GRAM_SKINNY_N = 8;
hipError_t gram_skinny(const GemmSpec& sp, int nsplit, double* part, int ldp, hipStream_t s);

// ---------------------------------------------------------------- eigensolver
// Batched Hermitian eigen-decomposition of FP64 Gram matrices followed by the
// keep rule, for the truncation of one bond.  Matrices are n x n (n a device
// value), stored full with leading dimension ld, batch stride gstride.
// Up to kcap eigenpairs (descending) are computed; the kept count k is
// written to *kout (device int, one per batch entry, stride kstride).
struct EigEmit {
  // Writes out[(p / lo) * s_hi + (p % lo) * s_lo + i * s_col] = f(V[p][i])
  // for p < n, i < k, where f applies conj (if conj) and multiplies by
  // sigma_i^pow (pow in {-1, 0, 1}).  dtype: 0 = complex float, 1 = complex double.
  void* ptr = nullptr;
  long long s_hi = 0, s_lo = 0, s_col = 0, s_batch = 0;
  int lo = 1;
  int conj = 0;
  int pow = 0;
  int dtype = 0;
  int all = 0;                // with EigSpec::lam_out: every computed vector, not only the kept ones (pow 0)
};

struct EigSpec {
  double* G;                  // n x n Hermitian (destroyed)
  int ld;
  long long gstride;
  DimExpr n;
  int n_bound;
  int kcap;                   // bond cap
  double cutoff, tau;
  int* kout;                  // device, kept counts
  long long kstride;
  const int* kcap_dev = nullptr;  // optional per-matrix cap (stride 1), e.g. per-field chi
  int batch;                  // number of matrices (host-known)
  // workspace pointers (carved by the caller; sizes from eig_ws_bytes)
  void* ws;
  int* status;
  EigEmit emit[3];
  int nemit;
  double* sigma_out;          // optional: device FP64 singular values [batch][kcap]
  // Optional full decomposition beside the truncation: with lam_out set,
  // every eigenpair up to kcap (normally n_bound) is computed, all of them
  // reach the emits marked `all` and the eigenvalues reach lam_out[b * lam_ld
  // + t] (t < n, descending), while the keep rule and the other emits use the
  // cap keep_cap.
  double* lam_out = nullptr;
  long long lam_ld = 0;
  int keep_cap = 0;
};

size_t eig_ws_bytes(int n_bound, int kcap, int batch);

// Optional per-launch timing of one kernel class (diagnostics for the
// roofline report): HIP events are recorded around every launch of the
// selected class on its stream, and the kernel writes its actual problem size
// to nlog[slot] so algorithmic work can be computed from real sizes.
enum ProfWhat { PROF_NONE = 0, PROF_TRIDIAG = 1, PROF_TRIDIAG_LDS = 2, PROF_GEMM = 3 };
struct ProfHook {
  int what = PROF_NONE;
  int* nlog = nullptr;       // device ints: per launch, per batch entry
  double* flog = nullptr;    // PROF_GEMM: device doubles, two per launch (FP32-MFMA and FP64-MFMA flops)
  int max = 0;               // capacity of nlog (entries)
  int slot = 0;              // next free entry
  int launches = 0;
  hipEvent_t* ev = nullptr;  // 2 * max_launches events
  int max_launches = 0;
};
extern ProfHook g_prof;
hipError_t eig_launch(const EigSpec& sp, hipStream_t s);
hipError_t eig_copy_evals(const EigSpec& sp, double* out, int ldo, hipStream_t s);
// Eigenvector-adjoint scaling after a full decomposition: Y[j][i] (row j =
// eigenvector index < n, column i < kk[f]) becomes
//   Y[j][i] / (lam_i - lam_j)  for kk[f] <= j < n where lam_i - lam_j >
//   1e-10 lam_1, and 0 otherwise (pairs whose Gram eigenvectors are not
//   resolved well enough for a term divided by their gap),
// with lam[f * lam_ld + t] the n eigenvalues (descending) of matrix f.
hipError_t eig_adjoint_scale(DimExpr n, int n_bound, const double* lam, long long lam_ld, int batch, void* Y,
                             long long ldy, long long s_batch, const int* kk, long long kk_stride, int kk_bound,
                             int dtype, hipStream_t s);

// ---------------------------------------------------------------- misc
// Quantics permutation of a row-major N x N image into the flat quantics
// vector (dir = 0) or back (dir = 1).  src/dst element types given by the
// qtt_dtype codes; the quantics side is always complex (float or double).
// nf fields at element strides s_src / s_dst (one launch).
hipError_t quantics_permute(const void* src, int src_dtype, void* dst, int dst_dtype, int log2_side,
                            int dir, hipStream_t s, int nf = 1, long long s_src = 0, long long s_dst = 0);
// Frobenius norm of a (rows x cols) complex block (strides ld_r, ld_c), FP64 result.
hipError_t block_norm(const void* p, int dtype, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                      long long ld_r, long long ld_c, double* out, hipStream_t s);
// Store complex 1 at p[0] (dtype 0 float, 1 double).
hipError_t set_one(void* p, int dtype, hipStream_t s);
// Copy a (rows x cols) complex block with arbitrary strides (dtype 0 float, 1 double).
hipError_t block_copy(const void* src, long long s_rs, long long s_cs, void* dst, long long d_rs,
                      long long d_cs, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound, int dtype,
                      hipStream_t s);
// Set dev[i] = val for the given list (used for boundary bonds).
hipError_t set_ints(int* dev, int count, int val, hipStream_t s);
hipError_t copy_ints(const int* src, int* dst, int count, hipStream_t s);
// Clamped copy of caller bonds (see misc.hip); nf fields at stride m+1.
// free_inner: inner bonds bounded by cap only (not by 2^min(k, m - k)).
hipError_t sanitize_bonds(const int* src, int* dst, int m, int cap, int* status, int nf, hipStream_t s,
                          int free_inner = 0);
// Batched (nf fields) versions of the small helpers: field f adds f * stride.
hipError_t block_copy_b(const void* src, long long s_rs, long long s_cs, long long s_f, void* dst, long long d_rs,
                        long long d_cs, long long d_f, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                        int dtype, int nf, hipStream_t s, int conj = 0);
// Complete Hermitian matrices from their lower triangle: G[i][j] =
// conj(G[j][i]) for i < j < n (n a device value per matrix, ld, stride gs).
hipError_t hermitian_fill(double* G, int ld, long long gs, DimExpr n, int n_bound, int nf, hipStream_t s);
// Zero a buffer (bytes a multiple of 16) with a plain kernel.
hipError_t zero_fill(void* p, size_t bytes, hipStream_t s);
// Phase-retrieval loss per field, L_f = sum (|E|^2 - I)^2, and its gradient
// 4 (|E|^2 - I) E (NULL grad skips it).  dtype 0: complex64 field and float
// target; 1: complex128 and double.  part: intensity_loss_ws(nf) bytes.
size_t intensity_loss_ws(int nf);
hipError_t intensity_loss(const void* field, const void* target, int dtype, long long per, int nf, double* loss,
                          void* grad, void* part, hipStream_t s);
hipError_t block_norm_b(const void* p, int dtype, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                        long long ld_r, long long ld_c, long long s_f, double* out, int nf, hipStream_t s);
hipError_t set_ints_strided(int* dev, int per, long long stride, int nf, int val, hipStream_t s);
hipError_t set_one_b(void* p, long long s_f, int dtype, int nf, hipStream_t s);
// Separable fields: interleave two 1-D MPS of n_per_axis sites (capacities
// ucap, vcap; device bonds ub, vb) into a 2 n_per_axis site MPS (capacity
// ocap, bonds ob).  dtype 0 complex64, 1 complex128.
hipError_t interleave(const void* U, const int* ub, int ucap, const void* V, const int* vb, int vcap, void* out,
                      int* ob, int ocap, int n_per_axis, int dtype, int* status, hipStream_t s);
// Point evaluation helpers: Lnext[p][r] = C[p][2 r + bit of point p at site];
// the final value is column 0; unit_rows sets every row to e_0.
hipError_t select_bit(const void* C, long long ldc, void* Lnext, long long ldl, const int* rows, const int* cols,
                      int count, int site, int n, const int* rbond, int cap, int dtype, hipStream_t s);
hipError_t gather_col0(const void* Lf, long long ldl, void* out, int count, int dtype, hipStream_t s);
hipError_t unit_rows(void* L, long long ldl, int count, int cap, int dtype, hipStream_t s);
hipError_t fill_point(int* rows, int* cols, int row, int col, hipStream_t s);
// Diagonal MPO of an MPS for the element-wise product: core k dense
// [D_k][t][s][D_(k+1)] at element offset k * dcap * 4 * dcap with D_k =
// min(cap, 2^k, 2^(m-k)), W = delta_ts A_k (conj if conj), zero outside the
// MPS's device bonds.  dtype 0 complex64, 1 complex128.
hipError_t mps_to_diag_mpo(const void* A, const int* bonds, int cap, int conj, void* W, int dcap, int m, int dtype,
                           hipStream_t s);
// Most terms a low-rank encode sums, and the status code of a sum whose
// bonds exceed the output capacity (QTT_ERR_CAPACITY).
constexpr int QTT_MAX_RANK = 16;
constexpr int ST_CAPACITY = -5;
// Direct sum of `rank` MPS of m sites (capacity tcap each, back to back with
// their device bonds) into one MPS of capacity ocap whose bond at every inner
// cut is the sum of the terms' bonds: first core side by side, last core
// stacked, the others block-diagonal; every element of the output capacity is
// written.  A sum that exceeds ocap flags QTT_ERR_CAPACITY in the status word.
hipError_t direct_sum(const void* terms, const int* tbonds, int rank, int tcap, int m, void* out, int* ob, int ocap,
                      int dtype, int* status, hipStream_t s);
// Perfect sampling, one site for every sample: from C[p][2 r + s] (the core
// of site k applied to sample p's boundary vector) draw bit s with
// probability |C[p][2 . + s]|^2 / |C[p]|^2 against uni[p * m + site], write
// the normalised C[p][2 . + s] to Rn[p] (zero beyond the bond) and the bit into
// rows[p] (even site) or cols[p] (odd site), most significant bit first.
hipError_t sample_select(const void* C, long long ldc, void* Rn, long long ldr, const double* uni, int m, int site,
                         const int* bond, int cap, int* rows, int* cols, int count, int dtype, hipStream_t s);
// Scan a complex buffer for non-finite values and flag the status word.
hipError_t check_finite(const void* p, int dtype, long long count, int* status, hipStream_t s);

}  // namespace qtt
