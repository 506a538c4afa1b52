// C ABI of libqtt: argument checks, workspace carving and the per-site launch
// sequences of the quantics-MPS path.  Everything is enqueued on the caller's
// stream; bond dimensions chosen on the device are consumed on the device.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qtt.h"
#include "kernels.h"

using namespace qtt;
typedef long long ll;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) return fail(QTT_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

DimExpr dx(int c, const int* p0 = nullptr, const int* p1 = nullptr, int bs = 0) {
  DimExpr d;
  d.c = c;
  d.p0 = p0;
  d.p1 = p1;
  d.bs = bs;
  return d;
}

// Operand view; sb = stride between fields.
Operand opd(const void* p, ll sxh, ll sxl, ll syh, ll syl, int conj = 0, ll sb = 0, ll sb2 = 0) {
  Operand o;
  o.ptr = const_cast<void*>(p);
  o.sxh = sxh; o.sxl = sxl; o.syh = syh; o.syl = syl;
  o.conj = conj;
  o.sb = sb;
  o.sb2 = sb2;
  return o;
}

ll pow2_cap(int e, ll cap) { return e >= 40 ? cap : std::min<ll>(cap, 1ll << e); }

// Workspace carving: the same code computes sizes (base == nullptr) and
// pointers, so the size queries and the entry points always agree.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    off = (off + 255) / 256 * 256;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

constexpr size_t PART_BYTES = 96ull << 20;   // Gram K-split partials (all fields)

int ksplit_for(int nb, ll kb, int nf) {
  // lower-triangle tiles only; aim at about eight workgroups per compute
  // unit, each K chunk at least 64 deep; partials are nb x nb per chunk
  const int t = (nb + 63) / 64;
  int tiles = t * (t + 1) / 2 * std::max(nf, 1);
  ll want = std::max<ll>(1, 2048 / std::max(tiles, 1));
  ll bykb = std::max<ll>(1, kb / 64);
  ll bymem = std::max<ll>(1, (ll)(PART_BYTES / (16ull * (size_t)nb * nb * std::max(nf, 1))));
  return (int)std::min<ll>({want, bykb, bymem, 256});
}

struct Ctx {
  hipStream_t s;
  int real;            // 0 float, 1 double
  int gemm_t;          // GEMM_F32 / GEMM_F64
  int gram_t;          // GEMM_F32_GRAM64 / GEMM_F64
  size_t csz;          // bytes per complex element
  int nf = 1;          // fields in the batch
  int bs = 0;          // per-field stride of bond arrays (ints)
  int* status;
  double* G;           // nf Gram matrices, ld gld, stride gld^2
  int gld;
  double* part;
  void* eigws;
  int eig_nb, eig_kc;
  const int* kcap_dev = nullptr;   // optional per-field bond cap
};

DimExpr dv(const Ctx& c, int k, const int* p0 = nullptr, const int* p1 = nullptr) { return dx(k, p0, p1, c.bs); }

// Diagnostics pass (tt_prof_begin_flops): every contraction below is
// bracketed by HIP events on its stream; after the closing event a one-thread
// kernel adds its algorithmic flops to the launch's two log entries.
struct GemmProf {
  bool on;
  hipStream_t s;
  explicit GemmProf(hipStream_t st) : s(st) {
    on = g_prof.what == PROF_GEMM && g_prof.launches < g_prof.max_launches;
    if (on) hipEventRecord(g_prof.ev[2 * g_prof.launches], s);
  }
  void done(const GemmSpec& g, double scale) {
    if (!on) return;
    hipEventRecord(g_prof.ev[2 * g_prof.launches + 1], s);
    gemm_flops(g, scale, g_prof.flog + 2 * g_prof.launches, s);
    g_prof.launches++;
  }
};

// Hermitian Gram matrices (one per field) into ctx.G: G = op(A) . op(B).
// Only the tiles touching the lower triangle are computed: the eigensolver
// references the lower triangle alone.  K-split partials are nb x nb.
int gram(Ctx& c, const Operand& A, const Operand& B, DimExpr n, int nlo, int nb, DimExpr K, int klo, ll kb) {
  const ll ld = c.gld, gs = ld * ld;
  const ll gsp = (ll)nb * nb;
  GemmSpec g;
  g.M = n; g.N = n; g.K = K; g.batch = dx(1);
  g.mlo = nlo; g.nlo = nlo; g.klo = klo;
  g.m_bound = nb; g.n_bound = nb; g.batch_bound = 1; g.nfield = c.nf;
  g.A = A; g.B = B;
  g.types = c.gram_t;
  g.lower = 1;
  // B = A^H over the same data: a few rows against a long K streams through
  // the dedicated kernel instead of mostly-padding MFMA tiles
  const bool herm = B.ptr == A.ptr && B.conj != A.conj && B.sxh == A.syh && B.sxl == A.syl && B.syh == A.sxh &&
                    B.syl == A.sxl && B.sb == A.sb && B.sb2 == A.sb2;
  // algorithmic work of a Hermitian Gram: the lower half, 4 n^2 K flops
  GemmProf prof(c.s);
  if (herm && nb <= GRAM_SKINNY_N) {
    ll want = std::max<ll>(1, 2048 / std::max(c.nf, 1));
    ll byk = std::max<ll>(1, kb / 1024);
    ll bymem = std::max<ll>(1, (ll)(PART_BYTES / (16ull * (size_t)gsp * std::max(c.nf, 1))));
    const int ns = (int)std::min<ll>({want, byk, bymem, 4096});
    HIPCHK(gram_skinny(g, ns, c.part, nb, c.s));
    HIPCHK(ksplit_reduce(c.part, gsp, ns, nb, c.G, c.gld, n, n, nb, nb, (ll)ns * gsp, gs, c.nf, 1, c.s));
    g.k_bound = (int)std::min<ll>(kb, 1 << 30);
    prof.done(g, 4.0);
    return QTT_OK;
  }
  int ks = ksplit_for(nb, kb, c.nf);
  // the result is a plain n x n matrix: address it through the same (hi, lo)
  // split as the M and N indices
  if (ks > 1) {
    g.C = opd(c.part, nlo * nb, nb, nlo, 1, 0, (ll)ks * gsp);
    g.ksplit = ks;
    g.csplit = gsp;
    HIPCHK(gemm_launch(g, c.s));
    HIPCHK(ksplit_reduce(c.part, gsp, ks, nb, c.G, c.gld, n, n, nb, nb, (ll)ks * gsp, gs, c.nf, 1, c.s));
  } else {
    g.C = opd(c.G, nlo * ld, ld, nlo, 1, 0, gs);
    HIPCHK(gemm_launch(g, c.s));
  }
  g.k_bound = (int)std::min<ll>(kb, 1 << 30);
  prof.done(g, 4.0);
  return QTT_OK;
}

int gemm(Ctx& c, DimExpr M, int mlo, int mb, DimExpr N, int nlo, int nb, DimExpr K, int klo, const Operand& A,
         const Operand& B, const Operand& C, DimExpr batch = dx(1), int batch_bound = 1, int accumulate = 0,
         int kb = 1 << 30) {
  GemmSpec g;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.mlo = mlo; g.nlo = nlo; g.klo = klo;
  g.m_bound = mb; g.n_bound = nb; g.k_bound = kb; g.batch_bound = batch_bound; g.nfield = c.nf;
  g.A = A; g.B = B; g.C = C;
  g.accumulate = accumulate;
  g.types = c.gemm_t;
  GemmProf prof(c.s);
  HIPCHK(gemm_launch(g, c.s));
  prof.done(g, 8.0);
  return QTT_OK;
}

EigEmit emit(void* p, int lo, ll s_hi, ll s_lo, ll s_col, int conj, int pow, int dtype, ll s_batch = 0, int all = 0) {
  EigEmit e;
  e.ptr = p; e.lo = lo; e.s_hi = s_hi; e.s_lo = s_lo; e.s_col = s_col;
  e.conj = conj; e.pow = pow; e.dtype = dtype; e.s_batch = s_batch; e.all = all;
  return e;
}

// A full decomposition beside a truncation (EigSpec::lam_out): every pair is
// computed, the eigenvalues go to lam (stride lam_ld per matrix), emits marked
// `all` receive every vector, and the keep rule uses keep_cap.
struct FullOut {
  double* lam = nullptr;
  ll lam_ld = 0;
  int keep_cap = 0;
};

int eig(Ctx& c, DimExpr n, int nb, int kcap, double cutoff, double tau, int* kout, std::initializer_list<EigEmit> em,
        EigSpec* spec_out = nullptr, FullOut full = FullOut()) {
  EigSpec e;
  e.G = c.G; e.ld = c.gld; e.gstride = (ll)c.gld * c.gld;
  e.n = n; e.n_bound = nb;
  e.kcap = std::min(kcap, c.eig_kc);
  e.cutoff = cutoff; e.tau = tau;
  e.kout = kout; e.kstride = c.bs;
  e.kcap_dev = c.kcap_dev;
  e.batch = c.nf;
  e.ws = c.eigws;
  e.status = c.status;
  e.nemit = 0;
  for (const EigEmit& x : em) e.emit[e.nemit++] = x;
  e.sigma_out = nullptr;
  e.lam_out = full.lam;
  e.lam_ld = full.lam_ld;
  e.keep_cap = full.keep_cap;
  if (nb > c.eig_nb) return fail(QTT_ERR_WORKSPACE, "eig size %d exceeds workspace bound %d", nb, c.eig_nb);
  HIPCHK(eig_launch(e, c.s));
  if (spec_out) *spec_out = e;
  return QTT_OK;
}

// ------------------------------------------------------------ bond bounds
std::vector<int> mps_bounds(int m, int chi) {
  std::vector<int> r(m + 1);
  for (int k = 0; k <= m; ++k) r[k] = (int)std::min<ll>(pow2_cap(k, chi), pow2_cap(m - k, chi));
  return r;
}

// ------------------------------------------------------------ apply plan
struct ApplyPlan {
  int m, chi_in, chi_out, chi_zip, chi_max, dcap, zc;   // zc: zip capacity stride
  int refine = 0;                                        // fitting sweep instead of the plain sweep
  int free_in = 0;                                       // inner input bonds bounded by the capacity only
  int diff = 0;                                          // keeps state (full decompositions) for an adjoint
  std::vector<int> rin, beta, rout, D;
  std::vector<int> kind;
  int gram_nb;     // largest Gram size
  int rmax, dmax;
};

// diff: the application keeps state for its adjoint and factors every bond
// on the side the adjoint differentiates (zip-up M^H M, sweep M M^H), so the
// Gram bound covers those sides.
// free_in: the input's inner bonds are bounded by its capacity only, not by
// the physical 2^k (TT-rounding of an arbitrary MPS, e.g. a sum of MPS whose
// bonds add up beyond 2^k at the ends of the chain).
ApplyPlan make_apply_plan(int m, int chi_in, int chi_out, int chi_max, int chi_zip, const int* dbonds,
                          const int* kind, int dcap, int refine = 0, int diff = 0, int free_in = 0) {
  ApplyPlan p;
  p.refine = refine;
  p.diff = diff;
  p.m = m; p.chi_in = chi_in; p.chi_out = chi_out; p.chi_max = chi_max;
  p.chi_zip = chi_zip; p.dcap = dcap;
  p.rin = mps_bounds(m, chi_in);
  p.free_in = free_in;
  if (free_in)
    for (int k = 1; k < m; ++k) p.rin[k] = chi_in;
  p.D.assign(dbonds, dbonds + m + 1);
  p.kind.assign(m, 0);
  if (kind) for (int k = 0; k < m; ++k) p.kind[k] = kind[k];
  p.beta.assign(m + 1, 1);
  for (int k = m - 1; k >= 1; --k) {
    ll b = std::min<ll>({(ll)chi_zip, pow2_cap(m - k, chi_zip), (ll)p.rin[k] * p.D[k], 2ll * p.beta[k + 1]});
    p.beta[k] = (int)std::max<ll>(1, b);
  }
  p.beta[0] = 1;
  p.rout.assign(m + 1, 1);
  for (int k = 0; k < m - 1; ++k)
    p.rout[k + 1] = std::max(1, std::min({chi_max, 2 * p.rout[k], p.beta[k + 1]}));
  p.rout[m] = 1;
  p.zc = 1;
  for (int k = 0; k <= m; ++k) p.zc = std::max(p.zc, p.beta[k]);
  int g = 1;
  for (int k = 1; k < m; ++k) {
    ll pb = (ll)p.rin[k] * p.D[k], qb = 2ll * p.beta[k + 1];
    g = (int)std::max<ll>(g, std::min(pb, qb));
  }
  for (int k = 0; k < m - 1; ++k) g = std::max(g, std::min(2 * p.rout[k], p.beta[k + 1]));
  if (diff) {
    for (int k = 1; k < m; ++k) g = std::max(g, 2 * p.beta[k + 1]);
    for (int k = 0; k < m - 1; ++k) g = std::max(g, 2 * p.rout[k]);
  }
  if (refine) {
    // fitting sweep: the pair (k, k+1) matrix is (2 r_k) x (2 beta_(k+2)), so
    // the output bonds may exceed the zip-up bonds; buffers use zc >= chi_max
    p.rout[0] = 1;
    for (int k = 0; k < m - 1; ++k) p.rout[k + 1] = std::max(1, std::min({chi_max, 2 * p.rout[k], 2 * p.beta[k + 2]}));
    p.rout[m] = 1;
    for (int k = 0; k < m - 1; ++k) g = std::max(g, std::min(2 * p.rout[k], 2 * p.beta[k + 2]));
    p.zc = std::max(p.zc, *std::max_element(p.rout.begin(), p.rout.end()));
  }
  p.gram_nb = g;
  p.rmax = *std::max_element(p.rin.begin(), p.rin.end());
  p.dmax = *std::max_element(p.D.begin(), p.D.end());
  return p;
}

struct ApplyBufs {
  int* status;
  int* inb;        // sanitised copy of the input bonds, nf x (m+1)
  int* zbonds;     // zip bonds, nf x (m+1)
  void* Z;         // zip cores [m][zc][2][zc] per field
  void* carry[2];  // [a][b][w]: rmax x zc x dmax per field
  void* X;         // [a][b][s][w]
  void* Mb;        // [a][w][b][t]
  void* V1;        // eigenvector copies [n][zc]
  void* V2;
  void* center[2]; // [r][t][b] with strides (2 zc, zc)
  void* R;         // [i][b] ld zc
  double* G;
  double* part;
  void* eigws;
  // fitting sweep (refine) only
  void* Renv;      // right environments: slot j (sites j..m-1) at j * nf * sC, carry layout
  void* Y;         // [b][w][a'][s] strides (dmax rmax 2, rmax 2, 2, 1)
  void* LX;        // [b][t][a'][w'] strides (2 rmax D', rmax D', D', 1)
  void* Th;        // pair matrix [(b, t1)][(beta'', t2)], row stride 2 zc
  void* Lenv[2];   // left environments [b][w][a] strides (dmax rmax, rmax, 1)
  // per-field strides (complex elements)
  ll sZ, sC, sX, sV, sCtr, sR, sY, sTh, sL;
};

ApplyBufs carve_apply(Carver& cv, const ApplyPlan& p, size_t csz, int nf) {
  ApplyBufs b;
  const size_t zc = p.zc;
  size_t nmax = std::max<size_t>(p.gram_nb, 1);
  b.sZ = (ll)p.m * zc * 2 * zc;
  b.sC = (ll)p.rmax * zc * p.dmax;
  b.sX = (ll)p.rmax * zc * 2 * p.dmax;
  b.sV = (ll)nmax * zc;
  b.sCtr = (ll)zc * 2 * zc;
  b.sR = (ll)zc * zc;
  b.status = (int*)cv.take(256);
  b.inb = (int*)cv.take((size_t)nf * (p.m + 1) * sizeof(int));
  b.zbonds = (int*)cv.take((size_t)nf * (p.m + 1) * sizeof(int));
  b.Z = cv.take(nf * b.sZ * csz);
  b.carry[0] = cv.take(nf * b.sC * csz);
  b.carry[1] = cv.take(nf * b.sC * csz);
  b.X = cv.take(nf * b.sX * csz);
  b.Mb = cv.take(nf * b.sX * csz);
  b.V1 = cv.take(nf * b.sV * csz);
  b.V2 = cv.take(nf * b.sV * csz);
  b.center[0] = cv.take(nf * b.sCtr * csz);
  b.center[1] = cv.take(nf * b.sCtr * csz);
  b.R = cv.take(nf * b.sR * csz);
  b.G = (double*)cv.take((size_t)nf * nmax * nmax * 16);
  b.part = (double*)cv.take(std::min<size_t>(PART_BYTES, 256 * nmax * nmax * 16 * (size_t)nf));
  // an application that keeps state computes every eigenpair of each Gram matrix
  b.eigws = cv.take(eig_ws_bytes((int)nmax, p.diff ? (int)nmax : std::max(p.chi_zip, p.chi_max), nf));
  b.sY = (ll)zc * p.dmax * p.rmax * 2;
  b.sTh = (ll)2 * zc * 2 * zc;
  b.sL = (ll)zc * p.dmax * p.rmax;
  b.Renv = b.Y = b.LX = b.Th = b.Lenv[0] = b.Lenv[1] = nullptr;
  if (p.refine) {
    b.Renv = cv.take((size_t)(p.m + 1) * nf * b.sC * csz);
    b.Y = cv.take(nf * b.sY * csz);
    b.LX = cv.take(nf * b.sY * csz);
    b.Th = cv.take(nf * b.sTh * csz);
    b.Lenv[0] = cv.take(nf * b.sL * csz);
    b.Lenv[1] = cv.take(nf * b.sL * csz);
  }
  return b;
}

// Largest eigenproblem of the adjoint: the Gram sides of every truncation.
int bwd_nmax(const ApplyPlan& p) {
  int g = 1;
  for (int k = 1; k < p.m; ++k) g = std::max(g, 2 * p.beta[k + 1]);
  for (int k = 0; k < p.m - 1; ++k) g = std::max(g, 2 * p.rout[k]);
  return g;
}

// What a forward application keeps for its adjoint (caller-owned `saved`
// buffer): the bonds it chose, the zip-up cores, the carry entering every
// zip-up site and its site matrix M, the centre entering every sweep step,
// and the full eigen-decomposition of every truncation's Gram matrix (all n eigenvectors,
// [p][i] with leading dimension L, in the working precision, and the n
// eigenvalues in FP64), computed once by the forward beside its keep rule, so
// that the adjoint differentiates the very factorisation the forward
// truncated with and runs no eigensolver of its own.  Slot k of the carries
// and centres holds all fields (field stride as in the workspace);
// decomposition slot k is zip-up site k, slot m + k sweep step k.
struct SavedBufs {
  int* inb;
  int* zbonds;
  void* Z;
  void* C;
  void* N;
  void* V;
  double* lam;
  void* M;
  ll sZ, sC, sCtr, sX;
  int L, nf;
  size_t csz;
  void* vslot(int j) const { return (char*)V + (size_t)j * nf * L * L * csz; }
  void* mslot(int k) const { return (char*)M + (size_t)k * nf * sX * csz; }
  double* lslot(int j) const { return lam + (size_t)j * nf * L; }
};

SavedBufs carve_saved(Carver& cv, const ApplyPlan& p, size_t csz, int nf) {
  Carver dry(nullptr);
  ApplyBufs t = carve_apply(dry, p, csz, nf);
  SavedBufs v;
  v.sZ = t.sZ; v.sC = t.sC; v.sCtr = t.sCtr; v.sX = t.sX;
  v.L = bwd_nmax(p);
  v.nf = nf;
  v.csz = csz;
  v.inb = (int*)cv.take((size_t)nf * (p.m + 1) * sizeof(int));
  v.zbonds = (int*)cv.take((size_t)nf * (p.m + 1) * sizeof(int));
  v.Z = cv.take(nf * v.sZ * csz);
  v.C = cv.take((size_t)p.m * nf * v.sC * csz);
  v.N = cv.take((size_t)p.m * nf * v.sCtr * csz);
  v.V = cv.take((size_t)2 * p.m * nf * v.L * v.L * csz);
  v.lam = (double*)cv.take((size_t)2 * p.m * nf * v.L * sizeof(double));
  v.M = cv.take((size_t)p.m * nf * v.sX * csz);
  return v;
}

size_t saved_bytes(const ApplyPlan& p, size_t csz, int nf) {
  Carver cv(nullptr);
  carve_saved(cv, p, csz, nf);
  return cv.off;
}

// Internal batched views (a single MPS is a batch of one).
struct MpsB {
  int nf, m, cap, dtype;
  void* cores;
  int* bonds;
  double* norms;
  ll fstride() const { return (ll)m * cap * 2 * cap; }
};
struct MpoB {
  int nf, m, dcap, dtype;
  const void* cores;
  const int* dbonds;
  const int* kind;
  ll fstride() const { return (ll)m * dcap * 4 * dcap; }
};

int check_mps(const qtt_mps* a, const char* name) {
  if (!a) return fail(QTT_ERR_ARG, "%s is NULL", name);
  if (!a->cores || !a->bonds) return fail(QTT_ERR_ARG, "%s has NULL cores/bonds", name);
  if (a->n_sites < 2 || (a->n_sites & 1)) return fail(QTT_ERR_SHAPE, "%s: n_sites must be even and >= 2", name);
  if (a->chi_cap < 1 || a->chi_cap > 256) return fail(QTT_ERR_CAPACITY, "%s: chi_cap must be in [1, 256]", name);
  if (a->dtype != QTT_C64 && a->dtype != QTT_C128) return fail(QTT_ERR_DTYPE, "%s: dtype must be C64 or C128", name);
  return QTT_OK;
}

int check_mpsb(const qtt_mps_batch* a, const char* name) {
  if (!a) return fail(QTT_ERR_ARG, "%s is NULL", name);
  if (a->count < 1 || a->count > 4096) return fail(QTT_ERR_ARG, "%s: count %d outside [1, 4096]", name, a->count);
  qtt_mps one;
  one.n_sites = a->n_sites; one.chi_cap = a->chi_cap; one.dtype = a->dtype;
  one.cores = a->cores; one.bonds = a->bonds; one.norm = a->norms;
  return check_mps(&one, name);
}

MpsB view(const qtt_mps* a) {
  MpsB v;
  v.nf = 1; v.m = a->n_sites; v.cap = a->chi_cap; v.dtype = a->dtype;
  v.cores = a->cores; v.bonds = a->bonds; v.norms = a->norm;
  return v;
}
MpsB view(const qtt_mps_batch* a) {
  MpsB v;
  v.nf = a->count; v.m = a->n_sites; v.cap = a->chi_cap; v.dtype = a->dtype;
  v.cores = a->cores; v.bonds = a->bonds; v.norms = a->norms;
  return v;
}

void opts_defaults(const qtt_opts* o, int cap, qtt_opts& out) {
  if (o) out = *o;
  else { out.chi_max = cap; out.chi_zip = 0; out.cutoff = 0.0; out.tau = 0.0; out.prec = QTT_PREC_FP32; out.refine = 0; }
  if (out.chi_zip <= 0) out.chi_zip = out.chi_max;
  if (!(out.tau > 0.0)) out.tau = 1e-13;
}

Ctx make_ctx(hipStream_t s, int real, int nf, int m, int* status) {
  Ctx c;
  c.s = s; c.real = real;
  c.gemm_t = real ? GEMM_F64 : GEMM_F32;
  c.gram_t = real ? GEMM_F64 : GEMM_F32_GRAM64;
  c.csz = real ? 16 : 8;
  c.nf = nf;
  c.bs = m + 1;
  c.status = status;
  return c;
}

// ------------------------------------------------------------ zip-up + sweep
int run_apply(const MpsB& in, const MpoB& W, const qtt_opts& o, const MpsB& out, const ApplyPlan& p, ApplyBufs& b,
              const int* chi_dev, const SavedBufs* sv, hipStream_t s) {
  if (sv) {                      // keep bonds and zip cores in the saved buffer
    b.inb = sv->inb;
    b.zbonds = sv->zbonds;
    b.Z = sv->Z;
  }
  const int m = p.m, nf = in.nf;
  const int real = in.dtype == QTT_C128 ? 1 : 0;
  Ctx c = make_ctx(s, real, nf, m, b.status);
  if (o.prec == QTT_PREC_BF16) c.gemm_t = GEMM_BF16;
  if (o.prec == QTT_PREC_BF16X3) c.gemm_t = GEMM_BF16X3;
  c.G = b.G; c.gld = std::max(p.gram_nb, 1); c.part = b.part; c.eigws = b.eigws;
  c.eig_nb = c.gld; c.eig_kc = p.diff ? c.gld : std::max(p.chi_zip, p.chi_max);
  const ll ci = in.cap, co = out.cap, zc = p.zc;
  const size_t csz = c.csz;
  const ll sIn = in.fstride(), sOut = out.fstride(), sW = W.fstride();
  char* inc = (char*)in.cores;
  char* outc = (char*)out.cores;
  char* Zc = (char*)b.Z;
  const char* Wc = (const char*)W.cores;
  auto core_in = [&](int k) { return inc + (size_t)k * ci * 2 * ci * csz; };
  auto core_out = [&](int k) { return outc + (size_t)k * co * 2 * co * csz; };
  auto core_z = [&](int k) { return Zc + (size_t)k * zc * 2 * zc * csz; };
  const ll dcap = p.dcap;
  const int bs = c.bs;
  // carry entering zip-up site k; centre entering sweep step k (k >= 1)
  auto carry_at = [&](int k) -> void* {
    return sv ? (char*)sv->C + (size_t)k * nf * b.sC * csz : b.carry[(m - 1 - k) & 1];
  };
  auto center_at = [&](int k) -> void* {
    return sv ? (char*)sv->N + (size_t)k * nf * b.sCtr * csz : b.center[(k - 1) & 1];
  };

  HIPCHK(sanitize_bonds(in.bonds, b.inb, m, (int)ci, b.status, nf, s, p.free_in));
  HIPCHK(set_ints(b.zbonds, nf * bs, 1, s));
  c.kcap_dev = chi_dev;          // per-field caps lower both the zip-up and the sweep caps
  HIPCHK(set_one_b(carry_at(m - 1), b.sC, real, nf, s));
  // ---- zip-up, right to left
  for (int k = m - 1; k >= 0; --k) {
    const int* ra = b.inb + k;
    const int* rb = b.inb + k + 1;
    const int* bet = b.zbonds + k + 1;
    const int Da = p.D[k], Db = p.D[k + 1];
    const bool ident = p.kind[k] == 1;
    void* carry = carry_at(k);
    void* carry_next = k > 0 ? carry_at(k - 1) : nullptr;
    // the site matrix M: in the saved buffer when the adjoint will need it
    void* Mb = sv ? sv->mslot(k) : b.Mb;
    // GEMM1: X[(a,s),(b,w)] = A_k[(a,s), a'] C[a', (b,w)]
    {
      Operand A = opd(core_in(k), 2 * ci, ci, 1, 0, 0, sIn);
      Operand B = opd(carry, zc * Db, 0, Db, 1, 0, b.sC);
      Operand C = ident ? opd(Mb, 2 * zc * Db, 1, 2, 2 * zc, 0, b.sX) : opd(b.X, zc * 2 * Db, Db, 2 * Db, 1, 0, b.sX);
      int r = gemm(c, dv(c, 2, ra), 2, 2 * p.rin[k], dv(c, Db, bet), Db, Db * p.beta[k + 1], dv(c, 1, rb), 1, A, B, C);
      if (r) return r;
    }
    if (p.kind[k] == 2) {
      // diagonal site (W[w'][t][s][w] = 0 for t != s): per output bit t,
      // M[a][w'][b][t] = sum_w X[a][b][t][w] W[w'][t][t][w] -- half the depth
      // of the general product, no reads of the zero blocks
      const char* Wk = Wc + (size_t)k * dcap * 4 * dcap * csz;
      for (int t = 0; t < 2; ++t) {
        Operand A = opd((const char*)b.X + (size_t)t * Db * csz, 2 * Db, 0, 1, 0, 0, b.sX, zc * 2 * Db);
        Operand B = opd(Wk + (size_t)3 * t * Db * csz, 1, 0, 4 * Db, 0, 0, sW);
        Operand C = opd((char*)Mb + (size_t)t * csz, 2, 0, 2 * zc, 0, 0, b.sX, (ll)Da * zc * 2);
        int r = gemm(c, dv(c, 1, bet), 1, p.beta[k + 1], dx(Da), 1, Da, dx(Db), 1, A, B, C, dv(c, 1, ra), p.rin[k]);
        if (r) return r;
      }
    } else if (!ident) {
      // GEMM2 (inner batch over a): M[a][w'][b][t] = sum_{s,w} X[a][b][s][w] W[w'][t][s][w]
      Operand A = opd(b.X, 2 * Db, 0, 1, 0, 0, b.sX, zc * 2 * Db);
      Operand B = opd(Wc + (size_t)k * dcap * 4 * dcap * csz, 1, 0, 4 * Db, 2 * Db, 0, sW);
      Operand C = opd(Mb, 2, 0, 2 * zc, 1, 0, b.sX, (ll)Da * zc * 2);
      int r = gemm(c, dv(c, 1, bet), 1, p.beta[k + 1], dx(2 * Da), 2, 2 * Da, dx(2 * Db), 1, A, B, C, dv(c, 1, ra),
                   p.rin[k]);
      if (r) return r;
    }
    // M_k = [(a, w'), (b, t)]: rows p = a*Da + w' (strides 2 zc Da, 2 zc), cols q = 2b + t (stride 1)
    if (k == 0) {
      // one row: B_0[0][t][b] = M[0][0][b][t]
      HIPCHK(block_copy_b(Mb, 2, 1, b.sX, core_z(0), 1, zc, b.sZ, dv(c, 1, bet), dx(2), p.beta[1], 2, real, nf, s));
      break;
    }
    const ll pb = (ll)p.rin[k] * Da, qb = 2ll * p.beta[k + 1];
    int* kout = b.zbonds + k;
    // a forward that keeps state for its adjoint factors on the side the
    // adjoint differentiates (M^H M here), so that both see the same Gram
    // matrix and the same kept eigenvectors bit for bit; the other side would
    // rebuild V_k as U^H M / sigma, whose small-sigma directions carry the
    // FP32 error of M divided by sigma
    if (qb <= pb || sv) {
      // column side: G = M^H M (q x q); with saved state the full
      // decomposition goes to the saved slot of this site beside the kept part
      Operand A = opd(Mb, 1, 0, 2 * zc * Da, 2 * zc, 1, b.sX);
      Operand B = opd(Mb, 2 * zc * Da, 2 * zc, 1, 0, 0, b.sX);
      int r = gram(c, A, B, dv(c, 2, bet), 1, (int)qb, dv(c, Da, ra), Da, pb);
      if (r) return r;
      const EigEmit eV = emit(b.V1, 1, zc, 0, 1, 0, 0, real, b.sV);              // V [q][i]
      const EigEmit eB = emit(core_z(k), 2, 1, zc, 2 * zc, 1, 0, real, b.sZ);   // B_k[i][t][b] = conj V[(b,t)][i]
      if (sv) {
        const ll L = sv->L;
        FullOut fo;
        fo.lam = sv->lslot(k); fo.lam_ld = L; fo.keep_cap = p.beta[k];
        r = eig(c, dv(c, 2, bet), (int)qb, (int)qb, o.cutoff, o.tau, kout,
                {eV, eB, emit(sv->vslot(k), 1, L, 0, 1, 0, 0, real, L * L, 1)}, nullptr, fo);
      } else {
        r = eig(c, dv(c, 2, bet), (int)qb, p.beta[k], o.cutoff, o.tau, kout, {eV, eB});
      }
      if (r) return r;
      // carry_next[a][i][w'] = sum_q M[(a,w')][q] V[q][i]
      Operand A2 = opd(Mb, 2 * zc * Da, 2 * zc, 1, 0, 0, b.sX);
      Operand B2 = opd(b.V1, zc, 0, 1, 0, 0, b.sV);
      Operand C2 = opd(carry_next, zc * Da, 1, Da, 0, 0, b.sC);
      r = gemm(c, dv(c, Da, ra), Da, (int)pb, dv(c, 1, kout), 1, p.beta[k], dv(c, 2, bet), 1, A2, B2, C2);
      if (r) return r;
    } else {
      // row side: G = M M^H (p x p)
      Operand A = opd(Mb, 2 * zc * Da, 2 * zc, 1, 0, 0, b.sX);
      Operand B = opd(Mb, 1, 0, 2 * zc * Da, 2 * zc, 1, b.sX);
      int r = gram(c, A, B, dv(c, Da, ra), Da, (int)pb, dv(c, 2, bet), 1, qb);
      if (r) return r;
      r = eig(c, dv(c, Da, ra), (int)pb, p.beta[k], o.cutoff, o.tau, kout,
              {emit(carry_next, Da, zc * Da, 1, Da, 0, 1, real, b.sC),         // carry = U sigma
               emit(b.V1, 1, zc, 0, 1, 0, -1, real, b.sV)});                   // U / sigma [p][i]
      if (r) return r;
      // B_k[i][t][b] = sum_p conj(U/sigma)[p][i] M[p][(b,t)]
      Operand A2 = opd(b.V1, 1, 0, (ll)Da * zc, zc, 1, b.sV);     // K index p = (a, w') of a plain [p][i] matrix
      Operand B2 = opd(Mb, 2 * zc * Da, 2 * zc, 2, 1, 0, b.sX);
      Operand C2 = opd(core_z(k), 2 * zc, 0, 1, zc, 0, b.sZ);
      r = gemm(c, dv(c, 1, kout), 1, p.beta[k], dv(c, 2, bet), 2, (int)qb, dv(c, Da, ra), Da, A2, B2, C2);
      if (r) return r;
    }
  }
  if (p.refine) {
    // ---- one two-site fitting sweep (left to right) against W . in, with
    // FP32 (or FP64) contractions whatever the zip-up precision was.  The
    // initial state is the right-canonical zip-up output Z.
    c.gemm_t = real ? GEMM_F64 : GEMM_F32;
    const ll rmax = p.rmax, dmax = p.dmax;
    auto env_at = [&](int j) { return (char*)b.Renv + (size_t)j * nf * b.sC * csz; };
    // M[a][w'][beta][t] of site j with right environment `env` (the zip-up's
    // first two contractions); identity sites write M directly
    auto make_M = [&](int j, const void* env, const int* bet) -> int {
      const int* ra = b.inb + j;
      const int* rb = b.inb + j + 1;
      const int Da = p.D[j], Db = p.D[j + 1];
      const bool ident = p.kind[j] == 1;
      Operand A = opd(core_in(j), 2 * ci, ci, 1, 0, 0, sIn);
      Operand B = opd(env, zc * Db, 0, Db, 1, 0, b.sC);
      Operand C = ident ? opd(b.Mb, 2 * zc * Db, 1, 2, 2 * zc, 0, b.sX) : opd(b.X, zc * 2 * Db, Db, 2 * Db, 1, 0, b.sX);
      int r = gemm(c, dv(c, 2, ra), 2, 2 * p.rin[j], dv(c, Db, bet), Db, Db * p.beta[j + 1], dv(c, 1, rb), 1, A, B, C);
      if (r || ident) return r;
      return gemm(c, dv(c, 1, bet), 1, p.beta[j + 1], dx(2 * Da), 2, 2 * Da, dx(2 * Db), 1,
                  opd(b.X, 2 * Db, 0, 1, 0, 0, b.sX, zc * 2 * Db),
                  opd(Wc + (size_t)j * dcap * 4 * dcap * csz, 1, 0, 4 * Db, 2 * Db, 0, sW),
                  opd(b.Mb, 2, 0, 2 * zc, 1, 0, b.sX, (ll)Da * zc * 2), dv(c, 1, ra), p.rin[j]);
    };
    // right environments of Z in full precision: env_j = M_j Z_j^H
    HIPCHK(set_one_b(env_at(m), b.sC, real, nf, s));
    for (int j = m - 1; j >= 2; --j) {
      const int Da = p.D[j];
      int r = make_M(j, env_at(j + 1), b.zbonds + j + 1);
      if (r) return r;
      r = gemm(c, dv(c, Da, b.inb + j), Da, p.rin[j] * Da, dv(c, 1, b.zbonds + j), 1, p.beta[j],
               dv(c, 2, b.zbonds + j + 1), 2, opd(b.Mb, 2 * zc * Da, 2 * zc, 2, 1, 0, b.sX),
               opd(core_z(j), 1, zc, 2 * zc, 0, 1, b.sZ), opd(env_at(j), zc * Da, 1, Da, 0, 0, b.sC));
      if (r) return r;
    }
    HIPCHK(set_ints_strided(out.bonds, 1, bs, nf, 1, s));
    HIPCHK(set_ints_strided(out.bonds + m, 1, bs, nf, 1, s));
    HIPCHK(set_one_b(b.Lenv[0], b.sL, real, nf, s));
    int ls = 0;
    for (int k = 0; k < m - 1; ++k) {
      const int* rk = out.bonds + k;
      int* kout = out.bonds + k + 1;
      const int Dk = p.D[k], D1 = p.D[k + 1];
      const bool ident = p.kind[k] == 1;
      const void* Lk = b.Lenv[ls];
      // Y[b][w][a'][s] = sum_a L[b][w][a] A_k[a][s][a']
      int r = gemm(c, dv(c, Dk, rk), Dk, p.rout[k] * Dk, dv(c, 2, b.inb + k + 1), 2, 2 * p.rin[k + 1],
                   dv(c, 1, b.inb + k), 1, opd(Lk, dmax * rmax, rmax, 1, 0, 0, b.sL),
                   opd(core_in(k), 2 * ci, 0, 1, ci, 0, sIn), opd(b.Y, dmax * rmax * 2, rmax * 2, 2, 1, 0, b.sY));
      if (r) return r;
      // LX[b][t][a'][w'] = sum_{w, s} Y[b][w][a'][s] W_k[w][t][s][w']  (identity site: a view of Y)
      Operand LXrows;    // rows (b, t) split lo 2, columns (a', w') split lo D1
      if (ident) {
        LXrows = opd(b.Y, dmax * rmax * 2, 1, 2, rmax * 2, 0, b.sY);
      } else {
        r = gemm(c, dv(c, 1, b.inb + k + 1), 1, p.rin[k + 1], dx(2 * D1), D1, 2 * D1, dx(2 * Dk), 2,
                 opd(b.Y, 2, 0, rmax * 2, 1, 0, b.sY, dmax * rmax * 2),
                 opd(Wc + (size_t)k * dcap * 4 * dcap * csz, 4 * D1, D1, 2 * D1, 1, 0, sW),
                 opd(b.LX, D1, 0, rmax * D1, 1, 0, b.sY, 2 * rmax * D1), dv(c, 1, rk), p.rout[k]);
        if (r) return r;
        LXrows = opd(b.LX, 2 * rmax * D1, rmax * D1, D1, 1, 0, b.sY);
      }
      // right part of the pair: M_(k+1)[a'][w'][beta''][t2] with env_(k+2)
      r = make_M(k + 1, env_at(k + 2), b.zbonds + k + 2);
      if (r) return r;
      // Theta[(b, t1)][(beta'', t2)] = LX[(b, t1)][(a', w')] M[(a', w')][(beta'', t2)]
      const int* bq = b.zbonds + k + 2;
      const ll pb = 2ll * p.rout[k], qb = 2ll * p.beta[k + 2];
      r = gemm(c, dv(c, 2, rk), 2, (int)pb, dv(c, 2, bq), 1, (int)qb, dv(c, D1, b.inb + k + 1), D1, LXrows,
               opd(b.Mb, 2 * zc * D1, 2 * zc, 1, 0, 0, b.sX), opd(b.Th, 4 * zc, 2 * zc, 1, 0, 0, b.sTh));
      if (r) return r;
      const Operand Th_rows = opd(b.Th, 4 * zc, 2 * zc, 1, 0, 0, b.sTh);    // [(b, t1)][q]
      const Operand U_out = opd(core_out(k), 2 * co, co, 1, 0, 0, sOut);     // [(b, t1)][i]
      if (qb < pb) {
        r = gram(c, opd(b.Th, 1, 0, 4 * zc, 2 * zc, 1, b.sTh), Th_rows, dv(c, 2, bq), 1, (int)qb, dv(c, 2, rk), 2, pb);
        if (r) return r;
        r = eig(c, dv(c, 2, bq), (int)qb, p.rout[k + 1], o.cutoff, o.tau, kout,
                {emit(b.V1, 1, zc, 0, 1, 0, -1, real, b.sV)});                  // V / sigma
        if (r) return r;
        r = gemm(c, dv(c, 2, rk), 2, (int)pb, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, 2, bq), 1, Th_rows,
                 opd(b.V1, zc, 0, 1, 0, 0, b.sV), U_out);
        if (r) return r;
      } else {
        r = gram(c, Th_rows, opd(b.Th, 1, 0, 4 * zc, 2 * zc, 1, b.sTh), dv(c, 2, rk), 2, (int)pb, dv(c, 2, bq), 1, qb);
        if (r) return r;
        r = eig(c, dv(c, 2, rk), (int)pb, p.rout[k + 1], o.cutoff, o.tau, kout,
                {emit(core_out(k), 2, 2 * co, co, 1, 0, 0, real, sOut)});       // U
        if (r) return r;
      }
      const Operand Uh = opd(core_out(k), 1, 0, 2 * co, co, 1, sOut);          // [i][(b, t1)] conjugated
      if (k == m - 2) {
        // last core [i][t2][0] = U^H Theta
        r = gemm(c, dv(c, 1, kout), 1, p.rout[k + 1], dx(2), 1, 2, dv(c, 2, rk), 2, Uh, Th_rows,
                 opd(core_out(m - 1), 2 * co, 0, co, 0, 0, sOut));
        if (r) return r;
      } else {
        // L_(k+1)[i][w'][a'] = sum_(b, t1) conj(U)[(b, t1)][i] LX[(b, t1)][(a', w')]
        r = gemm(c, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, D1, b.inb + k + 1), D1, p.rin[k + 1] * D1,
                 dv(c, 2, rk), 2, Uh, LXrows, opd(b.Lenv[ls ^ 1], dmax * rmax, 0, 1, rmax, 0, b.sL));
        if (r) return r;
        ls ^= 1;
      }
    }
    const int* rl = out.bonds + m - 1;
    if (out.norms)
      HIPCHK(block_norm_b(core_out(m - 1), real, dv(c, 1, rl), dx(2), p.rout[m - 1], 2, 2 * co, co, sOut, out.norms,
                          nf, s));
    return QTT_OK;
  }
  // ---- sweep, left to right
  HIPCHK(set_ints_strided(out.bonds, 1, bs, nf, 1, s));
  HIPCHK(set_ints_strided(out.bonds + m, 1, bs, nf, 1, s));
  const char* center = core_z(0);
  ll sCenter = b.sZ;
  c.kcap_dev = chi_dev;
  for (int k = 0; k < m - 1; ++k) {
    const int* rk = out.bonds + k;
    const int* bk = b.zbonds + k + 1;
    const int* bk2 = b.zbonds + k + 2;
    int* kout = out.bonds + k + 1;
    const ll pb = 2ll * p.rout[k], qb = p.beta[k + 1];
    void* next = center_at(k + 1);
    const char* znext = core_z(k + 1);
    // M = center [(r,t), b]: strides (2 zc, zc) rows, 1 cols.  With saved
    // state the row side (M M^H), the factorisation the adjoint differentiates
    if (qb < pb && !sv) {
      Operand A = opd(center, 1, 0, 2 * zc, zc, 1, sCenter);
      Operand B = opd(center, 2 * zc, zc, 1, 0, 0, sCenter);
      int r = gram(c, A, B, dv(c, 1, bk), 1, (int)qb, dv(c, 2, rk), 2, pb);
      if (r) return r;
      r = eig(c, dv(c, 1, bk), (int)qb, p.rout[k + 1], o.cutoff, o.tau, kout,
              {emit(b.V1, 1, zc, 0, 1, 0, -1, real, b.sV),     // V / sigma
               emit(b.V2, 1, zc, 0, 1, 0, 1, real, b.sV)});    // V * sigma
      if (r) return r;
      // out core k [(r,t)][i] = M V/sigma
      r = gemm(c, dv(c, 2, rk), 2, (int)pb, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, 1, bk), 1,
               opd(center, 2 * zc, zc, 1, 0, 0, sCenter), opd(b.V1, zc, 0, 1, 0, 0, b.sV),
               opd(core_out(k), 2 * co, co, 1, 0, 0, sOut));
      if (r) return r;
      // next [i][t][b''] = sum_b sigma_i conj(V[b][i]) Z_{k+1}[b][t][b'']
      r = gemm(c, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, 2, bk2), 2, 2 * p.beta[k + 2], dv(c, 1, bk), 1,
               opd(b.V2, 1, 0, zc, 0, 1, b.sV), opd(znext, 2 * zc, 0, 1, zc, 0, b.sZ),
               opd(next, 2 * zc, 0, 1, zc, 0, b.sCtr));
      if (r) return r;
    } else {
      Operand A = opd(center, 2 * zc, zc, 1, 0, 0, sCenter);
      Operand B = opd(center, 1, 0, 2 * zc, zc, 1, sCenter);
      int r = gram(c, A, B, dv(c, 2, rk), 2, (int)pb, dv(c, 1, bk), 1, qb);
      if (r) return r;
      const EigEmit eU = emit(core_out(k), 2, 2 * co, co, 1, 0, 0, real, sOut);   // out core k = U
      const EigEmit eV1 = emit(b.V1, 1, zc, 0, 1, 0, 0, real, b.sV);             // U [p][i]
      if (sv) {
        const ll L = sv->L;
        FullOut fo;
        fo.lam = sv->lslot(m + k); fo.lam_ld = L; fo.keep_cap = p.rout[k + 1];
        r = eig(c, dv(c, 2, rk), (int)pb, (int)pb, o.cutoff, o.tau, kout,
                {eU, eV1, emit(sv->vslot(m + k), 1, L, 0, 1, 0, 0, real, L * L, 1)}, nullptr, fo);
      } else {
        r = eig(c, dv(c, 2, rk), (int)pb, p.rout[k + 1], o.cutoff, o.tau, kout, {eU, eV1});
      }
      if (r) return r;
      // R[i][b] = sum_p conj(U[p][i]) M[p][b]
      r = gemm(c, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, 1, bk), 1, (int)qb, dv(c, 2, rk), 2,
               opd(b.V1, 1, 0, 2 * zc, zc, 1, b.sV), opd(center, 2 * zc, zc, 1, 0, 0, sCenter),
               opd(b.R, zc, 0, 1, 0, 0, b.sR));
      if (r) return r;
      r = gemm(c, dv(c, 1, kout), 1, p.rout[k + 1], dv(c, 2, bk2), 2, 2 * p.beta[k + 2], dv(c, 1, bk), 1,
               opd(b.R, zc, 0, 1, 0, 0, b.sR), opd(znext, 2 * zc, 0, 1, zc, 0, b.sZ),
               opd(next, 2 * zc, 0, 1, zc, 0, b.sCtr));
      if (r) return r;
    }
    center = (const char*)next;
    sCenter = b.sCtr;
  }
  // last core: out[m-1][r][t][0] = center[r][t][0]
  const int* rl = out.bonds + m - 1;
  HIPCHK(block_copy_b(center, 2 * zc, zc, sCenter, core_out(m - 1), 2 * co, co, sOut, dv(c, 1, rl), dx(2),
                      p.rout[m - 1], 2, real, nf, s));
  if (out.norms)
    HIPCHK(block_norm_b(core_out(m - 1), real, dv(c, 1, rl), dx(2), p.rout[m - 1], 2, 2 * co, co, sOut, out.norms,
                        nf, s));
  return QTT_OK;
}

size_t apply_bytes(const ApplyPlan& p, size_t csz, int nf) {
  Carver cv(nullptr);
  carve_apply(cv, p, csz, nf);
  return cv.off;
}

// Validated arguments of one (batched) application.
struct ApplySetup {
  qtt_opts o;
  std::vector<int> dbonds, kind;
  MpoB W;
  ApplyPlan p;
  size_t csz;
};

// Validate the arguments of an application.  identity: W ignored, every site
// an identity pass-through of bond 1 (used by tt_truncate).
int apply_setup(const MpsB& in, const qtt_mpo* W1, const MpoB* Wb, const qtt_opts* opts, const MpsB& out,
                bool identity, ApplySetup& su, bool diff = false) {
  if (in.m != out.m) return fail(QTT_ERR_SHAPE, "in/out n_sites differ");
  if (in.nf != out.nf) return fail(QTT_ERR_SHAPE, "in/out batch counts differ");
  if (in.dtype != out.dtype) return fail(QTT_ERR_DTYPE, "in/out dtypes differ");
  const int m = in.m;
  qtt_opts& o = su.o;
  opts_defaults(opts, out.cap, o);
  if (o.chi_max < 1 || o.chi_max > out.cap) return fail(QTT_ERR_CAPACITY, "chi_max %d outside [1, %d]", o.chi_max, out.cap);
  if (o.chi_zip < 1 || o.chi_zip > 256) return fail(QTT_ERR_CAPACITY, "chi_zip %d outside [1, 256]", o.chi_zip);
  if (o.prec != QTT_PREC_FP32 && o.prec != QTT_PREC_FP64 && o.prec != QTT_PREC_BF16 && o.prec != QTT_PREC_BF16X3)
    return fail(QTT_ERR_ARG, "precision %d not supported", o.prec);
  if ((o.prec == QTT_PREC_FP64) != (in.dtype == QTT_C128)) return fail(QTT_ERR_DTYPE, "precision and dtype disagree");
  if (o.refine != 0 && o.refine != 1) return fail(QTT_ERR_ARG, "refine must be 0 or 1");
  su.dbonds.assign(m + 1, 1);
  su.kind.assign(m, 1);
  MpoB& W = su.W;
  W.nf = in.nf; W.m = m; W.dcap = 1; W.dtype = in.dtype; W.cores = nullptr;
  if (!identity) {
    const int* db;
    const int* kd;
    int n_sites, dcap, dtype;
    if (W1) {
      if (!W1->cores || !W1->d_bonds) return fail(QTT_ERR_ARG, "MPO is NULL or incomplete");
      n_sites = W1->n_sites; dcap = W1->d_cap; dtype = W1->dtype; db = W1->d_bonds; kd = W1->site_kind;
      W.cores = W1->cores;
      if (in.nf != 1) return fail(QTT_ERR_ARG, "single MPO with a batch");
    } else {
      if (!Wb || !Wb->cores || !Wb->dbonds) return fail(QTT_ERR_ARG, "MPO batch is NULL or incomplete");
      if (Wb->nf != in.nf) return fail(QTT_ERR_SHAPE, "MPO batch count differs from MPS batch count");
      n_sites = Wb->m; dcap = Wb->dcap; dtype = Wb->dtype; db = Wb->dbonds; kd = Wb->kind;
      W.cores = Wb->cores;
    }
    if (n_sites != m) return fail(QTT_ERR_SHAPE, "MPO has %d sites, MPS %d", n_sites, m);
    if (dtype != in.dtype) return fail(QTT_ERR_DTYPE, "MPO dtype differs from MPS dtype");
    if (db[0] != 1 || db[m] != 1) return fail(QTT_ERR_SHAPE, "MPO boundary bonds must be 1");
    if (dcap < 1 || dcap > 512) return fail(QTT_ERR_CAPACITY, "MPO d_cap %d outside [1, 512]", dcap);
    for (int k = 0; k <= m; ++k) {
      if (db[k] < 1 || db[k] > dcap) return fail(QTT_ERR_CAPACITY, "MPO bond %d = %d outside [1, d_cap]", k, db[k]);
      su.dbonds[k] = db[k];
    }
    for (int k = 0; k < m; ++k) {
      su.kind[k] = kd ? kd[k] : 0;
      if (su.kind[k] < 0 || su.kind[k] > 2) return fail(QTT_ERR_ARG, "site_kind[%d] = %d not in {0, 1, 2}", k, su.kind[k]);
      if (su.kind[k] == 1 && su.dbonds[k] != su.dbonds[k + 1])
        return fail(QTT_ERR_SHAPE, "identity site %d changes the bond", k);
    }
    W.dcap = dcap;
  }
  W.dbonds = su.dbonds.data();
  W.kind = su.kind.data();
  su.p = make_apply_plan(m, in.cap, out.cap, o.chi_max, o.chi_zip, su.dbonds.data(), su.kind.data(), W.dcap,
                         identity ? 0 : o.refine, diff ? 1 : 0, identity ? 1 : 0);
  su.csz = in.dtype == QTT_C128 ? 16 : 8;
  return QTT_OK;
}

int apply_common(const MpsB& in, const qtt_mpo* W1, const MpoB* Wb, const qtt_opts* opts, const MpsB& out,
                 const int* chi_dev, void* ws, size_t ws_bytes, void* stream, bool identity, void* saved = nullptr,
                 size_t saved_sz = 0) {
  if (!ws) return fail(QTT_ERR_ARG, "workspace is NULL");
  ApplySetup su;
  int r = apply_setup(in, W1, Wb, opts, out, identity, su, saved != nullptr);
  if (r) return r;
  size_t need = apply_bytes(su.p, su.csz, in.nf);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  SavedBufs sv;
  if (saved && su.p.refine) return fail(QTT_ERR_ARG, "the adjoint covers the plain sweep only (refine = 0)");
  if (saved) {
    size_t sneed = saved_bytes(su.p, su.csz, in.nf);
    if (saved_sz < sneed) return fail(QTT_ERR_WORKSPACE, "saved buffer %zu < required %zu bytes", saved_sz, sneed);
    Carver cs(saved);
    sv = carve_saved(cs, su.p, su.csz, in.nf);
  }
  Carver cw(ws);
  ApplyBufs b = carve_apply(cw, su.p, su.csz, in.nf);
  return run_apply(in, su.W, su.o, out, su.p, b, chi_dev, saved ? &sv : nullptr, (hipStream_t)stream);
}

// ------------------------------------------------------------ adjoint of the application
// Reverse of the sweep (right to left), then of the zip-up (left to right).
// Every truncation M -> (V_k, M V_k) (zip-up: B = V_k^H, carry = M V_k; sweep
// on N^H: U = V_k, R = U^H N) is differentiated with the full FP64 eigen-
// decomposition G = M^H M = V diag(lam) V^H that the forward computed beside
// its keep rule and saved (no eigensolver runs here, and the adjoint sees the
// very factorisation the forward truncated with):
//   Vbar = gV + M^H gC,  Z = F o (V^H Vbar) with F_ji = 1/(lam_i - lam_j) for
//   discarded j and kept i (0 elsewhere),  P = V Z,
//   Mbar = (gC + M P) V_k^H + (M V_k) P^H.
// The kept-kept block is left out: the chain of truncations is invariant
// under unitary rotations of each kept block, so that block contributes
// nothing to the gradient of any function of the final field.
struct BwdBufs {
  int* status;
  void *Mbar, *Xbar;
  void* gC[2];
  void* Zbar;
  void* Nbar[2];
  void *R, *Rbar;
  void *Vbar, *Y, *P;
  ll sX, sC, sZ, sCtr, sR, sE;
  int nmax;
};

BwdBufs carve_bwd(Carver& cv, const ApplyPlan& p, size_t csz, int nf) {
  Carver dry(nullptr);
  ApplyBufs t = carve_apply(dry, p, csz, nf);
  BwdBufs b;
  b.nmax = bwd_nmax(p);
  b.sX = t.sX; b.sC = t.sC; b.sZ = t.sZ; b.sCtr = t.sCtr; b.sR = t.sR;
  b.sE = (ll)b.nmax * b.nmax;
  b.status = (int*)cv.take(256);
  b.Mbar = cv.take(nf * b.sX * csz);
  b.Xbar = cv.take(nf * b.sX * csz);
  b.gC[0] = cv.take(nf * b.sC * csz);
  b.gC[1] = cv.take(nf * b.sC * csz);
  b.Zbar = cv.take(nf * b.sZ * csz);
  b.Nbar[0] = cv.take(nf * b.sCtr * csz);
  b.Nbar[1] = cv.take(nf * b.sCtr * csz);
  b.R = cv.take(nf * b.sR * csz);
  b.Rbar = cv.take(nf * b.sR * csz);
  b.Vbar = cv.take(nf * b.sE * csz);
  b.Y = cv.take(nf * b.sE * csz);
  b.P = cv.take(nf * b.sE * csz);
  return b;
}

size_t bwd_bytes(const ApplyPlan& p, size_t csz, int nf) {
  Carver cv(nullptr);
  carve_bwd(cv, p, csz, nf);
  return cv.off;
}

int run_apply_backward(const MpsB& in, const MpoB& W, const MpsB& out, const MpsB& gout, const MpsB& gin,
                       const ApplyPlan& p, const SavedBufs& sv, BwdBufs& b, hipStream_t s) {
  const int m = p.m, nf = in.nf;
  const int real = in.dtype == QTT_C128 ? 1 : 0;
  Ctx c = make_ctx(s, real, nf, m, b.status);
  c.G = nullptr; c.gld = 0; c.part = nullptr; c.eigws = nullptr;
  c.eig_nb = 0; c.eig_kc = 0;
  c.kcap_dev = nullptr;
  const ll ci = in.cap, co = out.cap, zc = p.zc, L = b.nmax;
  const size_t csz = c.csz;
  const ll sIn = in.fstride(), sOut = out.fstride(), sW = W.fstride();
  const int bs = c.bs;
  auto core_in = [&](int k) { return (char*)in.cores + (size_t)k * ci * 2 * ci * csz; };
  auto core_gin = [&](int k) { return (char*)gin.cores + (size_t)k * ci * 2 * ci * csz; };
  auto core_out = [&](int k) { return (char*)out.cores + (size_t)k * co * 2 * co * csz; };
  auto core_gout = [&](int k) { return (char*)gout.cores + (size_t)k * co * 2 * co * csz; };
  auto core_z = [&](int k) { return (char*)sv.Z + (size_t)k * zc * 2 * zc * csz; };
  auto core_zbar = [&](int k) { return (char*)b.Zbar + (size_t)k * zc * 2 * zc * csz; };
  auto carry_at = [&](int k) { return (char*)sv.C + (size_t)k * nf * b.sC * csz; };
  auto center_at = [&](int k) { return k == 0 ? core_z(0) : (char*)sv.N + (size_t)k * nf * b.sCtr * csz; };
  const char* Wc = (const char*)W.cores;
  const ll dcap = p.dcap;
  int r;

  HIPCHK(zero_fill(gin.cores, (size_t)nf * sIn * csz, s));
  HIPCHK(copy_ints(sv.inb, gin.bonds, nf * bs, s));
  // ---- sweep, reversed.  cbar: gradient of the centre entering step k + 1.
  const char* cbar = core_gout(m - 1);
  ll cbar_rs = 2 * co, cbar_ts = co, sCbar = sOut;
  int nsel = 0;
  for (int k = m - 2; k >= 0; --k) {
    const int* rk = out.bonds + k;
    const int* rk1 = out.bonds + k + 1;
    const int* bk = sv.zbonds + k + 1;
    const int* bk2 = sv.zbonds + k + 2;
    const int nr = 2 * p.rout[k], nr1 = p.rout[k + 1], nbk = p.beta[k + 1], nbk2 = p.beta[k + 2];
    const char* N = center_at(k);
    const ll sN = k == 0 ? b.sZ : b.sCtr;
    const char* U = core_out(k);
    // R = U^H N
    r = gemm(c, dv(c, 1, rk1), 1, nr1, dv(c, 1, bk), 1, nbk, dv(c, 2, rk), 1, opd(U, 1, 0, co, 0, 1, sOut),
             opd(N, zc, 0, 1, 0, 0, sN), opd(b.R, zc, 0, 1, 0, 0, b.sR));
    if (r) return r;
    // Rbar = cbar Z_{k+1}^H   (K = (b'', t))
    r = gemm(c, dv(c, 1, rk1), 1, nr1, dv(c, 1, bk), 1, nbk, dv(c, 2, bk2), 2,
             opd(cbar, cbar_rs, 0, 1, cbar_ts, 0, sCbar), opd(core_z(k + 1), 1, zc, 2 * zc, 0, 1, b.sZ),
             opd(b.Rbar, zc, 0, 1, 0, 0, b.sR));
    if (r) return r;
    // Zbar_{k+1} = R^H cbar
    r = gemm(c, dv(c, 1, bk), 1, nbk, dv(c, 2, bk2), 2, 2 * nbk2, dv(c, 1, rk1), 1, opd(b.R, 1, 0, zc, 0, 1, b.sR),
             opd(cbar, cbar_rs, 0, 1, cbar_ts, 0, sCbar), opd(core_zbar(k + 1), 2 * zc, 0, 1, zc, 0, b.sZ));
    if (r) return r;
    // Vbar = gout_k + N Rbar^H   ([p = (r, t)][i], ld L)
    HIPCHK(block_copy_b(core_gout(k), co, 1, sOut, b.Vbar, L, 1, b.sE, dv(c, 2, rk), dv(c, 1, rk1), nr, nr1, real,
                        nf, s));
    r = gemm(c, dv(c, 2, rk), 1, nr, dv(c, 1, rk1), 1, nr1, dv(c, 1, bk), 1, opd(N, zc, 0, 1, 0, 0, sN),
             opd(b.Rbar, 1, 0, zc, 0, 1, b.sR), opd(b.Vbar, L, 0, 1, 0, 0, b.sE), dx(1), 1, 1);
    if (r) return r;
    // the full decomposition of N N^H the forward computed: Y = Vall^H Vbar,
    // scaled in place to Z; P = Vall Z
    const void* Vall = sv.vslot(m + k);
    r = gemm(c, dv(c, 2, rk), 1, nr, dv(c, 1, rk1), 1, nr1, dv(c, 2, rk), 1, opd(Vall, 1, 0, L, 0, 1, b.sE),
             opd(b.Vbar, L, 0, 1, 0, 0, b.sE), opd(b.Y, L, 0, 1, 0, 0, b.sE));
    if (r) return r;
    HIPCHK(eig_adjoint_scale(dv(c, 2, rk), nr, sv.lslot(m + k), L, nf, b.Y, L, b.sE, rk1, bs, nr1, real, s));
    r = gemm(c, dv(c, 2, rk), 1, nr, dv(c, 1, rk1), 1, nr1, dv(c, 2, rk), 1, opd(Vall, L, 0, 1, 0, 0, b.sE),
             opd(b.Y, L, 0, 1, 0, 0, b.sE), opd(b.P, L, 0, 1, 0, 0, b.sE));
    if (r) return r;
    // Rbar += P^H N;  Nbar = U Rbar + P R
    r = gemm(c, dv(c, 1, rk1), 1, nr1, dv(c, 1, bk), 1, nbk, dv(c, 2, rk), 1, opd(b.P, 1, 0, L, 0, 1, b.sE),
             opd(N, zc, 0, 1, 0, 0, sN), opd(b.Rbar, zc, 0, 1, 0, 0, b.sR), dx(1), 1, 1);
    if (r) return r;
    void* nbar = k == 0 ? (void*)core_zbar(0) : b.Nbar[nsel];
    const ll sNbar = k == 0 ? b.sZ : b.sCtr;
    r = gemm(c, dv(c, 2, rk), 1, nr, dv(c, 1, bk), 1, nbk, dv(c, 1, rk1), 1, opd(U, co, 0, 1, 0, 0, sOut),
             opd(b.Rbar, zc, 0, 1, 0, 0, b.sR), opd(nbar, zc, 0, 1, 0, 0, sNbar));
    if (r) return r;
    r = gemm(c, dv(c, 2, rk), 1, nr, dv(c, 1, bk), 1, nbk, dv(c, 1, rk1), 1, opd(b.P, L, 0, 1, 0, 0, b.sE),
             opd(b.R, zc, 0, 1, 0, 0, b.sR), opd(nbar, zc, 0, 1, 0, 0, sNbar), dx(1), 1, 1);
    if (r) return r;
    cbar = (const char*)nbar;
    cbar_rs = 2 * zc;
    cbar_ts = zc;
    sCbar = sNbar;
    nsel ^= 1;
  }
  // ---- zip-up, reversed (left to right).  gcur: gradient of the carry leaving site k.
  void* gcur = b.gC[0];
  void* gnext = b.gC[1];
  for (int k = 0; k < m; ++k) {
    const int* ra = sv.inb + k;
    const int* rb = sv.inb + k + 1;
    const int* bet = sv.zbonds + k + 1;
    const int* kkp = sv.zbonds + k;
    const int Da = p.D[k], Db = p.D[k + 1];
    const bool ident = p.kind[k] == 1;
    void* Cin = carry_at(k);
    const ll pb = (ll)p.rin[k] * Da, qb = 2ll * p.beta[k + 1];
    // the site matrix M the forward formed (and truncated), from the saved buffer
    const void* Mk = sv.mslot(k);
    const Operand Mrows = opd(Mk, 2 * zc * Da, 2 * zc, 1, 0, 0, b.sX);        // [p = (a, w')][q]
    const Operand Mbar_v = opd(b.Mbar, 2 * zc * Da, 2 * zc, 2, 1, 0, b.sX);   // [p][q = (b, t)], N split lo 2
    if (k == 0) {
      // M[0][0][b][t] = B_0[0][t][b]
      HIPCHK(block_copy_b(core_zbar(0), zc, 1, b.sZ, b.Mbar, 1, 2, b.sX, dx(2), dv(c, 1, bet), 2, p.beta[1], real, nf,
                          s));
    } else {
      // Vbar[q = 2b + t][i] = conj(Zbar_k[i][t][b]) + (M^H gC)[q][i]
      for (int t = 0; t < 2; ++t)
        HIPCHK(block_copy_b(core_zbar(k) + (size_t)t * zc * csz, 1, 2 * zc, b.sZ, (char*)b.Vbar + (size_t)t * L * csz,
                            2 * L, 1, b.sE, dv(c, 1, bet), dv(c, 1, kkp), p.beta[k + 1], p.beta[k], real, nf, s, 1));
      r = gemm(c, dv(c, 2, bet), 1, (int)qb, dv(c, 1, kkp), 1, p.beta[k], dv(c, Da, ra), Da,
               opd(Mk, 1, 0, 2 * zc * Da, 2 * zc, 1, b.sX), opd(gcur, zc * Da, 1, Da, 0, 0, b.sC),
               opd(b.Vbar, L, 0, 1, 0, 0, b.sE), dx(1), 1, 1);
      if (r) return r;
      // the full decomposition of M^H M the forward computed
      const void* Vall = sv.vslot(k);
      r = gemm(c, dv(c, 2, bet), 1, (int)qb, dv(c, 1, kkp), 1, p.beta[k], dv(c, 2, bet), 1,
               opd(Vall, 1, 0, L, 0, 1, b.sE), opd(b.Vbar, L, 0, 1, 0, 0, b.sE), opd(b.Y, L, 0, 1, 0, 0, b.sE));
      if (r) return r;
      HIPCHK(eig_adjoint_scale(dv(c, 2, bet), (int)qb, sv.lslot(k), L, nf, b.Y, L, b.sE, kkp, bs, p.beta[k], real,
                               s));
      r = gemm(c, dv(c, 2, bet), 1, (int)qb, dv(c, 1, kkp), 1, p.beta[k], dv(c, 2, bet), 1,
               opd(Vall, L, 0, 1, 0, 0, b.sE), opd(b.Y, L, 0, 1, 0, 0, b.sE), opd(b.P, L, 0, 1, 0, 0, b.sE));
      if (r) return r;
      // gC += M P;  Mbar = gC V^H (V^H is B_k itself) + (M V) P^H
      r = gemm(c, dv(c, Da, ra), Da, (int)pb, dv(c, 1, kkp), 1, p.beta[k], dv(c, 2, bet), 1, Mrows,
               opd(b.P, L, 0, 1, 0, 0, b.sE), opd(gcur, zc * Da, 1, Da, 0, 0, b.sC), dx(1), 1, 1);
      if (r) return r;
      r = gemm(c, dv(c, Da, ra), Da, (int)pb, dv(c, 2, bet), 2, (int)qb, dv(c, 1, kkp), 1,
               opd(gcur, zc * Da, 1, Da, 0, 0, b.sC), opd(core_z(k), 2 * zc, 0, 1, zc, 0, b.sZ), Mbar_v);
      if (r) return r;
      r = gemm(c, dv(c, Da, ra), Da, (int)pb, dv(c, 2, bet), 2, (int)qb, dv(c, 1, kkp), 1,
               opd(carry_at(k - 1), zc * Da, 1, Da, 0, 0, b.sC), opd(b.P, 1, 0, 2 * L, L, 1, b.sE), Mbar_v, dx(1), 1,
               1);
      if (r) return r;
    }
    // Xbar[a][b][(s, w)] = sum_{(w', t)} Mbar[a][w'][b][t] conj(W[w'][t][s][w])
    if (!ident) {
      r = gemm(c, dv(c, 1, bet), 1, p.beta[k + 1], dx(2 * Db), 1, 2 * Db, dx(2 * Da), 2,
               opd(b.Mbar, 2, 0, 2 * zc, 1, 0, b.sX, (ll)Da * zc * 2),
               opd(Wc + (size_t)k * dcap * 4 * dcap * csz, 4 * Db, 2 * Db, 1, 0, 1, sW),
               opd(b.Xbar, 2 * Db, 0, 1, 0, 0, b.sX, zc * 2 * Db), dv(c, 1, ra), p.rin[k]);
      if (r) return r;
    }
    const Operand XA = ident ? opd(b.Mbar, 2 * zc * Db, 1, 2, 2 * zc, 0, b.sX)
                             : opd(b.Xbar, zc * 2 * Db, Db, 2 * Db, 1, 0, b.sX);
    // grad of A_k = Xbar Cin^H
    r = gemm(c, dv(c, 2, ra), 2, 2 * p.rin[k], dv(c, 1, rb), 1, p.rin[k + 1], dv(c, Db, bet), Db, XA,
             opd(Cin, Db, 1, zc * Db, 0, 1, b.sC), opd(core_gin(k), 2 * ci, ci, 1, 0, 0, sIn));
    if (r) return r;
    // grad of the carry entering site k (= leaving site k + 1) = A_k^H Xbar
    if (k < m - 1) {
      r = gemm(c, dv(c, 1, rb), 1, p.rin[k + 1], dv(c, Db, bet), Db, Db * p.beta[k + 1], dv(c, 2, ra), 2,
               opd(core_in(k), 1, 0, 2 * ci, ci, 1, sIn), XA, opd(gnext, zc * Db, 0, Db, 1, 0, b.sC));
      if (r) return r;
    }
    std::swap(gcur, gnext);
  }
  return QTT_OK;
}

int backward_common(const MpsB& in, const qtt_mpo* W1, const MpoB* Wb, const qtt_opts* opts, const void* saved,
                    size_t saved_sz, const MpsB& out, const MpsB& gout, const MpsB& gin, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!ws || !saved) return fail(QTT_ERR_ARG, "workspace/saved is NULL");
  if (gout.m != out.m || gout.nf != out.nf || gout.cap != out.cap || gout.dtype != out.dtype)
    return fail(QTT_ERR_SHAPE, "grad_out must match out (sites, count, chi_cap, dtype)");
  if (gin.m != in.m || gin.nf != in.nf || gin.cap != in.cap || gin.dtype != in.dtype)
    return fail(QTT_ERR_SHAPE, "grad_in must match in (sites, count, chi_cap, dtype)");
  if (gin.cores == in.cores || gout.cores == out.cores) return fail(QTT_ERR_ARG, "gradients must not alias the states");
  ApplySetup su;
  int r = apply_setup(in, W1, Wb, opts, out, false, su, true);
  if (r) return r;
  if (su.p.refine) return fail(QTT_ERR_ARG, "the adjoint covers the plain sweep only (refine = 0)");
  if (bwd_nmax(su.p) > 512) return fail(QTT_ERR_CAPACITY, "adjoint eigenproblem larger than 512");
  size_t sneed = saved_bytes(su.p, su.csz, in.nf);
  if (saved_sz < sneed) return fail(QTT_ERR_WORKSPACE, "saved buffer %zu < required %zu bytes", saved_sz, sneed);
  size_t need = bwd_bytes(su.p, su.csz, in.nf);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  Carver cs(const_cast<void*>(saved));
  SavedBufs sv = carve_saved(cs, su.p, su.csz, in.nf);
  Carver cw(ws);
  BwdBufs b = carve_bwd(cw, su.p, su.csz, in.nf);
  return run_apply_backward(in, su.W, out, gout, gin, su.p, sv, b, (hipStream_t)stream);
}

ApplyPlan capacity_plan(int m, int chi_cap, int d_cap, bool identity, int refine = 0) {
  std::vector<int> db(m + 1, identity ? 1 : d_cap);
  db[0] = db[m] = 1;
  std::vector<int> kind(m, identity ? 1 : 0);
  // upper bound for every use: any precision, the refinement sweep and the
  // Gram sides of an application that keeps state for its adjoint
  return make_apply_plan(m, chi_cap, chi_cap, chi_cap, chi_cap, db.data(), kind.data(), identity ? 1 : d_cap,
                         refine, identity ? 0 : 1, identity ? 1 : 0);
}

size_t apply_ws(int m, int chi_cap, int d_cap, int prec, bool identity, int nf) {
  return apply_bytes(capacity_plan(m, chi_cap, d_cap, identity), prec == QTT_PREC_FP64 ? 16 : 8, nf);
}

// ------------------------------------------------------------ encode
struct EncBufs {
  int* status;
  void* v;
  void* Rb[2];
  void* V1;
  double* G;
  double* part;
  void* eigws;
  ll sq;      // per-field stride of the 2^m vectors
  ll sV;
  int nmax;
};

EncBufs carve_encode(Carver& cv, int m, int chi, size_t csz, int nf) {
  EncBufs b;
  b.sq = 1ll << m;
  b.nmax = std::max(2, std::min(2 * chi, 1 << (m / 2 + 1)));
  b.sV = (ll)b.nmax * chi;
  b.status = (int*)cv.take(256);
  b.v = cv.take(nf * b.sq * csz);
  b.Rb[0] = cv.take(nf * b.sq * csz);
  b.Rb[1] = cv.take(nf * b.sq * csz);
  b.V1 = cv.take(nf * b.sV * csz);
  b.G = (double*)cv.take((size_t)nf * b.nmax * b.nmax * 16);
  b.part = (double*)cv.take(std::min<size_t>(PART_BYTES, 256ull * b.nmax * b.nmax * 16 * nf));
  b.eigws = cv.take(eig_ws_bytes(b.nmax, chi, nf));
  return b;
}

// img: nf images of N x N (field stride N^2 elements of img_dtype)
// dir 0: a 2^n x 2^n image, quantics-permuted; dir 2: a flat vector of
// length 2^(2n) taken as is (a 1-D signal of 2n bits).
int encode_impl(const void* img, int img_dtype, int n, const qtt_opts& o, const MpsB& out, EncBufs& b,
                const int* chi_dev, hipStream_t s, int dir = 0) {
  const int m = 2 * n, nf = out.nf;
  const int real = out.dtype == QTT_C128 ? 1 : 0;
  const int chi = o.chi_max;
  Ctx c = make_ctx(s, real, nf, m, b.status);
  c.G = b.G; c.gld = b.nmax; c.part = b.part; c.eigws = b.eigws; c.eig_nb = b.nmax; c.eig_kc = chi;
  c.kcap_dev = chi_dev;
  const ll co = out.cap, sOut = out.fstride();
  char* outc = (char*)out.cores;
  auto core_out = [&](int k) { return outc + (size_t)k * co * 2 * co * c.csz; };
  std::vector<int> rb = mps_bounds(m, chi);
  const size_t isz = img_dtype == QTT_C128 ? 16 : (img_dtype == QTT_F32 ? 4 : 8);
  (void)isz;
  HIPCHK(quantics_permute(img, img_dtype, b.v, real ? QTT_C128 : QTT_C64, n, dir, s, nf, b.sq, b.sq));
  HIPCHK(set_ints_strided(out.bonds, 1, c.bs, nf, 1, s));
  HIPCHK(set_ints_strided(out.bonds + m, 1, c.bs, nf, 1, s));
  const void* Rcur = b.v;
  int rsel = 0;
  for (int k = 0; k < m - 1; ++k) {
    const int* rk = out.bonds + k;
    int* kout = out.bonds + k + 1;
    const ll q = 1ll << (m - k - 1);
    const ll pb = 2ll * rb[k];
    void* Rn = b.Rb[rsel];
    // M[(r,s)][c] = R_k[r][s*q + c]: row strides (2q, q), col stride 1
    if (pb <= q) {
      int r = gram(c, opd(Rcur, 2 * q, q, 1, 0, 0, b.sq), opd(Rcur, 1, 0, 2 * q, q, 1, b.sq), dv(c, 2, rk), 2,
                   (int)pb, dx((int)q), 1, q);
      if (r) return r;
      r = eig(c, dv(c, 2, rk), (int)pb, rb[k + 1], o.cutoff, o.tau, kout,
              {emit(core_out(k), 2, 2 * co, co, 1, 0, 0, real, sOut),   // A_k = U
               emit(b.V1, 1, chi, 0, 1, 0, 0, real, b.sV)});           // U [p][i]
      if (r) return r;
      // R_{k+1}[i][c] = sum_p conj(U[p][i]) M[p][c]
      r = gemm(c, dv(c, 1, kout), 1, rb[k + 1], dx((int)q), 1, (int)q, dv(c, 2, rk), 2,
               opd(b.V1, 1, 0, 2 * chi, chi, 1, b.sV), opd(Rcur, 2 * q, q, 1, 0, 0, b.sq),
               opd(Rn, q, 0, 1, 0, 0, b.sq), dx(1), 1, 0, (int)pb);
      if (r) return r;
    } else {
      int r = gram(c, opd(Rcur, 1, 0, 2 * q, q, 1, b.sq), opd(Rcur, 2 * q, q, 1, 0, 0, b.sq), dx((int)q), 1, (int)q,
                   dv(c, 2, rk), 2, pb);
      if (r) return r;
      r = eig(c, dx((int)q), (int)q, rb[k + 1], o.cutoff, o.tau, kout,
              {emit(b.V1, 1, chi, 0, 1, 0, -1, real, b.sV),            // V / sigma [c][i]
               emit(Rn, 1, 1, 0, q, 1, 1, real, b.sq)});               // R_{k+1}[i][c] = sigma_i conj V[c][i]
      if (r) return r;
      r = gemm(c, dv(c, 2, rk), 2, (int)pb, dv(c, 1, kout), 1, rb[k + 1], dx((int)q), 1,
               opd(Rcur, 2 * q, q, 1, 0, 0, b.sq), opd(b.V1, chi, 0, 1, 0, 0, b.sV),
               opd(core_out(k), 2 * co, co, 1, 0, 0, sOut));
      if (r) return r;
    }
    Rcur = Rn;
    rsel ^= 1;
  }
  // last core: [r][s][0] = R[r][s]
  const int* rl = out.bonds + m - 1;
  HIPCHK(block_copy_b(Rcur, 2, 1, b.sq, core_out(m - 1), 2 * co, co, sOut, dv(c, 1, rl), dx(2), rb[m - 1], 2, real,
                      nf, s));
  if (out.norms)
    HIPCHK(block_norm_b(core_out(m - 1), real, dv(c, 1, rl), dx(2), rb[m - 1], 2, 2 * co, co, sOut, out.norms, nf, s));
  return QTT_OK;
}

// ------------------------------------------------------------ to_dense
struct DenseBufs {
  int* status;
  int* bonds;
  void* P[2];
  void* Q[2];
  void* E;
  ll sP, sQ, sE;
};

DenseBufs carve_dense(Carver& cv, int m, int chi, size_t csz, int nf) {
  DenseBufs b;
  int h = m / 2;
  b.sP = ((ll)1 << h) * chi;
  b.sQ = ((ll)1 << (m - h)) * chi;
  b.sE = (ll)1 << m;
  b.status = (int*)cv.take(256);
  b.bonds = (int*)cv.take((size_t)nf * (m + 1) * sizeof(int));
  b.P[0] = cv.take(nf * b.sP * csz);
  b.P[1] = cv.take(nf * b.sP * csz);
  b.Q[0] = cv.take(nf * b.sQ * csz);
  b.Q[1] = cv.take(nf * b.sQ * csz);
  b.E = cv.take(nf * b.sE * csz);
  return b;
}

// out: nf dense N x N fields (stride N^2 elements of out_dtype)
// Decompression of sites off..m-1.  off = 0: the whole MPS (core 0 has left
// bond 1).  off > 0: `boundary` is the row vector (1 x bond off, stride ch,
// per-field stride bsf) of the first off sites contracted at fixed bits, so
// the result is the 2^((m-off)/2) square block those bits select.
int dense_impl(const MpsB& in, void* out, int out_dtype, DenseBufs& b, hipStream_t s, int off = 0,
               const void* boundary = nullptr, ll bsf = 0) {
  const int m = in.m, mp = m - off, h = mp / 2, nf = in.nf;
  const int real = in.dtype == QTT_C128 ? 1 : 0;
  Ctx c = make_ctx(s, real, nf, m, b.status);
  const ll ch = in.cap, sIn = in.fstride();
  std::vector<int> rb = mps_bounds(m, ch);
  char* inc = (char*)in.cores;
  auto core = [&](int k) { return inc + (size_t)k * ch * 2 * ch * c.csz; };
  HIPCHK(sanitize_bonds(in.bonds, b.bonds, m, (int)ch, b.status, nf, s));
  const int* bonds = b.bonds;
  // left: P_(k+1)[(l, s)][b] = P_k[l][r] A_(off+k)[r][s][b], rows 2^(k+1)
  const void* P = off ? boundary : core(0);
  ll pld = ch, sP = off ? bsf : sIn;
  int psel = 0;
  for (int k = off ? 0 : 1; k < h; ++k) {
    const ll rows = 1ll << k;
    const int g = off + k;
    void* Pn = b.P[psel];
    int r = gemm(c, dx((int)rows), 1, (int)rows, dv(c, 2, bonds + g + 1), 2, 2 * rb[g + 1], dv(c, 1, bonds + g), 1,
                 opd(P, pld, 0, 1, 0, 0, sP), opd(core(g), 2 * ch, 0, 1, ch, 0, sIn),
                 opd(Pn, 2 * ch, 0, 1, ch, 0, b.sP));
    if (r) return r;
    P = Pn;
    pld = ch;
    sP = b.sP;
    psel ^= 1;
  }
  // right: Q_(m-1)[r][s] = core m-1 [r][s][0]; Q_k[(r,s)][c] = A_k[(r,s)][b] Q_(k+1)[b][c]
  const void* Q = core(m - 1);
  ll qrs = 2 * ch, qcs = ch, sQ = sIn;   // row / column strides of Q_(k+1)
  int qsel = 0;
  for (int k = m - 2; k >= off + h; --k) {
    const ll cols = 1ll << (m - k - 1);
    void* Qn = b.Q[qsel];
    int r = gemm(c, dv(c, 2, bonds + k), 2, 2 * rb[k], dx((int)cols), 1, (int)cols, dv(c, 1, bonds + k + 1), 1,
                 opd(core(k), 2 * ch, ch, 1, 0, 0, sIn), opd(Q, qrs, 0, qcs, 0, 0, sQ),
                 opd(Qn, 2 * cols, cols, 1, 0, 0, b.sQ));
    if (r) return r;
    Q = Qn;
    qrs = 2 * cols;
    qcs = 1;
    sQ = b.sQ;
    qsel ^= 1;
  }
  // E[l][c] = P_h[l][r] Q_h[r][c]
  const ll L = 1ll << h, Rn = 1ll << (mp - h);
  int r = gemm(c, dx((int)L), 1, (int)L, dx((int)Rn), 1, (int)Rn, dv(c, 1, bonds + off + h), 1,
               opd(P, pld, 0, 1, 0, 0, sP), opd(Q, qrs, 0, qcs, 0, 0, sQ), opd(b.E, Rn, 0, 1, 0, 0, b.sE));
  if (r) return r;
  HIPCHK(quantics_permute(b.E, real ? QTT_C128 : QTT_C64, out, out_dtype, mp / 2, 1, s, nf, b.sE, b.sE));
  return QTT_OK;
}

// ------------------------------------------------------------ point evaluation
// Every point's row vector is carried site by site: one contraction of all
// rows with the core (both bit values), then the half each point's bit picks.
struct EvalBufs {
  int* status;
  int* bonds;
  void* L[2];
  void* C;
  int* pts;                  // two ints (row, col) for the block boundary
  ll ldl, ldc;
};

EvalBufs carve_eval(Carver& cv, int m, int cap, int count, size_t csz) {
  EvalBufs b;
  b.ldl = cap;
  b.ldc = 2ll * cap;
  b.status = (int*)cv.take(256);
  b.bonds = (int*)cv.take((size_t)(m + 1) * sizeof(int));
  b.L[0] = cv.take((size_t)count * b.ldl * csz);
  b.L[1] = cv.take((size_t)count * b.ldl * csz);
  b.C = cv.take((size_t)count * b.ldc * csz);
  b.pts = (int*)cv.take(2 * sizeof(int));
  return b;
}

// Contract sites 0..nsite-1 at each point's bits; returns the buffer that
// holds the row vectors (count x bond nsite, stride ldl).
int eval_rows(const MpsB& in, const int* rows, const int* cols, int count, int nsite, EvalBufs& b, hipStream_t s,
              void** result) {
  const int m = in.m, n = m / 2;
  const int real = in.dtype == QTT_C128 ? 1 : 0;
  Ctx c = make_ctx(s, real, 1, m, b.status);
  const ll ch = in.cap;
  std::vector<int> rb = mps_bounds(m, ch);
  auto core = [&](int k) { return (char*)in.cores + (size_t)k * ch * 2 * ch * c.csz; };
  HIPCHK(sanitize_bonds(in.bonds, b.bonds, m, (int)ch, b.status, 1, s));
  HIPCHK(unit_rows(b.L[0], b.ldl, count, (int)ch, real, s));
  int cur = 0;
  for (int k = 0; k < nsite; ++k) {
    // C[p][(r', s)] = L[p][r] A_k[r][s][r']
    int r = gemm(c, dx(count), 1, count, dv(c, 2, b.bonds + k + 1), 2, 2 * rb[k + 1], dv(c, 1, b.bonds + k), 1,
                 opd(b.L[cur], b.ldl, 0, 1, 0), opd(core(k), 2 * ch, 0, 1, ch), opd(b.C, b.ldc, 0, 2, 1));
    if (r) return r;
    HIPCHK(select_bit(b.C, b.ldc, b.L[cur ^ 1], b.ldl, rows, cols, count, k, n, b.bonds + k + 1, (int)ch, real, s));
    cur ^= 1;
  }
  *result = b.L[cur];
  return QTT_OK;
}

// ------------------------------------------------------------ adjoint of the decompression
// Forward: E = P_h Q_h with the left half-chain P_(k+1) = P_k A_k (k < h) and
// the right half-chain Q_k = A_k Q_(k+1) (k >= h).  Backward: Pbar_h =
// Ebar Q_h^H, Qbar_h = P_h^H Ebar, then each product is undone:
// Abar_k = P_k^H Pbar_(k+1), Pbar_k = Pbar_(k+1) A_k^H (left) and
// Abar_k = Qbar_k Q_(k+1)^H, Qbar_(k+1) = A_k^H Qbar_k (right).
struct DenseBwdBufs {
  int* status;
  int* bonds;
  void* E;
  void* P;              // P_k (2 <= k <= h) at element offset poff[k] (per field sP)
  void* Q;              // Q_k (h <= k <= m - 2) at element offset qoff[k] (per field sQ)
  void* PB[2];
  void* QB[2];
  ll sE, sP, sQ, sPB, sQB;
  std::vector<ll> poff, qoff;
};

DenseBwdBufs carve_dense_bwd(Carver& cv, int m, int ch, size_t csz, int nf) {
  DenseBwdBufs b;
  const int h = m / 2;
  b.poff.assign(m + 1, 0);
  b.qoff.assign(m + 1, 0);
  ll o = 0;
  for (int k = 2; k <= h; ++k) { b.poff[k] = o; o += ((ll)1 << k) * ch; }
  b.sP = std::max<ll>(o, 1);
  o = 0;
  for (int k = m - 2; k >= h; --k) { b.qoff[k] = o; o += ((ll)1 << (m - k)) * ch; }
  b.sQ = std::max<ll>(o, 1);
  b.sE = (ll)1 << m;
  b.sPB = ((ll)1 << h) * ch;
  b.sQB = ((ll)1 << (m - h)) * ch;
  b.status = (int*)cv.take(256);
  b.bonds = (int*)cv.take((size_t)nf * (m + 1) * sizeof(int));
  b.E = cv.take(nf * b.sE * csz);
  b.P = cv.take(nf * b.sP * csz);
  b.Q = cv.take(nf * b.sQ * csz);
  b.PB[0] = cv.take(nf * b.sPB * csz);
  b.PB[1] = cv.take(nf * b.sPB * csz);
  b.QB[0] = cv.take(nf * b.sQB * csz);
  b.QB[1] = cv.take(nf * b.sQB * csz);
  return b;
}

int dense_backward_impl(const MpsB& in, const void* gdense, const MpsB& g, DenseBwdBufs& b, hipStream_t s) {
  const int m = in.m, h = m / 2, nf = in.nf;
  const int real = in.dtype == QTT_C128 ? 1 : 0;
  Ctx c = make_ctx(s, real, nf, m, b.status);
  const ll ch = in.cap, cg = g.cap, sIn = in.fstride(), sG = g.fstride();
  const size_t csz = c.csz;
  std::vector<int> rb = mps_bounds(m, ch);
  auto core = [&](int k) { return (char*)in.cores + (size_t)k * ch * 2 * ch * csz; };
  auto gcore = [&](int k) { return (char*)g.cores + (size_t)k * cg * 2 * cg * csz; };
  auto pslot = [&](int k) { return (char*)b.P + (size_t)b.poff[k] * csz; };
  auto qslot = [&](int k) { return (char*)b.Q + (size_t)b.qoff[k] * csz; };
  HIPCHK(sanitize_bonds(in.bonds, b.bonds, m, (int)ch, b.status, nf, s));
  const int* bonds = b.bonds;
  HIPCHK(zero_fill(g.cores, (size_t)nf * sG * csz, s));
  HIPCHK(copy_ints(bonds, g.bonds, nf * (m + 1), s));
  HIPCHK(quantics_permute(gdense, real ? QTT_C128 : QTT_C64, b.E, real ? QTT_C128 : QTT_C64, m / 2, 0, s, nf, b.sE,
                          b.sE));
  // left half-chain, every P_k kept: P_k = [l][r] with ld pld[k]
  std::vector<const void*> Pp(h + 1);
  std::vector<ll> pld(h + 1), psb(h + 1);
  Pp[1] = core(0); pld[1] = ch; psb[1] = sIn;
  for (int k = 1; k < h; ++k) {
    const ll rows = 1ll << k;
    void* Pn = pslot(k + 1);
    int r = gemm(c, dx((int)rows), 1, (int)rows, dv(c, 2, bonds + k + 1), 2, 2 * rb[k + 1], dv(c, 1, bonds + k), 1,
                 opd(Pp[k], pld[k], 0, 1, 0, 0, psb[k]), opd(core(k), 2 * ch, 0, 1, ch, 0, sIn),
                 opd(Pn, 2 * ch, 0, 1, ch, 0, b.sP));
    if (r) return r;
    Pp[k + 1] = Pn; pld[k + 1] = ch; psb[k + 1] = b.sP;
  }
  // right half-chain: Q_k = [(r, s)][c] with row stride qrs[k] (per r) and column stride qcs[k]
  std::vector<const void*> Qp(m);
  std::vector<ll> qrs(m), qcs(m), qsb(m);
  Qp[m - 1] = core(m - 1); qrs[m - 1] = 2 * ch; qcs[m - 1] = ch; qsb[m - 1] = sIn;
  for (int k = m - 2; k >= h; --k) {
    const ll cols = 1ll << (m - k - 1);
    void* Qn = qslot(k);
    int r = gemm(c, dv(c, 2, bonds + k), 2, 2 * rb[k], dx((int)cols), 1, (int)cols, dv(c, 1, bonds + k + 1), 1,
                 opd(core(k), 2 * ch, ch, 1, 0, 0, sIn), opd(Qp[k + 1], qrs[k + 1], 0, qcs[k + 1], 0, 0, qsb[k + 1]),
                 opd(Qn, 2 * cols, cols, 1, 0, 0, b.sQ));
    if (r) return r;
    Qp[k] = Qn; qrs[k] = 2 * cols; qcs[k] = 1; qsb[k] = b.sQ;
  }
  const ll Lh = 1ll << h, Rn = 1ll << (m - h);
  // Pbar_h = Ebar Q_h^H ([l][r], ld ch); Qbar_h = P_h^H Ebar ([r][c], row stride Rn)
  int r = gemm(c, dx((int)Lh), 1, (int)Lh, dv(c, 1, bonds + h), 1, rb[h], dx((int)Rn), 1,
               opd(b.E, Rn, 0, 1, 0, 0, b.sE), opd(Qp[h], qcs[h], 0, qrs[h], 0, 1, qsb[h]),
               opd(b.PB[0], ch, 0, 1, 0, 0, b.sPB));
  if (r) return r;
  r = gemm(c, dv(c, 1, bonds + h), 1, rb[h], dx((int)Rn), 1, (int)Rn, dx((int)Lh), 1,
           opd(Pp[h], 1, 0, pld[h], 0, 1, psb[h]), opd(b.E, Rn, 0, 1, 0, 0, b.sE), opd(b.QB[0], Rn, 0, 1, 0, 0, b.sQB));
  if (r) return r;
  // left chain backwards
  int ps = 0;
  for (int k = h - 1; k >= 1; --k) {
    const ll rows = 1ll << k;
    const void* PB = b.PB[ps];
    // Abar_k[r][(b, s)] = P_k^H Pbar_(k+1), Pbar_(k+1) = [(l, s)][b] with ld ch
    r = gemm(c, dv(c, 1, bonds + k), 1, rb[k], dv(c, 2, bonds + k + 1), 2, 2 * rb[k + 1], dx((int)rows), 1,
             opd(Pp[k], 1, 0, pld[k], 0, 1, psb[k]), opd(PB, 2 * ch, 0, 1, ch, 0, b.sPB),
             opd(gcore(k), 2 * cg, 0, 1, cg, 0, sG));
    if (r) return r;
    // Pbar_k = Pbar_(k+1) A_k^H  (K = (b, s))
    r = gemm(c, dx((int)rows), 1, (int)rows, dv(c, 1, bonds + k), 1, rb[k], dv(c, 2, bonds + k + 1), 2,
             opd(PB, 2 * ch, 0, 1, ch, 0, b.sPB), opd(core(k), 1, ch, 2 * ch, 0, 1, sIn),
             opd(b.PB[ps ^ 1], ch, 0, 1, 0, 0, b.sPB));
    if (r) return r;
    ps ^= 1;
  }
  // Pbar_1 = grad of core 0 ([s][b])
  HIPCHK(block_copy_b(b.PB[ps], ch, 1, b.sPB, gcore(0), cg, 1, sG, dx(2), dv(c, 1, bonds + 1), 2, rb[1], real, nf, s));
  // right chain forwards: Qbar_k = [(r, s)][c] with row stride 2 * cols_k
  int qs = 0;
  for (int k = h; k <= m - 2; ++k) {
    const ll cols = 1ll << (m - k - 1);
    const void* QB = b.QB[qs];
    // Abar_k[(r, s)][b] = Qbar_k Q_(k+1)^H
    r = gemm(c, dv(c, 2, bonds + k), 2, 2 * rb[k], dv(c, 1, bonds + k + 1), 1, rb[k + 1], dx((int)cols), 1,
             opd(QB, 2 * cols, cols, 1, 0, 0, b.sQB), opd(Qp[k + 1], qcs[k + 1], 0, qrs[k + 1], 0, 1, qsb[k + 1]),
             opd(gcore(k), 2 * cg, cg, 1, 0, 0, sG));
    if (r) return r;
    // Qbar_(k+1)[b][c] = A_k^H Qbar_k (row stride cols)
    r = gemm(c, dv(c, 1, bonds + k + 1), 1, rb[k + 1], dx((int)cols), 1, (int)cols, dv(c, 2, bonds + k), 2,
             opd(core(k), 1, 0, 2 * ch, ch, 1, sIn), opd(QB, 2 * cols, cols, 1, 0, 0, b.sQB),
             opd(b.QB[qs ^ 1], cols, 0, 1, 0, 0, b.sQB));
    if (r) return r;
    qs ^= 1;
  }
  // Qbar_(m-1) = grad of core m-1 ([r][s], row stride 2)
  HIPCHK(block_copy_b(b.QB[qs], 2, 1, b.sQB, gcore(m - 1), 2 * cg, cg, sG, dv(c, 1, bonds + m - 1), dx(2), rb[m - 1], 2,
                      real, nf, s));
  return QTT_OK;
}

int dense_bwd_common(const MpsB& in, const void* gdense, const MpsB& g, void* ws, size_t ws_bytes, void* stream) {
  if (!gdense || !ws) return fail(QTT_ERR_ARG, "grad_dense/workspace is NULL");
  if (g.m != in.m || g.nf != in.nf || g.dtype != in.dtype || g.cap != in.cap)
    return fail(QTT_ERR_SHAPE, "grad must match in (sites, count, chi_cap, dtype)");
  if (g.cores == in.cores) return fail(QTT_ERR_ARG, "grad must not alias in");
  size_t csz = in.dtype == QTT_C128 ? 16 : 8;
  Carver cv(nullptr);
  carve_dense_bwd(cv, in.m, in.cap, csz, in.nf);
  if (ws_bytes < cv.off) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, cv.off);
  Carver cw(ws);
  DenseBwdBufs b = carve_dense_bwd(cw, in.m, in.cap, csz, in.nf);
  return dense_backward_impl(in, gdense, g, b, (hipStream_t)stream);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* tt_last_error(void) { return g_err.c_str(); }
const char* tt_version(void) { return "libqtt 0.1 (gfx950)"; }

size_t tt_workspace_size(int op, int n_sites, int chi_cap, int d_cap, int prec) {
  return tt_workspace_size_batched(op, 1, n_sites, chi_cap, d_cap, prec);
}

size_t tt_workspace_size_batched(int op, int count, int n_sites, int chi_cap, int d_cap, int prec) {
  if (n_sites < 2 || (n_sites & 1) || chi_cap < 1 || chi_cap > 256 || count < 1) return 0;
  size_t csz = prec == QTT_PREC_FP64 ? 16 : 8;
  switch (op) {
    case QTT_OP_ENCODE: {
      Carver cv(nullptr);
      carve_encode(cv, n_sites, chi_cap, csz, count);
      return cv.off;
    }
    case QTT_OP_APPLY:
      if (d_cap < 1) return 0;
      // covers every precision and the refinement sweep
      return apply_bytes(capacity_plan(n_sites, chi_cap, d_cap, false, 1), csz, count);
    case QTT_OP_TRUNCATE:
      return apply_ws(n_sites, chi_cap, 1, prec, true, count);
    case QTT_OP_TO_DENSE: {
      Carver cv(nullptr);
      carve_dense(cv, n_sites, chi_cap, csz, count);
      return cv.off;
    }
    case QTT_OP_APPLY_BACKWARD:
      if (d_cap < 1) return 0;
      return bwd_bytes(capacity_plan(n_sites, chi_cap, d_cap, false), csz, count);
    case QTT_OP_TO_DENSE_BACKWARD: {
      Carver cv(nullptr);
      carve_dense_bwd(cv, n_sites, chi_cap, csz, count);
      return cv.off;
    }
    case QTT_OP_LOSS:
      return 256 + intensity_loss_ws(count);
    default:
      return 0;
  }
}

size_t tt_saved_size(int n_sites, int chi_cap, int d_cap, int prec) {
  return tt_saved_size_batched(1, n_sites, chi_cap, d_cap, prec);
}

size_t tt_saved_size_batched(int count, int n_sites, int chi_cap, int d_cap, int prec) {
  if (n_sites < 2 || (n_sites & 1) || chi_cap < 1 || chi_cap > 256 || count < 1 || d_cap < 1) return 0;
  return saved_bytes(capacity_plan(n_sites, chi_cap, d_cap, false), prec == QTT_PREC_FP64 ? 16 : 8, count);
}

static int encode_common(const void* img, int img_dtype, int log2_side, const qtt_opts* opts, const MpsB& out,
                         const int* chi_dev, void* ws, size_t ws_bytes, void* stream) {
  if (!img) return fail(QTT_ERR_ARG, "img is NULL");
  if (log2_side < 1 || log2_side > 15) return fail(QTT_ERR_SHAPE, "log2_side %d outside [1, 15]", log2_side);
  if (out.m != 2 * log2_side) return fail(QTT_ERR_SHAPE, "out has %d sites, need %d", out.m, 2 * log2_side);
  if (img_dtype < QTT_C64 || img_dtype > QTT_F64) return fail(QTT_ERR_DTYPE, "bad img dtype %d", img_dtype);
  if (!ws) return fail(QTT_ERR_ARG, "workspace is NULL");
  qtt_opts o;
  opts_defaults(opts, out.cap, o);
  if (o.chi_max < 1 || o.chi_max > out.cap) return fail(QTT_ERR_CAPACITY, "chi_max %d outside [1, %d]", o.chi_max, out.cap);
  if ((o.prec == QTT_PREC_FP64) != (out.dtype == QTT_C128)) return fail(QTT_ERR_DTYPE, "precision and dtype disagree");
  size_t csz = out.dtype == QTT_C128 ? 16 : 8;
  Carver cv(nullptr);
  carve_encode(cv, out.m, o.chi_max, csz, out.nf);
  if (ws_bytes < cv.off) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, cv.off);
  Carver cw(ws);
  EncBufs b = carve_encode(cw, out.m, o.chi_max, csz, out.nf);
  return encode_impl(img, img_dtype, log2_side, o, out, b, chi_dev, (hipStream_t)stream);
}

int tt_encode(const void* img, int img_dtype, int log2_side, const qtt_opts* opts, qtt_mps* out, void* ws,
              size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if (!img) return fail(QTT_ERR_ARG, "img is NULL");
  if (log2_side < 1 || log2_side > 15) return fail(QTT_ERR_SHAPE, "log2_side %d outside [1, 15]", log2_side);
  if ((r = check_mps(out, "out"))) return r;
  return encode_common(img, img_dtype, log2_side, opts, view(out), nullptr, ws, ws_bytes, stream);
}

int tt_encode_batched(const void* img, int img_dtype, int log2_side, const qtt_opts* opts, const int32_t* chi_dev,
                      qtt_mps_batch* out, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mpsb(out, "out"))) return r;
  return encode_common(img, img_dtype, log2_side, opts, view(out), chi_dev, ws, ws_bytes, stream);
}

int mpo_apply(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts, qtt_mps* out, void* saved,
              size_t saved_bytes, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if ((r = check_mps(out, "out"))) return r;
  if (in->cores == out->cores) return fail(QTT_ERR_ARG, "in and out must not alias");
  if (!W) return fail(QTT_ERR_ARG, "MPO is NULL");
  return apply_common(view(in), W, nullptr, opts, view(out), nullptr, ws, ws_bytes, stream, false, saved,
                      saved_bytes);
}

static MpoB mpob_view(const qtt_mpo_batch* W) {
  MpoB wb;
  wb.nf = W->count; wb.m = W->n_sites; wb.dcap = W->d_cap; wb.dtype = W->dtype;
  wb.cores = W->cores; wb.dbonds = W->d_bonds; wb.kind = W->site_kind;
  return wb;
}

int mpo_apply_batched(const qtt_mps_batch* in, const qtt_mpo_batch* W, const qtt_opts* opts, const int32_t* chi_dev,
                      qtt_mps_batch* out, void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mpsb(in, "in"))) return r;
  if ((r = check_mpsb(out, "out"))) return r;
  if (in->cores == out->cores) return fail(QTT_ERR_ARG, "in and out must not alias");
  if (!W) return fail(QTT_ERR_ARG, "MPO batch is NULL");
  MpoB wb = mpob_view(W);
  return apply_common(view(in), nullptr, &wb, opts, view(out), chi_dev, ws, ws_bytes, stream, false, saved,
                      saved_bytes);
}

static size_t hadamard_mpo_bytes(int m, int cap_a, size_t csz) {
  return ((size_t)m * cap_a * 4 * cap_a * csz + 255) / 256 * 256;
}

size_t tt_hadamard_workspace_size(int n_sites, int chi_cap_a, int chi_cap, int prec) {
  const size_t ap = tt_workspace_size(QTT_OP_APPLY, n_sites, chi_cap, chi_cap_a, prec);
  if (!ap || chi_cap_a < 1 || chi_cap_a > 256) return 0;
  return hadamard_mpo_bytes(n_sites, chi_cap_a, prec == QTT_PREC_FP64 ? 16 : 8) + ap;
}

int tt_hadamard(const qtt_mps* a, int conj_a, const qtt_mps* b, const qtt_opts* opts, qtt_mps* out, void* ws,
                size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(a, "a"))) return r;
  if ((r = check_mps(b, "b"))) return r;
  if ((r = check_mps(out, "out"))) return r;
  if (a->n_sites != b->n_sites) return fail(QTT_ERR_SHAPE, "a has %d sites, b %d", a->n_sites, b->n_sites);
  if (a->dtype != b->dtype) return fail(QTT_ERR_DTYPE, "a and b dtypes differ");
  if (out->cores == b->cores || out->cores == a->cores) return fail(QTT_ERR_ARG, "out must not alias a or b");
  if (!ws) return fail(QTT_ERR_ARG, "workspace is NULL");
  const int m = a->n_sites, dcap = a->chi_cap;
  const size_t csz = a->dtype == QTT_C128 ? 16 : 8;
  const size_t wsz = hadamard_mpo_bytes(m, dcap, csz);
  if (ws_bytes < wsz) return fail(QTT_ERR_WORKSPACE, "workspace %zu < %zu bytes for the operator", ws_bytes, wsz);
  // the element-wise product a (.) b is the diagonal operator of a applied to
  // b: its cores are delta_ts A_k, bonds those of any MPS of a's capacity
  std::vector<int> db = mps_bounds(m, dcap);
  std::vector<int> kind(m, 2);
  qtt_mpo W;
  W.n_sites = m;
  W.d_cap = dcap;
  W.dtype = a->dtype;
  W.cores = ws;
  W.d_bonds = db.data();
  W.site_kind = kind.data();
  HIPCHK(mps_to_diag_mpo(a->cores, a->bonds, a->chi_cap, conj_a ? 1 : 0, ws, dcap, m, a->dtype == QTT_C128 ? 1 : 0,
                         (hipStream_t)stream));
  return apply_common(view(b), &W, nullptr, opts, view(out), nullptr, (char*)ws + wsz, ws_bytes - wsz, stream, false);
}

int tt_truncate(qtt_mps* inout, const qtt_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(inout, "inout"))) return r;
  qtt_opts o;
  opts_defaults(opts, inout->chi_cap, o);
  o.chi_zip = inout->chi_cap;     // the right-to-left pass only removes numerical zeros
  return apply_common(view(inout), nullptr, nullptr, &o, view(inout), nullptr, ws, ws_bytes, stream, true);
}

static int dense_common(const MpsB& in, void* out, int out_dtype, void* ws, size_t ws_bytes, void* stream) {
  if (!out || !ws) return fail(QTT_ERR_ARG, "out/workspace is NULL");
  if (out_dtype != QTT_C64 && out_dtype != QTT_C128) return fail(QTT_ERR_DTYPE, "out dtype must be C64 or C128");
  size_t csz = in.dtype == QTT_C128 ? 16 : 8;
  Carver cv(nullptr);
  carve_dense(cv, in.m, in.cap, csz, in.nf);
  if (ws_bytes < cv.off) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, cv.off);
  Carver cw(ws);
  DenseBufs b = carve_dense(cw, in.m, in.cap, csz, in.nf);
  return dense_impl(in, out, out_dtype, b, (hipStream_t)stream);
}

int tt_to_dense(const qtt_mps* in, void* out, int out_dtype, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  return dense_common(view(in), out, out_dtype, ws, ws_bytes, stream);
}

int tt_to_dense_batched(const qtt_mps_batch* in, void* out, int out_dtype, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mpsb(in, "in"))) return r;
  return dense_common(view(in), out, out_dtype, ws, ws_bytes, stream);
}

int mpo_apply_backward(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts, const void* saved,
                       size_t saved_bytes, const qtt_mps* out, const qtt_mps* grad_out, qtt_mps* grad_in, void* ws,
                       size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if ((r = check_mps(out, "out"))) return r;
  if ((r = check_mps(grad_out, "grad_out"))) return r;
  if ((r = check_mps(grad_in, "grad_in"))) return r;
  if (!W) return fail(QTT_ERR_ARG, "MPO is NULL");
  return backward_common(view(in), W, nullptr, opts, saved, saved_bytes, view(out), view(grad_out), view(grad_in), ws,
                         ws_bytes, stream);
}

int mpo_apply_backward_batched(const qtt_mps_batch* in, const qtt_mpo_batch* W, const qtt_opts* opts,
                               const void* saved, size_t saved_bytes, const qtt_mps_batch* out,
                               const qtt_mps_batch* grad_out, qtt_mps_batch* grad_in, void* ws, size_t ws_bytes,
                               void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mpsb(in, "in"))) return r;
  if ((r = check_mpsb(out, "out"))) return r;
  if ((r = check_mpsb(grad_out, "grad_out"))) return r;
  if ((r = check_mpsb(grad_in, "grad_in"))) return r;
  if (!W) return fail(QTT_ERR_ARG, "MPO batch is NULL");
  MpoB wb = mpob_view(W);
  return backward_common(view(in), nullptr, &wb, opts, saved, saved_bytes, view(out), view(grad_out), view(grad_in),
                         ws, ws_bytes, stream);
}

int tt_to_dense_backward(const qtt_mps* in, const void* grad_dense, qtt_mps* grad, void* ws, size_t ws_bytes,
                         void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if ((r = check_mps(grad, "grad"))) return r;
  return dense_bwd_common(view(in), grad_dense, view(grad), ws, ws_bytes, stream);
}

int tt_to_dense_backward_batched(const qtt_mps_batch* in, const void* grad_dense, qtt_mps_batch* grad, void* ws,
                                 size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mpsb(in, "in"))) return r;
  if ((r = check_mpsb(grad, "grad"))) return r;
  return dense_bwd_common(view(in), grad_dense, view(grad), ws, ws_bytes, stream);
}

int tt_intensity_loss(const void* field, const void* target, int dtype, int log2_side, int count, double* loss,
                      void* grad, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!field || !target || !loss || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (dtype != QTT_C64 && dtype != QTT_C128) return fail(QTT_ERR_DTYPE, "field dtype must be C64 or C128");
  if (log2_side < 1 || log2_side > 15) return fail(QTT_ERR_SHAPE, "log2_side %d outside [1, 15]", log2_side);
  if (count < 1) return fail(QTT_ERR_ARG, "count %d < 1", count);
  if (ws_bytes < 256 + intensity_loss_ws(count)) return fail(QTT_ERR_WORKSPACE, "workspace too small");
  const long long per = 1ll << (2 * log2_side);
  HIPCHK(intensity_loss(field, target, dtype == QTT_C128 ? 1 : 0, per, count, loss, grad, (char*)ws + 256,
                        (hipStream_t)stream));
  return QTT_OK;
}

// ---- separable encode, point evaluation, block decompression
static int sep_cap(int chi_cap) {
  int c = 1;
  while ((c + 1) * (c + 1) <= chi_cap) ++c;
  return c;
}

size_t tt_encode_separable_workspace_size(int log2_side, int chi_cap, int prec) {
  if (log2_side < 2 || (log2_side & 1) || log2_side > 30 || chi_cap < 1 || chi_cap > 256) return 0;
  const size_t csz = prec == QTT_PREC_FP64 ? 16 : 8;
  const int c1 = sep_cap(chi_cap), n = log2_side;
  Carver cv(nullptr);
  cv.take(256);
  for (int i = 0; i < 2; ++i) {
    cv.take((size_t)n * c1 * 2 * c1 * csz);
    cv.take((size_t)(n + 1) * sizeof(int));
  }
  carve_encode(cv, n, c1, csz, 1);
  return cv.off;
}

int tt_encode_separable(const void* vec_a, const void* vec_b, int vec_dtype, int log2_side, qtt_mps* out, void* ws,
                        size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if (!vec_a || !vec_b || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if ((r = check_mps(out, "out"))) return r;
  if (log2_side < 2 || (log2_side & 1) || log2_side > 30)
    return fail(QTT_ERR_SHAPE, "log2_side %d must be even and in [2, 30]", log2_side);
  if (out->n_sites != 2 * log2_side) return fail(QTT_ERR_SHAPE, "out has %d sites, need %d", out->n_sites, 2 * log2_side);
  if (vec_dtype < QTT_C64 || vec_dtype > QTT_F64) return fail(QTT_ERR_DTYPE, "bad vector dtype %d", vec_dtype);
  const int real = out->dtype == QTT_C128 ? 1 : 0;
  const size_t csz = real ? 16 : 8;
  const size_t need = tt_encode_separable_workspace_size(log2_side, out->chi_cap, real ? QTT_PREC_FP64 : QTT_PREC_FP32);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  const int c1 = sep_cap(out->chi_cap), n = log2_side;
  Carver cw(ws);
  int* status = (int*)cw.take(256);
  MpsB f[2];
  for (int i = 0; i < 2; ++i) {
    f[i].nf = 1; f[i].m = n; f[i].cap = c1; f[i].dtype = out->dtype;
    f[i].cores = cw.take((size_t)n * c1 * 2 * c1 * csz);
    f[i].bonds = (int*)cw.take((size_t)(n + 1) * sizeof(int));
    f[i].norms = nullptr;
  }
  EncBufs eb = carve_encode(cw, n, c1, csz, 1);
  eb.status = status;          // report eigensolver failures in the workspace head
  qtt_opts o;
  opts_defaults(nullptr, c1, o);
  o.prec = real ? QTT_PREC_FP64 : QTT_PREC_FP32;
  hipStream_t s = (hipStream_t)stream;
  const void* vecs[2] = {vec_a, vec_b};
  for (int i = 0; i < 2; ++i) {
    r = encode_impl(vecs[i], vec_dtype, n / 2, o, f[i], eb, nullptr, s, 2);
    if (r) return r;
  }
  HIPCHK(interleave(f[0].cores, f[0].bonds, c1, f[1].cores, f[1].bonds, c1, out->cores, out->bonds, out->chi_cap, n,
                    real, status, s));
  (void)eb;
  return QTT_OK;
}

// ---- low-rank encode: a sum of separable terms, never densified
static size_t vec_elem_bytes(int vec_dtype) {
  return vec_dtype == QTT_C128 ? 16 : (vec_dtype == QTT_C64 || vec_dtype == QTT_F64) ? 8 : 4;
}

size_t tt_encode_low_rank_workspace_size(int log2_side, int rank, int term_cap, int chi_cap, int prec) {
  if (rank < 1 || rank > QTT_MAX_RANK || term_cap < 1 || term_cap > 256 || chi_cap < 1 || chi_cap > 256) return 0;
  const size_t sep = tt_encode_separable_workspace_size(log2_side, term_cap, prec);
  if (!sep) return 0;
  const size_t csz = prec == QTT_PREC_FP64 ? 16 : 8;
  const int m = 2 * log2_side;
  const size_t tru = tt_workspace_size(QTT_OP_TRUNCATE, m, chi_cap, 1, prec);
  Carver cv(nullptr);
  cv.take(std::max(sep, tru));
  cv.take((size_t)rank * m * term_cap * 2 * term_cap * csz);
  cv.take((size_t)rank * (m + 1) * sizeof(int));
  return cv.off;
}

int tt_encode_low_rank(const void* vecs_a, const void* vecs_b, int vec_dtype, int log2_side, int rank, int term_cap,
                       qtt_mps* out, const qtt_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if (!vecs_a || !vecs_b || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if ((r = check_mps(out, "out"))) return r;
  if (rank < 1 || rank > QTT_MAX_RANK) return fail(QTT_ERR_ARG, "rank %d outside [1, %d]", rank, QTT_MAX_RANK);
  if (log2_side < 2 || (log2_side & 1) || log2_side > 30)
    return fail(QTT_ERR_SHAPE, "log2_side %d must be even and in [2, 30]", log2_side);
  if (out->n_sites != 2 * log2_side) return fail(QTT_ERR_SHAPE, "out has %d sites, need %d", out->n_sites, 2 * log2_side);
  if (vec_dtype < QTT_C64 || vec_dtype > QTT_F64) return fail(QTT_ERR_DTYPE, "bad vector dtype %d", vec_dtype);
  if (term_cap < 1 || (long long)rank * term_cap > out->chi_cap)
    return fail(QTT_ERR_CAPACITY, "rank %d x term_cap %d exceeds out->chi_cap %d", rank, term_cap, out->chi_cap);
  const int real = out->dtype == QTT_C128 ? 1 : 0;
  const int prec = real ? QTT_PREC_FP64 : QTT_PREC_FP32;
  const size_t csz = real ? 16 : 8;
  const size_t need = tt_encode_low_rank_workspace_size(log2_side, rank, term_cap, out->chi_cap, prec);
  if (!need) return fail(QTT_ERR_CAPACITY, "term_cap %d outside [1, 256]", term_cap);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  const int m = 2 * log2_side;
  const size_t sub_bytes = std::max(tt_encode_separable_workspace_size(log2_side, term_cap, prec),
                                    tt_workspace_size(QTT_OP_TRUNCATE, m, out->chi_cap, 1, prec));
  // the sub-calls' workspace comes first, so their status word is this call's
  Carver cw(ws);
  void* sub = cw.take(sub_bytes);
  char* terms = (char*)cw.take((size_t)rank * m * term_cap * 2 * term_cap * csz);
  int* tbonds = (int*)cw.take((size_t)rank * (m + 1) * sizeof(int));
  const size_t tstride = (size_t)m * term_cap * 2 * term_cap * csz;
  const size_t vstride = ((size_t)1 << log2_side) * vec_elem_bytes(vec_dtype);
  for (int t = 0; t < rank; ++t) {
    qtt_mps term;
    term.n_sites = m;
    term.chi_cap = term_cap;
    term.dtype = out->dtype;
    term.cores = terms + t * tstride;
    term.bonds = tbonds + t * (m + 1);
    term.norm = nullptr;
    r = tt_encode_separable((const char*)vecs_a + t * vstride, (const char*)vecs_b + t * vstride, vec_dtype,
                            log2_side, &term, sub, sub_bytes, stream);
    if (r) return r;
  }
  HIPCHK(direct_sum(terms, tbonds, rank, term_cap, m, out->cores, out->bonds, out->chi_cap, real, (int*)sub,
                    (hipStream_t)stream));
  return tt_truncate(out, opts, sub, sub_bytes, stream);
}

// ---- perfect sampling (right to left over a left-canonical MPS)
size_t tt_sample_workspace_size(int n_sites, int chi_cap, int count, int prec) {
  return tt_eval_points_workspace_size(n_sites, chi_cap, count, prec);
}

int tt_sample(const qtt_mps* in, const double* uniforms, int count, int32_t* rows, int32_t* cols, void* ws,
              size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if (!uniforms || !rows || !cols || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (count < 1) return fail(QTT_ERR_ARG, "count %d < 1", count);
  const int m = in->n_sites;
  const int real = in->dtype == QTT_C128 ? 1 : 0;
  const size_t csz = real ? 16 : 8;
  Carver cv(nullptr);
  carve_eval(cv, m, in->chi_cap, count, csz);
  if (ws_bytes < cv.off) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, cv.off);
  Carver cw(ws);
  EvalBufs b = carve_eval(cw, m, in->chi_cap, count, csz);
  hipStream_t s = (hipStream_t)stream;
  Ctx c = make_ctx(s, real, 1, m, b.status);
  const ll ch = in->chi_cap;
  std::vector<int> rb = mps_bounds(m, ch);
  auto core = [&](int k) { return (char*)in->cores + (size_t)k * ch * 2 * ch * c.csz; };
  HIPCHK(sanitize_bonds(in->bonds, b.bonds, m, (int)ch, b.status, 1, s));
  HIPCHK(unit_rows(b.L[0], b.ldl, count, (int)ch, real, s));
  int cur = 0;
  for (int k = m - 1; k >= 0; --k) {
    // C[p][(r, s)] = sum_r' A_k[r][s][r'] R_p[r']
    r = gemm(c, dx(count), 1, count, dv(c, 2, b.bonds + k), 2, 2 * rb[k], dv(c, 1, b.bonds + k + 1), 1,
             opd(b.L[cur], b.ldl, 0, 1, 0), opd(core(k), 1, 0, 2 * ch, ch), opd(b.C, b.ldc, 0, 2, 1));
    if (r) return r;
    HIPCHK(sample_select(b.C, b.ldc, b.L[cur ^ 1], b.ldl, uniforms, m, k, b.bonds + k, (int)ch, rows, cols, count,
                         real, s));
    cur ^= 1;
  }
  return QTT_OK;
}

size_t tt_eval_points_workspace_size(int n_sites, int chi_cap, int count, int prec) {
  if (n_sites < 2 || (n_sites & 1) || chi_cap < 1 || chi_cap > 256 || count < 1) return 0;
  Carver cv(nullptr);
  carve_eval(cv, n_sites, chi_cap, count, prec == QTT_PREC_FP64 ? 16 : 8);
  return cv.off;
}

int tt_eval_points(const qtt_mps* in, const int32_t* rows, const int32_t* cols, int count, void* out, void* ws,
                   size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if (!rows || !cols || !out || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (count < 1) return fail(QTT_ERR_ARG, "count %d < 1", count);
  const int real = in->dtype == QTT_C128 ? 1 : 0;
  const size_t csz = real ? 16 : 8;
  Carver cv(nullptr);
  carve_eval(cv, in->n_sites, in->chi_cap, count, csz);
  if (ws_bytes < cv.off) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, cv.off);
  Carver cw(ws);
  EvalBufs b = carve_eval(cw, in->n_sites, in->chi_cap, count, csz);
  void* res = nullptr;
  hipStream_t s = (hipStream_t)stream;
  r = eval_rows(view(in), rows, cols, count, in->n_sites, b, s, &res);
  if (r) return r;
  HIPCHK(gather_col0(res, b.ldl, out, count, real, s));
  return QTT_OK;
}

size_t tt_to_dense_block_workspace_size(int n_sites, int chi_cap, int log2_block, int prec) {
  if (n_sites < 2 || (n_sites & 1) || chi_cap < 1 || chi_cap > 256) return 0;
  if (log2_block < 1 || 2 * log2_block > n_sites) return 0;
  const size_t csz = prec == QTT_PREC_FP64 ? 16 : 8;
  Carver cv(nullptr);
  carve_eval(cv, n_sites, chi_cap, 1, csz);
  carve_dense(cv, 2 * log2_block, chi_cap, csz, 1);
  cv.take((size_t)(n_sites + 1) * sizeof(int));
  return cv.off;
}

int tt_to_dense_block(const qtt_mps* in, int log2_block, int block_row, int block_col, void* out, int out_dtype,
                      void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if (!out || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (out_dtype != QTT_C64 && out_dtype != QTT_C128) return fail(QTT_ERR_DTYPE, "out dtype must be C64 or C128");
  const int n = in->n_sites / 2;
  if (log2_block < 1 || log2_block > n) return fail(QTT_ERR_SHAPE, "log2_block %d outside [1, %d]", log2_block, n);
  const long long nblk = 1ll << (n - log2_block);
  if (block_row < 0 || block_col < 0 || block_row >= nblk || block_col >= nblk)
    return fail(QTT_ERR_SHAPE, "block (%d, %d) outside the %lld x %lld grid of blocks", block_row, block_col, nblk, nblk);
  const int real = in->dtype == QTT_C128 ? 1 : 0;
  const size_t csz = real ? 16 : 8;
  const size_t need = tt_to_dense_block_workspace_size(in->n_sites, in->chi_cap, log2_block,
                                                       real ? QTT_PREC_FP64 : QTT_PREC_FP32);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  Carver cw(ws);
  EvalBufs eb = carve_eval(cw, in->n_sites, in->chi_cap, 1, csz);
  DenseBufs db = carve_dense(cw, 2 * log2_block, in->chi_cap, csz, 1);
  db.status = eb.status;
  db.bonds = (int*)cw.take((size_t)(in->n_sites + 1) * sizeof(int));   // bonds of the whole MPS
  hipStream_t s = (hipStream_t)stream;
  const MpsB v = view(in);
  if (log2_block == n) return dense_impl(v, out, out_dtype, db, s);
  const int off = 2 * (n - log2_block);
  HIPCHK(fill_point(eb.pts, eb.pts + 1, (int)((long long)block_row << log2_block), (int)((long long)block_col << log2_block), s));
  void* bnd = nullptr;
  r = eval_rows(v, eb.pts, eb.pts + 1, 1, off, eb, s, &bnd);
  if (r) return r;
  return dense_impl(v, out, out_dtype, db, s, off, bnd, 0);
}

// log2 of the block side a window is assembled from: half the window's
// longer side rounded up to a power of two (at most 3 x 3 blocks, so at most
// 2.25 times the window's pixels are decompressed), within [1, n]
static int window_log2_block(int n, int rows, int cols, int log2_block) {
  if (log2_block > 0) return log2_block;
  const int w = std::max(rows, cols);
  int lb = 1;
  while (lb < n && (1 << (lb + 1)) < w) ++lb;
  return lb;
}

size_t tt_to_dense_window_workspace_size(int n_sites, int chi_cap, int rows, int cols, int log2_block, int prec) {
  if (n_sites < 2 || (n_sites & 1) || rows < 1 || cols < 1) return 0;
  const int n = n_sites / 2;
  const int lb = window_log2_block(n, rows, cols, log2_block);
  if (lb < 1 || lb > n) return 0;
  const size_t wb = tt_to_dense_block_workspace_size(n_sites, chi_cap, lb, prec);
  if (!wb) return 0;
  const size_t csz = prec == QTT_PREC_FP64 ? 16 : 8;
  return (wb + 255) / 256 * 256 + ((size_t)1 << (2 * lb)) * csz;
}

int tt_to_dense_window(const qtt_mps* in, int row0, int col0, int rows, int cols, int log2_block, void* out,
                       int out_dtype, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if (!out || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (out_dtype != QTT_C64 && out_dtype != QTT_C128) return fail(QTT_ERR_DTYPE, "out dtype must be C64 or C128");
  const int n = in->n_sites / 2;
  const long long N = 1ll << n;
  if (rows < 1 || cols < 1 || row0 < 0 || col0 < 0 || row0 + (long long)rows > N || col0 + (long long)cols > N)
    return fail(QTT_ERR_SHAPE, "window (%d, %d) + (%d, %d) outside the %lld x %lld field", row0, col0, rows, cols, N, N);
  const int lb = window_log2_block(n, rows, cols, log2_block);
  if (lb < 1 || lb > n) return fail(QTT_ERR_SHAPE, "log2_block %d outside [1, %d]", lb, n);
  const int prec = in->dtype == QTT_C128 ? QTT_PREC_FP64 : QTT_PREC_FP32;
  const size_t need = tt_to_dense_window_workspace_size(in->n_sites, in->chi_cap, rows, cols, log2_block, prec);
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  const size_t wb = (tt_to_dense_block_workspace_size(in->n_sites, in->chi_cap, lb, prec) + 255) / 256 * 256;
  char* blk = (char*)ws + wb;
  const size_t osz = out_dtype == QTT_C128 ? 16 : 8;
  const long long side = 1ll << lb;
  hipStream_t s = (hipStream_t)stream;
  for (long long br = row0 / side; br <= (row0 + rows - 1) / side; ++br) {
    for (long long bc = col0 / side; bc <= (col0 + cols - 1) / side; ++bc) {
      if ((r = tt_to_dense_block(in, lb, (int)br, (int)bc, blk, out_dtype, ws, wb, stream))) return r;
      const long long r0 = br * side, c0 = bc * side;
      const long long ra = std::max<long long>(row0, r0), rb = std::min<long long>(row0 + rows, r0 + side);
      const long long ca = std::max<long long>(col0, c0), cb = std::min<long long>(col0 + cols, c0 + side);
      const int nr = (int)(rb - ra), nc = (int)(cb - ca);
      HIPCHK(block_copy(blk + ((ra - r0) * side + (ca - c0)) * osz, side, 1,
                        (char*)out + ((ra - row0) * cols + (ca - col0)) * osz, cols, 1, dx(nr), dx(nc), nr, nc,
                        out_dtype == QTT_C128 ? 1 : 0, s));
    }
  }
  return QTT_OK;
}

int tt_cgemm(int M, int N, int K, const void* A, int lda, int conj_a, const void* B, int ldb, int conj_b, void* C,
             int ldc, int prec, void* stream) {
  g_err.clear();
  if (!A || !B || !C) return fail(QTT_ERR_ARG, "NULL operand");
  if (M < 1 || N < 1 || K < 1 || lda < K || ldb < N || ldc < N) return fail(QTT_ERR_SHAPE, "bad GEMM shape");
  if (prec != QTT_PREC_FP32 && prec != QTT_PREC_FP64 && prec != QTT_PREC_BF16 && prec != QTT_PREC_BF16X3)
    return fail(QTT_ERR_ARG, "precision %d not supported", prec);
  GemmSpec g;
  g.M = dx(M); g.N = dx(N); g.K = dx(K); g.batch = dx(1);
  g.mlo = g.nlo = g.klo = 1;
  g.m_bound = M; g.n_bound = N; g.batch_bound = 1; g.k_bound = K;
  g.A = opd(A, lda, 0, 1, 0, conj_a);
  g.B = opd(B, ldb, 0, 1, 0, conj_b);
  g.C = opd(C, ldc, 0, 1, 0);
  g.types = prec == QTT_PREC_FP64 ? GEMM_F64
            : prec == QTT_PREC_BF16 ? GEMM_BF16
            : prec == QTT_PREC_BF16X3 ? GEMM_BF16X3 : GEMM_F32;
  HIPCHK(gemm_launch(g, (hipStream_t)stream));
  return QTT_OK;
}

size_t tt_heev_workspace_size(int n, int kcap, int batch) {
  if (n < 1 || n > 512 || kcap < 1 || batch < 1) return 0;
  return 256 + eig_ws_bytes(n, kcap, batch) + 256;
}

int tt_heev(void* G, int n, int batch, int kcap, double cutoff, double tau, int* kept, double* evals, void* evecs,
            void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!G || !kept || !ws) return fail(QTT_ERR_ARG, "NULL argument");
  if (n < 1 || n > 512) return fail(QTT_ERR_SHAPE, "n %d outside [1, 512]", n);
  if (kcap < 1 || batch < 1) return fail(QTT_ERR_ARG, "bad kcap/batch");
  if (ws_bytes < tt_heev_workspace_size(n, kcap, batch)) return fail(QTT_ERR_WORKSPACE, "workspace too small");
  int kc = std::min(kcap, n);
  EigSpec e;
  e.G = (double*)G; e.ld = n; e.gstride = (ll)n * n;
  e.n = dx(n); e.n_bound = n; e.kcap = kc;
  e.cutoff = cutoff; e.tau = tau > 0.0 ? tau : 1e-13;
  e.kout = kept; e.kstride = 1; e.batch = batch;
  e.status = (int*)ws;
  e.ws = (char*)ws + 256;
  e.nemit = 0;
  if (evecs) e.emit[e.nemit++] = emit(evecs, 1, kcap, 0, 1, 0, 0, 1);
  if (evecs) e.emit[0].s_batch = (ll)n * kcap;
  e.sigma_out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(eig_launch(e, s));
  if (evals) HIPCHK(eig_copy_evals(e, evals, kcap, s));
  return QTT_OK;
}

static int prof_events(int max_launches) {
  if (g_prof.ev) {
    for (int i = 0; i < 2 * g_prof.max_launches; ++i) hipEventDestroy(g_prof.ev[i]);
    delete[] g_prof.ev;
    g_prof.ev = nullptr;
  }
  g_prof.ev = new hipEvent_t[2 * (size_t)max_launches];
  for (int i = 0; i < 2 * max_launches; ++i) HIPCHK(hipEventCreate(&g_prof.ev[i]));
  g_prof.slot = 0;
  g_prof.launches = 0;
  g_prof.max_launches = max_launches;
  return QTT_OK;
}

int tt_prof_begin(int what, int* nlog, int max_entries, int max_launches) {
  g_err.clear();
  if ((what != PROF_TRIDIAG && what != PROF_TRIDIAG_LDS) || !nlog || max_entries < 1 || max_launches < 1)
    return fail(QTT_ERR_ARG, "tt_prof_begin: bad arguments");
  const int rc = prof_events(max_launches);
  if (rc != QTT_OK) return rc;
  g_prof.what = what;
  g_prof.nlog = nlog;
  g_prof.flog = nullptr;
  g_prof.max = max_entries;
  return QTT_OK;
}

int tt_prof_begin_flops(double* flog, int max_launches) {
  g_err.clear();
  if (!flog || max_launches < 1) return fail(QTT_ERR_ARG, "tt_prof_begin_flops: bad arguments");
  const int rc = prof_events(max_launches);
  if (rc != QTT_OK) return rc;
  g_prof.what = PROF_GEMM;
  g_prof.nlog = nullptr;
  g_prof.flog = flog;
  g_prof.max = 0;
  return QTT_OK;
}

int tt_prof_times(float* ms, int max) {
  g_err.clear();
  if (!ms || max < 0) return fail(QTT_ERR_ARG, "tt_prof_times: bad arguments");
  const int n = std::min(max, g_prof.launches);
  for (int i = 0; i < n; ++i) {
    HIPCHK(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    HIPCHK(hipEventElapsedTime(&ms[i], g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
  }
  return n;
}

int tt_prof_end(int* launches, int* entries, double* total_ms) {
  g_err.clear();
  double tot = 0.0;
  for (int i = 0; i < g_prof.launches; ++i) {
    HIPCHK(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
    tot += ms;
  }
  if (launches) *launches = g_prof.launches;
  if (entries) *entries = g_prof.slot;
  if (total_ms) *total_ms = tot;
  g_prof.what = PROF_NONE;
  return QTT_OK;
}

int tt_autotune_record(int on) {
  g_err.clear();
  autotune_record(on != 0);
  return QTT_OK;
}

size_t tt_autotune_workspace_size(void) { return autotune_ws_bytes() + 256; }

int tt_autotune_run(void* ws, size_t ws_bytes, void* stream, int* n_tuned) {
  g_err.clear();
  const size_t need = autotune_ws_bytes();
  if (!ws && need > 0) return fail(QTT_ERR_ARG, "workspace is NULL");
  if (ws_bytes < need) return fail(QTT_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  if (need > 0) HIPCHK(zero_fill(ws, need / 16 * 16, s));
  HIPCHK(autotune_run(ws, ws_bytes, s, n_tuned));
  return QTT_OK;
}

int tt_autotune_export(int32_t* entries, int max_entries) {
  g_err.clear();
  if (max_entries < 0) return fail(QTT_ERR_ARG, "max_entries < 0");
  return autotune_export(entries, max_entries);
}

int tt_autotune_import(const int32_t* entries, int n) {
  g_err.clear();
  if (n < 0 || (n > 0 && !entries)) return fail(QTT_ERR_ARG, "bad entries");
  int bad = autotune_import(entries, n);
  if (bad) return fail(QTT_ERR_ARG, "%d invalid entries ignored", bad);
  return QTT_OK;
}

int tt_autotune_clear(void) {
  g_err.clear();
  autotune_clear();
  return QTT_OK;
}

}  // extern "C"

// ---- allocation-free application --------------------------------------------
// The workspace of mpo_apply_noalloc is this file-scope device array: every
// GPU the library runs on holds its own copy (QTT_NOALLOC_SCRATCH_BYTES) until
// the process ends, and every call on that GPU reuses it.  In host code the
// array's name is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace {
__device__ __align__(256) unsigned char scratch[QTT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_ptr(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(QTT_ERR_ARG, "device %d outside [0, %d)", dev, kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(QTT_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    if (!p) return fail(QTT_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QTT_OK;
}
}  // namespace

extern "C" {

int mpo_apply_noalloc(const qtt_mps* in, const qtt_mpo* W, const qtt_opts* opts, qtt_mps* out,
                      int32_t* status_out, void* stream) {
  g_err.clear();
  int r;
  if ((r = check_mps(in, "in"))) return r;
  if ((r = check_mps(out, "out"))) return r;
  if (in->cores == out->cores) return fail(QTT_ERR_ARG, "in and out must not alias");
  if (!W) return fail(QTT_ERR_ARG, "MPO is NULL");
  ApplySetup su;
  if ((r = apply_setup(view(in), W, nullptr, opts, view(out), false, su))) return r;
  const size_t need = apply_bytes(su.p, su.csz, 1);
  if (need > QTT_NOALLOC_SCRATCH_BYTES)
    return fail(QTT_ERR_WORKSPACE, "mpo_apply_noalloc: this problem needs %zu bytes of scratch, the static "
                "scratch holds %zu (use mpo_apply with a caller workspace)", need, (size_t)QTT_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((r = scratch_ptr(&ws))) return r;
  hipStream_t s = (hipStream_t)stream;
  // the status word starts at zero on every call (a fill kernel, not a
  // memset node, so the call can be captured into a graph)
  HIPCHK(zero_fill(ws, 256, s));
  if ((r = apply_common(view(in), W, nullptr, opts, view(out), nullptr, ws, QTT_NOALLOC_SCRATCH_BYTES, stream,
                        false)))
    return r;
  if (status_out) HIPCHK(copy_ints((const int*)ws, status_out, 1, s));
  return QTT_OK;
}

int tt_check_status(void* ws, void* stream) {
  g_err.clear();
  if (!ws) return fail(QTT_ERR_ARG, "workspace is NULL");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(QTT_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
  int st = 0;
  e = hipMemcpy(&st, ws, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(QTT_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
  int zero = 0;
  e = hipMemcpy(ws, &zero, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(QTT_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
  if (st != 0) return fail(st, "device status %d", st);
  return QTT_OK;
}

}  // extern "C"
