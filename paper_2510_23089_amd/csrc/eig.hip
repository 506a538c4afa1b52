// Batched FP64 Hermitian eigensolver for bond truncation.
//
// Every truncation of the path (zip-up, sweep, encode) needs the dominant
// eigenpairs of a Gram matrix G = M^H M (or M M^H) of size <= 2*chi: the
// squared singular values decide the kept rank (Sec. 4: each bond is a
// Schmidt cut) and the eigenvectors give the kept singular subspace.  Stages,
// one kernel each, all stream-ordered with device-side sizes:
//   1. tridiag   Householder reduction to real tridiagonal form, one
//                workgroup per matrix; the rank-2 update of step j is fused
//                with the matrix-vector product of step j+1 so the trailing
//                matrix is streamed once per step (column-per-thread, rows
//                read coalesced).  Reflectors are kept in the upper triangle.
//   2. eigvals   the top min(n, cap) eigenvalues, one wave per eigenvalue:
//                64-way multisection on Sturm counts (division-free
//                three-term recurrence with exponent rescaling), so a wave
//                narrows the interval by 64x per pass.
//   3. keep      the keep rule (cap, relative discarded weight, tau) and the
//                non-finite check; writes the bond dimension.
//   4. inviter   inverse iteration, one lane per kept eigenvector, tridiagonal
//                LU with partial pivoting in per-lane (coalesced) scratch.
//   5. cluster   Gram-Schmidt (twice) inside clusters of near-equal
//                eigenvalues, where inverse iteration alone is not orthogonal.
//   6. backtr    back-transformation by the reflectors, one wave per vector,
//                and emission of the layouts the caller needs (conjugated,
//                scaled by sigma^{+-1}, cast to complex64 or kept FP64).
#include "common.h"
#include "kernels.h"

namespace qtt {

constexpr int EIG_NMAX = 512;       // largest Gram matrix (2 * chi_cap, chi_cap <= 256)
constexpr int TRI_NT = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {   // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Per-matrix scratch layout inside the eigen workspace.
struct EigWs {
  double *d, *e, *e2, *lam, *sig;
  double2* tau;
  double *lu_dl, *lu_d, *lu_du, *lu_du2, *z;
  int* piv;
  int* clus;
};

__host__ __device__ inline size_t eig_ws_per_matrix(int nb, int kc) {
  size_t s = 0;
  s += 5 * (size_t)nb * sizeof(double);          // d, e, e2, lam, sig
  s += (size_t)nb * sizeof(double2);             // tau
  s += 5 * (size_t)nb * kc * sizeof(double);     // LU (4) + z
  s += (size_t)nb * kc * sizeof(int);            // pivots
  s += (size_t)kc * sizeof(int);                 // cluster starts
  return (s + 255) / 256 * 256;
}

__host__ __device__ inline EigWs eig_ws_carve(void* base, int b, int nb, int kc) {
  char* p = (char*)base + (size_t)b * eig_ws_per_matrix(nb, kc);
  EigWs w;
  w.d = (double*)p; p += nb * sizeof(double);
  w.e = (double*)p; p += nb * sizeof(double);
  w.e2 = (double*)p; p += nb * sizeof(double);
  w.lam = (double*)p; p += nb * sizeof(double);
  w.sig = (double*)p; p += nb * sizeof(double);
  w.tau = (double2*)p; p += nb * sizeof(double2);
  w.lu_dl = (double*)p; p += (size_t)nb * kc * sizeof(double);
  w.lu_d = (double*)p; p += (size_t)nb * kc * sizeof(double);
  w.lu_du = (double*)p; p += (size_t)nb * kc * sizeof(double);
  w.lu_du2 = (double*)p; p += (size_t)nb * kc * sizeof(double);
  w.z = (double*)p; p += (size_t)nb * kc * sizeof(double);
  w.piv = (int*)p; p += (size_t)nb * kc * sizeof(int);
  w.clus = (int*)p;
  return w;
}

// ------------------------------------------------------------ 1. tridiag
__global__ __launch_bounds__(TRI_NT) void tridiag_kernel(double2* Gall, int ld, long long gstride, DimExpr nexp,
                                                         void* wsbase, int nb, int kc) {
  const int b = blockIdx.x;
  const int n = dim_eval(nexp);
  double2* A = Gall + (long long)b * gstride;
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  __shared__ double2 vp[EIG_NMAX], wp[EIG_NMAX], vn[EIG_NMAX], pn[EIG_NMAX];
  __shared__ double red[TRI_NT / 64];
  __shared__ double2 s_tau, s_scale;
  __shared__ double s_beta;
  const int tid = threadIdx.x;
  bool pending = false;
  for (int j = 0; j < n - 1; ++j) {
    const int j1 = j + 1;
    // (a) finish row j with the pending rank-2 update of step j-1
    for (int c = j + tid; c < n; c += TRI_NT) {
      double2 a = A[(long long)j * ld + c];
      if (pending) {
        a = csub(a, cmul(vp[j], make_double2(wp[c].x, -wp[c].y)));
        a = csub(a, cmul(wp[j], make_double2(vp[c].x, -vp[c].y)));
      }
      A[(long long)j * ld + c] = a;
      if (c == j && false) {}
    }
    __syncthreads();
    // (b) reflector annihilating column j below the subdiagonal
    //     (column j = conj(row j) by Hermiticity)
    double loc = 0.0;
    for (int c = j1 + 1 + tid; c < n; c += TRI_NT) {
      double2 a = A[(long long)j * ld + c];
      loc += a.x * a.x + a.y * a.y;
    }
    double xnorm2 = block_sum<TRI_NT>(loc, red);
    if (tid == 0) {
      W.d[j] = A[(long long)j * ld + j].x;
      double2 a = A[(long long)j * ld + j1];
      double2 alpha = make_double2(a.x, -a.y);
      double2 tau, scale;
      double beta;
      if (xnorm2 == 0.0 && alpha.y == 0.0) {
        tau = make_double2(0.0, 0.0);
        beta = alpha.x;
        scale = make_double2(0.0, 0.0);
      } else {
        double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        double2 den = make_double2(alpha.x - beta, alpha.y);
        double dd = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dd, -den.y / dd);
      }
      s_tau = tau;
      s_scale = scale;
      s_beta = beta;
      W.e[j] = beta;
      W.e2[j] = beta * beta;
      W.tau[j] = tau;
    }
    __syncthreads();
    const double2 tau = s_tau, scale = s_scale;
    for (int c = j1 + tid; c < n; c += TRI_NT) {
      double2 v;
      if (c == j1) {
        v = make_double2(1.0, 0.0);
      } else {
        double2 a = A[(long long)j * ld + c];
        v = cmul(make_double2(a.x, -a.y), scale);
        A[(long long)j * ld + c] = v;            // reflector stored in row j
      }
      vn[c] = v;
    }
    __syncthreads();
    // (c) fused pass over the trailing block: apply the pending update and
    //     accumulate p = tau * A v (A Hermitian: (A v)_c = sum_r conj(A[r][c]) v_r)
    for (int c = j1 + tid; c < n; c += TRI_NT) {
      double2 acc = make_double2(0.0, 0.0);
      const double2 wpc = make_double2(wp[c].x, -wp[c].y);
      const double2 vpc = make_double2(vp[c].x, -vp[c].y);
#pragma unroll 4
      for (int r = j1; r < n; ++r) {
        double2 a = A[(long long)r * ld + c];
        if (pending) {
          a = csub(a, cmul(vp[r], wpc));
          a = csub(a, cmul(wp[r], vpc));
          A[(long long)r * ld + c] = a;
        }
        acc = cadd(acc, cmulc(a, vn[r]));
      }
      pn[c] = cmul(tau, acc);
    }
    __syncthreads();
    // (d) w = p - (tau/2)(p^H v) v  -> becomes the pending update
    double lre = 0.0, lim = 0.0;
    for (int c = j1 + tid; c < n; c += TRI_NT) {
      double2 q = cmulc(pn[c], vn[c]);
      lre += q.x;
      lim += q.y;
    }
    double dre = block_sum<TRI_NT>(lre, red);
    double dim_ = block_sum<TRI_NT>(lim, red);
    double2 alpha2 = cmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), make_double2(dre, dim_));
    for (int c = j1 + tid; c < n; c += TRI_NT) {
      wp[c] = cadd(pn[c], cmul(alpha2, vn[c]));
      vp[c] = vn[c];
    }
    pending = (tau.x != 0.0 || tau.y != 0.0);
    __syncthreads();
  }
  if (tid == 0 && n >= 1) {
    double2 a = A[(long long)(n - 1) * ld + (n - 1)];
    if (pending && n >= 2) {
      double2 t1 = cmul(vp[n - 1], make_double2(wp[n - 1].x, -wp[n - 1].y));
      double2 t2 = cmul(wp[n - 1], make_double2(vp[n - 1].x, -vp[n - 1].y));
      a = csub(csub(a, t1), t2);
    }
    W.d[n - 1] = a.x;
  }
}

// ------------------------------------------------------------ 2. eigenvalues
// Number of eigenvalues of the symmetric tridiagonal (d, e2 = e^2) below x.
__device__ int sturm_count(const double* d, const double* e2, int n, double x) {
  double p0 = 1.0, p1 = d[0] - x;
  int sprev = p1 > 0.0 ? 1 : -1;
  int cnt = sprev < 0 ? 1 : 0;
  for (int i = 1; i < n; ++i) {
    double p2 = fma(d[i] - x, p1, -e2[i - 1] * p0);
    int s = p2 > 0.0 ? 1 : (p2 < 0.0 ? -1 : -sprev);
    cnt += (s != sprev);
    sprev = s;
    p0 = p1;
    p1 = p2;
    if ((i & 7) == 0) {
      double m = fmax(fabs(p0), fabs(p1));
      if (m > 0x1p+600 || (m < 0x1p-600 && m > 0.0)) {
        int ex = ilogb(m);
        p0 = ldexp(p0, -ex);
        p1 = ldexp(p1, -ex);
      }
    }
  }
  return cnt;
}

constexpr int EV_NT = 256;
__global__ __launch_bounds__(EV_NT) void eigvals_kernel(DimExpr nexp, int kcap, void* wsbase, int nb, int kc) {
  const int b = blockIdx.y;
  const int n = dim_eval(nexp);
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  __shared__ double sd[EIG_NMAX], se2[EIG_NMAX];
  for (int i = threadIdx.x; i < n; i += EV_NT) {
    sd[i] = W.d[i];
    se2[i] = i < n - 1 ? W.e2[i] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (EV_NT / 64) + (threadIdx.x >> 6);
  const int kmax = min(n, kcap);
  if (t >= kmax) return;
  // Gershgorin interval
  double glo = 1e300, ghi = -1e300;
  for (int i = lane; i < n; i += 64) {
    double r = 0.0;
    if (i > 0) r += sqrt(se2[i - 1]);
    if (i < n - 1) r += sqrt(se2[i]);
    glo = fmin(glo, sd[i] - r);
    ghi = fmax(ghi, sd[i] + r);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o));
    ghi = fmax(ghi, __shfl_xor(ghi, o));
  }
  const double gn = fmax(fabs(glo), fabs(ghi));
  const double pad = 2.2e-16 * gn * n + 1e-300;
  double lo = glo - pad, hi = ghi + pad;
  const double tol_abs = 1e-19 * gn + 1e-300;
  const int target = n - 1 - t;               // ascending index of the t-th largest
  for (int it = 0; it < 40; ++it) {
    double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
    int c = sturm_count(sd, se2, n, x);
    unsigned long long mask = __ballot(c > target);
    int first = mask ? __ffsll((long long)mask) - 1 : 64;
    double xf = __shfl(x, first < 64 ? first : 63);
    double xp = __shfl(x, first > 0 ? first - 1 : 0);
    double nhi = first < 64 ? xf : hi;
    double nlo = first > 0 ? xp : lo;
    lo = nlo;
    hi = nhi;
    if (hi - lo <= fmax(4.4e-16 * fmax(fabs(lo), fabs(hi)), tol_abs)) break;
  }
  if (lane == 0) W.lam[t] = 0.5 * (lo + hi);
}

// ------------------------------------------------------------ 3. keep rule
__global__ void keep_kernel(DimExpr nexp, int kcap, double cutoff, double tau, int* kout, long long kstride,
                            void* wsbase, int nb, int kc, int batch, int* status, double* sigma_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int n = dim_eval(nexp);
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  const int kmax = min(n, kcap);
  double total = 0.0;
  for (int i = 0; i < n; ++i) total += W.d[i];
  const double l0 = W.lam[0];
  int k = 0;
  bool bad = !isfinite(l0) || !isfinite(total);
  if (!bad && l0 > 0.0) {
    for (int t = 0; t < kmax; ++t) {
      if (W.lam[t] > tau * l0) k = t + 1;
      else break;
    }
    if (cutoff > 0.0) {
      double kept = 0.0;
      for (int t = 0; t < k; ++t) {
        kept += fmax(W.lam[t], 0.0);
        if (total - kept <= cutoff * total) { k = t + 1; break; }
      }
    }
  }
  if (bad) set_status(status, ST_NONFINITE);
  if (k < 1) k = 1;
  for (int t = 0; t < kmax; ++t) {
    double s = W.lam[t] > 0.0 ? sqrt(W.lam[t]) : 0.0;
    W.sig[t] = s;
    if (sigma_out) sigma_out[(long long)b * kcap + t] = t < k ? s : 0.0;
  }
  kout[b * kstride] = k;
}

// ------------------------------------------------------------ 4. inverse iteration
__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)h / 4294967296.0) - 0.5;
}

__global__ __launch_bounds__(64) void inviter_kernel(DimExpr nexp, int* kin, long long kstride, void* wsbase,
                                                     int nb, int kc) {
  const int b = blockIdx.y;
  const int n = dim_eval(nexp);
  const int k = kin[b * kstride];
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= k) return;
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  const double mu = W.lam[t];
  const double tn = fmax(fabs(W.lam[0]), 1e-300);
  const double pivmin = 1e-300 + 2.2e-16 * tn * 1e-3;
  // strided per-lane arrays: element i of lane t at i*kc + t
#define IX(i) ((long long)(i) * kc + t)
  double* DL = W.lu_dl;
  double* D = W.lu_d;
  double* DU = W.lu_du;
  double* DU2 = W.lu_du2;
  double* X = W.z;
  int* P = W.piv;
  if (n == 1) { X[IX(0)] = 1.0; return; }
  for (int i = 0; i < n; ++i) {
    D[IX(i)] = W.d[i] - mu;
    if (i < n - 1) { DL[IX(i)] = W.e[i]; DU[IX(i)] = W.e[i]; }
  }
  // LU with partial pivoting (tridiagonal)
  for (int i = 0; i < n - 1; ++i) {
    double di = D[IX(i)], dli = DL[IX(i)];
    if (fabs(di) >= fabs(dli)) {
      if (di == 0.0) { di = pivmin; D[IX(i)] = di; }
      double f = dli / di;
      DL[IX(i)] = f;
      D[IX(i + 1)] -= f * DU[IX(i)];
      if (i < n - 2) DU2[IX(i)] = 0.0;
      P[IX(i)] = 0;
    } else {
      double f = di / dli;
      D[IX(i)] = dli;
      DL[IX(i)] = f;
      double tmp = DU[IX(i)];
      DU[IX(i)] = D[IX(i + 1)];
      D[IX(i + 1)] = tmp - f * D[IX(i + 1)];
      if (i < n - 2) {
        DU2[IX(i)] = DU[IX(i + 1)];
        DU[IX(i + 1)] = -f * DU[IX(i + 1)];
      }
      P[IX(i)] = 1;
    }
  }
  if (D[IX(n - 1)] == 0.0) D[IX(n - 1)] = pivmin;
  for (int i = 0; i < n; ++i) X[IX(i)] = hash_unit(t + 1, i + 7 * b);
  for (int it = 0; it < 3; ++it) {
    // forward: L
    for (int i = 0; i < n - 1; ++i) {
      if (P[IX(i)] == 0) {
        X[IX(i + 1)] -= DL[IX(i)] * X[IX(i)];
      } else {
        double tmp = X[IX(i)];
        X[IX(i)] = X[IX(i + 1)];
        X[IX(i + 1)] = tmp - DL[IX(i)] * X[IX(i)];
      }
    }
    // backward: U
    double mx = 0.0;
    X[IX(n - 1)] /= D[IX(n - 1)];
    mx = fabs(X[IX(n - 1)]);
    X[IX(n - 2)] = (X[IX(n - 2)] - DU[IX(n - 2)] * X[IX(n - 1)]) / D[IX(n - 2)];
    mx = fmax(mx, fabs(X[IX(n - 2)]));
    for (int i = n - 3; i >= 0; --i) {
      X[IX(i)] = (X[IX(i)] - DU[IX(i)] * X[IX(i + 1)] - DU2[IX(i)] * X[IX(i + 2)]) / D[IX(i)];
      mx = fmax(mx, fabs(X[IX(i)]));
    }
    double sc = mx > 0.0 && isfinite(mx) ? 1.0 / mx : 1.0;
    for (int i = 0; i < n; ++i) X[IX(i)] *= sc;
  }
  double s2 = 0.0;
  for (int i = 0; i < n; ++i) s2 += X[IX(i)] * X[IX(i)];
  double sc = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  for (int i = 0; i < n; ++i) X[IX(i)] *= sc;
#undef IX
}

// ------------------------------------------------------------ 5. clusters
constexpr int CL_NT = 256;
__global__ __launch_bounds__(CL_NT) void cluster_kernel(DimExpr nexp, int* kin, long long kstride, void* wsbase,
                                                        int nb, int kc, double reltol) {
  const int b = blockIdx.x;
  const int n = dim_eval(nexp);
  const int k = kin[b * kstride];
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  __shared__ double red[CL_NT / 64];
  __shared__ double coef[EIG_NMAX];
  const double tn = fabs(W.lam[0]);
  int cs = 0;
  for (int t = 1; t < k; ++t) {
    if (W.lam[t - 1] - W.lam[t] > reltol * tn) { cs = t; continue; }
    // t belongs to the cluster [cs, t]: orthogonalise twice against [cs, t)
    for (int pass = 0; pass < 2; ++pass) {
      for (int s = cs; s < t; ++s) {
        double loc = 0.0;
        for (int i = threadIdx.x; i < n; i += CL_NT) loc += W.z[(long long)i * kc + s] * W.z[(long long)i * kc + t];
        double dot = block_sum<CL_NT>(loc, red);
        if (threadIdx.x == 0) coef[s] = dot;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += CL_NT) {
        double v = W.z[(long long)i * kc + t];
        for (int s = cs; s < t; ++s) v -= coef[s] * W.z[(long long)i * kc + s];
        W.z[(long long)i * kc + t] = v;
      }
      __syncthreads();
    }
    double loc = 0.0;
    for (int i = threadIdx.x; i < n; i += CL_NT) {
      double v = W.z[(long long)i * kc + t];
      loc += v * v;
    }
    double nrm = sqrt(block_sum<CL_NT>(loc, red));
    double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = threadIdx.x; i < n; i += CL_NT) W.z[(long long)i * kc + t] *= sc;
    __syncthreads();
  }
}

// ------------------------------------------------------------ 6. back-transform + emit
struct EmitPack {
  EigEmit e[3];
  int ne;
};

constexpr int BT_NT = 256;
constexpr int BT_PER_LANE = EIG_NMAX / 64;
__global__ __launch_bounds__(BT_NT) void backtr_kernel(const double2* Gall, int ld, long long gstride,
                                                       DimExpr nexp, int* kin, long long kstride, void* wsbase,
                                                       int nb, int kc, EmitPack ep) {
  const int b = blockIdx.y;
  const int n = dim_eval(nexp);
  const int k = kin[b * kstride];
  const int t = blockIdx.x * (BT_NT / 64) + (threadIdx.x >> 6);
  if (t >= k) return;
  const int lane = threadIdx.x & 63;
  const double2* A = Gall + (long long)b * gstride;
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  double2 v[BT_PER_LANE];
#pragma unroll
  for (int q = 0; q < BT_PER_LANE; ++q) {
    int i = lane + 64 * q;
    v[q] = make_double2(i < n ? W.z[(long long)i * kc + t] : 0.0, 0.0);
  }
  for (int j = n - 2; j >= 0; --j) {
    const double2 tau = W.tau[j];
    if (tau.x == 0.0 && tau.y == 0.0) continue;
    const int j1 = j + 1;
    double2 u[BT_PER_LANE];
    double dre = 0.0, dim_ = 0.0;
#pragma unroll
    for (int q = 0; q < BT_PER_LANE; ++q) {
      int i = lane + 64 * q;
      double2 uu = make_double2(0.0, 0.0);
      if (i == j1) uu = make_double2(1.0, 0.0);
      else if (i > j1 && i < n) uu = A[(long long)j * ld + i];
      u[q] = uu;
      double2 p = cmulc(uu, v[q]);
      dre += p.x;
      dim_ += p.y;
    }
    dre = wave_sum(dre);
    dim_ = wave_sum(dim_);
    const double2 f = cmul(tau, make_double2(dre, dim_));
#pragma unroll
    for (int q = 0; q < BT_PER_LANE; ++q) v[q] = csub(v[q], cmul(f, u[q]));
  }
  const double sg = W.sig[t];
  for (int e = 0; e < ep.ne; ++e) {
    const EigEmit& em = ep.e[e];
    double sc = 1.0;
    if (em.pow == 1) sc = sg;
    else if (em.pow == -1) sc = sg > 0.0 ? 1.0 / sg : 0.0;
    char* base = (char*)em.ptr;
#pragma unroll
    for (int q = 0; q < BT_PER_LANE; ++q) {
      int i = lane + 64 * q;
      if (i >= n) continue;
      double2 x = make_double2(v[q].x * sc, (em.conj ? -v[q].y : v[q].y) * sc);
      int h = i / em.lo, l = i - h * em.lo;
      long long off = (long long)b * em.s_batch + (long long)h * em.s_hi + (long long)l * em.s_lo +
                      (long long)t * em.s_col;
      if (em.dtype == 0) ((float2*)base)[off] = make_float2((float)x.x, (float)x.y);
      else ((double2*)base)[off] = x;
    }
  }
}

// Kept eigenvalues to a caller array (zero beyond the kept count).
__global__ void copy_evals_kernel(DimExpr nexp, int kcap, int* kin, long long kstride, void* wsbase, int nb, int kc,
                                  double* out, int ldo) {
  const int b = blockIdx.x;
  const int k = kin[b * kstride];
  EigWs W = eig_ws_carve(wsbase, b, nb, kc);
  for (int t = threadIdx.x; t < ldo; t += blockDim.x) out[(long long)b * ldo + t] = t < k ? W.lam[t] : 0.0;
}

// ---------------------------------------------------------------- host

size_t eig_ws_bytes(int n_bound, int kcap, int batch) {
  int kc = kcap < n_bound ? kcap : n_bound;
  if (kc < 1) kc = 1;
  return eig_ws_per_matrix(n_bound, kc) * (size_t)batch;
}

hipError_t eig_launch(const EigSpec& sp, hipStream_t s) {
  const int nb = sp.n_bound;
  if (nb < 1 || nb > EIG_NMAX || sp.batch < 1) return hipErrorInvalidValue;
  const int kc = sp.kcap < nb ? sp.kcap : nb;
  const double tau = sp.tau > 0.0 ? sp.tau : 1e-13;
  hipLaunchKernelGGL(tridiag_kernel, dim3(sp.batch), dim3(TRI_NT), 0, s, (double2*)sp.G, sp.ld, sp.gstride,
                     sp.n, sp.ws, nb, kc);
  hipLaunchKernelGGL(eigvals_kernel, dim3((kc + 3) / 4, sp.batch), dim3(EV_NT), 0, s, sp.n, kc, sp.ws, nb, kc);
  hipLaunchKernelGGL(keep_kernel, dim3((sp.batch + 63) / 64), dim3(64), 0, s, sp.n, kc, sp.cutoff, tau, sp.kout,
                     sp.kstride, sp.ws, nb, kc, sp.batch, sp.status, sp.sigma_out);
  hipLaunchKernelGGL(inviter_kernel, dim3((kc + 63) / 64, sp.batch), dim3(64), 0, s, sp.n, sp.kout, sp.kstride,
                     sp.ws, nb, kc);
  // inverse-iteration vectors are orthogonal to ~eps*||T||/gap: re-orthogonalise
  // runs of eigenvalues closer than 1e-8 ||T||
  hipLaunchKernelGGL(cluster_kernel, dim3(sp.batch), dim3(CL_NT), 0, s, sp.n, sp.kout, sp.kstride, sp.ws, nb, kc,
                     1e-8);
  EmitPack ep;
  ep.ne = sp.nemit;
  for (int i = 0; i < sp.nemit && i < 3; ++i) ep.e[i] = sp.emit[i];
  hipLaunchKernelGGL(backtr_kernel, dim3((kc + 3) / 4, sp.batch), dim3(BT_NT), 0, s, (const double2*)sp.G, sp.ld,
                     sp.gstride, sp.n, sp.kout, sp.kstride, sp.ws, nb, kc, ep);
  return hipGetLastError();
}

hipError_t eig_copy_evals(const EigSpec& sp, double* out, int ldo, hipStream_t s) {
  const int nb = sp.n_bound;
  const int kc = sp.kcap < nb ? sp.kcap : nb;
  hipLaunchKernelGGL(copy_evals_kernel, dim3(sp.batch), dim3(64), 0, s, sp.n, kc, sp.kout, sp.kstride, sp.ws, nb, kc,
                     out, ldo);
  return hipGetLastError();
}

}  // namespace qtt
