// Element-wise and reduction kernels of libqtt: the quantics index map of
// Sec. 3 (row-major image <-> bit-interleaved vector), block copies, FP64
// Frobenius norms and the non-finite scan.
#include "common.h"
#include <algorithm>

#include "kernels.h"

namespace qtt {

// Compact the bits at even positions of x (bit 2q -> bit q).
__device__ __forceinline__ uint32_t compact_even(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}
// Spread the bits of x (bit q -> bit 2q).
__device__ __forceinline__ uint32_t spread_even(uint32_t x) {
  x &= 0x0000FFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

__device__ __forceinline__ void load_elem(const void* p, int dtype, long long i, double& re, double& im) {
  switch (dtype) {
    case 1: { float2 v = ((const float2*)p)[i]; re = v.x; im = v.y; break; }      // C64
    case 2: { double2 v = ((const double2*)p)[i]; re = v.x; im = v.y; break; }    // C128
    case 3: { re = ((const float*)p)[i]; im = 0.0; break; }                       // F32
    default: { re = ((const double*)p)[i]; im = 0.0; break; }                     // F64
  }
}
__device__ __forceinline__ void store_elem(void* p, int dtype, long long i, double re, double im) {
  if (dtype == 1) ((float2*)p)[i] = make_float2((float)re, (float)im);
  else ((double2*)p)[i] = make_double2(re, im);
}

// dir 0: dst[q] = src[a*N + b]  (q = quantics index of pixel (a, b))
// dir 1: dst[a*N + b] = src[q]
// The quantics index interleaves a_1 b_1 a_2 b_2 ... (a bits at odd positions
// counted from the least significant bit, b bits at even positions).
__global__ void quantics_kernel(const void* src, int sdt, void* dst, int ddt, int n, long long total, int dir,
                                long long s_src, long long s_dst) {
  // field blockIdx.y: element offsets f * s_src / f * s_dst
  const long long fs = blockIdx.y * s_src, fd = blockIdx.y * s_dst;
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    long long in;
    if (dir == 2) {
      in = o;                                  // flat copy (1-D vectors)
    } else if (dir == 0) {
      uint32_t q = (uint32_t)o;
      uint32_t a = compact_even(q >> 1), b = compact_even(q);
      in = ((long long)a << n) | b;
    } else {
      uint32_t a = (uint32_t)(o >> n), b = (uint32_t)(o & ((1ll << n) - 1));
      in = (long long)((spread_even(a) << 1) | spread_even(b));
    }
    double re, im;
    load_elem(src, sdt, fs + in, re, im);
    store_elem(dst, ddt, fd + o, re, im);
  }
}

// Tiled form (log2_side >= 5): one 32 x 32 pixel block per step of the
// grid-stride loop.  Its pixels are 1024 consecutive quantics indices (the
// low 10 bits of q interleave the low 5 bits of a and b, the high bits those
// of the block's position), so the quantics side moves as one contiguous run
// and the row-major side as 32 runs of 32 pixels; the block passes through
// LDS.  The per-element form above reads (dir 1) or writes (dir 0) the
// row-major side in runs of one or two pixels.
constexpr int QT_J = 5, QT_T = 1 << QT_J, QT_E = QT_T * QT_T;
__global__ __launch_bounds__(256) void quantics_tiled_kernel(const void* src, int sdt, void* dst, int ddt, int n,
                                                             long long tiles, int dir, long long s_src,
                                                             long long s_dst) {
  __shared__ double2 tile[QT_T][QT_T + 1];
  const long long fs = blockIdx.y * s_src, fd = blockIdx.y * s_dst;
  for (long long tq = blockIdx.x; tq < tiles; tq += gridDim.x) {
    const uint32_t ah = compact_even((uint32_t)tq >> 1), bh = compact_even((uint32_t)tq);
    const long long qbase = tq << (2 * QT_J);
    const long long rbase = ((long long)ah << (QT_J + n)) + ((long long)bh << QT_J);   // pixel (ah T, bh T)
    for (int e = threadIdx.x; e < QT_E; e += 256) {
      int al, bl;
      long long in;
      if (dir == 0) { al = e >> QT_J; bl = e & (QT_T - 1); in = rbase + ((long long)al << n) + bl; }
      else { al = (int)compact_even((uint32_t)e >> 1); bl = (int)compact_even((uint32_t)e); in = qbase + e; }
      double re, im;
      load_elem(src, sdt, fs + in, re, im);
      tile[al][bl] = make_double2(re, im);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < QT_E; e += 256) {
      int al, bl;
      long long o;
      if (dir == 0) { al = (int)compact_even((uint32_t)e >> 1); bl = (int)compact_even((uint32_t)e); o = qbase + e; }
      else { al = e >> QT_J; bl = e & (QT_T - 1); o = rbase + ((long long)al << n) + bl; }
      const double2 v = tile[al][bl];
      store_elem(dst, ddt, fd + o, v.x, v.y);
    }
    __syncthreads();
  }
}

hipError_t quantics_permute(const void* src, int src_dtype, void* dst, int dst_dtype, int log2_side, int dir,
                            hipStream_t s, int nf, long long s_src, long long s_dst) {
  if (nf < 1) return hipSuccess;
  if (dir != 2 && log2_side >= QT_J) {
    const long long tiles = 1ll << (2 * (log2_side - QT_J));
    const long long cap = std::max<long long>(1, 65536 / nf);
    hipLaunchKernelGGL(quantics_tiled_kernel, dim3((unsigned)std::min(tiles, cap), nf), dim3(256), 0, s, src,
                       src_dtype, dst, dst_dtype, log2_side, tiles, dir, s_src, s_dst);
    return hipGetLastError();
  }
  long long total = 1ll << (2 * log2_side);
  long long blocks = (total + 255) / 256;
  long long cap = std::max<long long>(1, 65536 / std::max(nf, 1));
  if (blocks > cap) blocks = cap;
  if (nf < 1) return hipSuccess;
  hipLaunchKernelGGL(quantics_kernel, dim3((unsigned)blocks, nf), dim3(256), 0, s, src, src_dtype, dst, dst_dtype,
                     log2_side, total, dir, s_src, s_dst);
  return hipGetLastError();
}

// Sum of |x|^2 over a rows x cols block (strides ld_r, ld_c), one workgroup,
// fixed reduction order (deterministic).
__global__ __launch_bounds__(1024) void block_norm_kernel(const void* p, int dtype, DimExpr rows, DimExpr cols,
                                                          int rmax, int cmax, long long ld_r, long long ld_c,
                                                          double* out) {
  const int nr = min(dim_eval(rows), rmax), nc = min(dim_eval(cols), cmax);
  const long long tot = (long long)nr * nc;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    long long r = e / nc, c = e - r * nc;
    long long off = r * ld_r + c * ld_c;
    double re, im;
    if (dtype == 0) { float2 v = ((const float2*)p)[off]; re = v.x; im = v.y; }
    else { double2 v = ((const double2*)p)[off]; re = v.x; im = v.y; }
    acc += re * re + im * im;
  }
  __shared__ double red[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    *out = sqrt(s);
  }
}

hipError_t block_norm(const void* p, int dtype, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                      long long ld_r, long long ld_c, double* out, hipStream_t s) {
  hipLaunchKernelGGL(block_norm_kernel, dim3(1), dim3(1024), 0, s, p, dtype, rows, cols, rows_bound, cols_bound,
                     ld_r, ld_c, out);
  return hipGetLastError();
}

__global__ void block_copy_kernel(const void* src, long long s_rs, long long s_cs, void* dst, long long d_rs,
                                  long long d_cs, DimExpr rows, DimExpr cols, int cmax, int dtype) {
  const int nr = min(dim_eval(rows), (int)gridDim.y), nc = min(dim_eval(cols), cmax);
  const int r = blockIdx.y;
  if (r >= nr) return;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    if (dtype == 0) ((float2*)dst)[r * d_rs + c * d_cs] = ((const float2*)src)[r * s_rs + c * s_cs];
    else ((double2*)dst)[r * d_rs + c * d_cs] = ((const double2*)src)[r * s_rs + c * s_cs];
  }
}

hipError_t block_copy(const void* src, long long s_rs, long long s_cs, void* dst, long long d_rs, long long d_cs,
                      DimExpr rows, DimExpr cols, int rows_bound, int cols_bound, int dtype, hipStream_t s) {
  if (rows_bound < 1 || cols_bound < 1) return hipSuccess;
  int bx = (cols_bound + 255) / 256;
  hipLaunchKernelGGL(block_copy_kernel, dim3(bx, rows_bound), dim3(256), 0, s, src, s_rs, s_cs, dst, d_rs, d_cs,
                     rows, cols, cols_bound, dtype);
  return hipGetLastError();
}

__global__ void set_ints_kernel(int* p, int count, int val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = val;
}
hipError_t set_ints(int* dev, int count, int val, hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(set_ints_kernel, dim3((count + 255) / 256), dim3(256), 0, s, dev, count, val);
  return hipGetLastError();
}
__global__ void copy_ints_kernel(const int* a, int* b, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = a[i];
}
hipError_t copy_ints(const int* src, int* dst, int count, hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(copy_ints_kernel, dim3((count + 255) / 256), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

__global__ void check_finite_kernel(const void* p, int dtype, long long count, int* status) {
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    double v = dtype == 0 ? (double)((const float*)p)[i] : ((const double*)p)[i];
    if (!isfinite(v)) bad = true;
  }
  if (bad) set_status(status, ST_NONFINITE);
}
hipError_t check_finite(const void* p, int dtype, long long count, int* status, hipStream_t s) {
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, dtype, count, status);
  return hipGetLastError();
}

// Copy caller-provided bond dimensions into the workspace, clamped to
// [1, min(cap, 2^k, 2^(m-k))]; out-of-range input flags the status word.  All
// kernels read the clamped copy, so no device-side size can exceed the
// storage the host sized its buffers and launch grids for.
__global__ void sanitize_bonds_kernel(const int* src, int* dst, int m, int cap, int* status, int free_inner) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > m) return;
  src += (long long)blockIdx.y * (m + 1);
  dst += (long long)blockIdx.y * (m + 1);
  int e = min(k, m - k);
  int bound = e >= 30 || (free_inner && e > 0) ? cap : min(cap, 1 << e);
  int v = src[k];
  int c = min(max(v, 1), bound);
  if (c != v) set_status(status, -5);
  dst[k] = c;
}
hipError_t sanitize_bonds(const int* src, int* dst, int m, int cap, int* status, int nf, hipStream_t s,
                          int free_inner) {
  hipLaunchKernelGGL(sanitize_bonds_kernel, dim3((m + 1 + 255) / 256, nf), dim3(256), 0, s, src, dst, m, cap, status,
                     free_inner);
  return hipGetLastError();
}

// ---- batched helpers (field f = blockIdx.z or blockIdx.y)
__global__ void block_copy_b_kernel(const void* src, long long s_rs, long long s_cs, long long s_f, void* dst,
                                    long long d_rs, long long d_cs, long long d_f, DimExpr rows, DimExpr cols,
                                    int cmax, int dtype, int conj) {
  const int f = blockIdx.z;
  const int nr = min(dim_eval(rows, f), (int)gridDim.y), nc = min(dim_eval(cols, f), cmax);
  const int r = blockIdx.y;
  if (r >= nr) return;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    long long so = f * s_f + r * s_rs + c * s_cs, dof = f * d_f + r * d_rs + c * d_cs;
    if (dtype == 0) {
      float2 v = ((const float2*)src)[so];
      if (conj) v.y = -v.y;
      ((float2*)dst)[dof] = v;
    } else {
      double2 v = ((const double2*)src)[so];
      if (conj) v.y = -v.y;
      ((double2*)dst)[dof] = v;
    }
  }
}
hipError_t block_copy_b(const void* src, long long s_rs, long long s_cs, long long s_f, void* dst, long long d_rs,
                        long long d_cs, long long d_f, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                        int dtype, int nf, hipStream_t s, int conj) {
  if (rows_bound < 1 || cols_bound < 1 || nf < 1) return hipSuccess;
  int bx = (cols_bound + 255) / 256;
  hipLaunchKernelGGL(block_copy_b_kernel, dim3(bx, rows_bound, nf), dim3(256), 0, s, src, s_rs, s_cs, s_f, dst, d_rs,
                     d_cs, d_f, rows, cols, cols_bound, dtype, conj);
  return hipGetLastError();
}

__global__ void hermitian_fill_kernel(double2* G, int ld, long long gs, DimExpr nexp, int nb) {
  const int f = blockIdx.y;
  const int n = min(dim_eval(nexp, f), nb);
  const int i = blockIdx.x;
  if (i >= n) return;
  double2* A = G + f * gs;
  for (int j = i + 1 + threadIdx.x; j < n; j += blockDim.x) {
    double2 v = A[(long long)j * ld + i];
    A[(long long)i * ld + j] = make_double2(v.x, -v.y);
  }
}
hipError_t hermitian_fill(double* G, int ld, long long gs, DimExpr n, int n_bound, int nf, hipStream_t s) {
  if (n_bound < 2 || nf < 1) return hipSuccess;
  hipLaunchKernelGGL(hermitian_fill_kernel, dim3(n_bound, nf), dim3(256), 0, s, (double2*)G, ld, gs, n, n_bound);
  return hipGetLastError();
}

// Zero `bytes` bytes (a multiple of 16) with vector stores; a plain kernel,
// so it is safe inside captured graphs.
__global__ void zero_fill_kernel(uint4* p, long long n16) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}
hipError_t zero_fill(void* p, size_t bytes, hipStream_t s) {
  long long n16 = (long long)(bytes / 16);
  if (n16 < 1) return hipSuccess;
  int blocks = (int)std::min<long long>((n16 + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, s, (uint4*)p, n16);
  return hipGetLastError();
}

// Intensity loss of the phase-retrieval problem, per field f:
//   L_f = sum_px (|E|^2 - I)^2,  grad = dL/dRe + i dL/dIm = 4 (|E|^2 - I) E.
// Two passes: per-block partial sums (fixed order), then one block per field.
constexpr int IL_NT = 256;
constexpr int IL_BLOCKS = 256;
template <typename C, typename R>
__global__ __launch_bounds__(IL_NT) void intensity_loss_kernel(const C* field, const R* target, long long per,
                                                               C* grad, double* part) {
  const int f = blockIdx.y;
  const C* e = field + f * per;
  const R* t = target + f * per;
  C* g = grad ? grad + f * per : nullptr;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)IL_NT + threadIdx.x; i < per; i += (long long)IL_BLOCKS * IL_NT) {
    C v = e[i];
    double re = v.x, im = v.y;
    double d = re * re + im * im - (double)t[i];
    acc += d * d;
    if (g) {
      C o;
      o.x = (decltype(o.x))(4.0 * d * re);
      o.y = (decltype(o.y))(4.0 * d * im);
      g[i] = o;
    }
  }
  __shared__ double red[IL_NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sm = 0.0;
    for (int i = 0; i < IL_NT / 64; ++i) sm += red[i];
    part[(long long)f * IL_BLOCKS + blockIdx.x] = sm;
  }
}
__global__ __launch_bounds__(IL_BLOCKS) void loss_reduce_kernel(const double* part, double* out) {
  const int f = blockIdx.x;
  double v = part[(long long)f * IL_BLOCKS + threadIdx.x];
  __shared__ double red[IL_BLOCKS / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sm = 0.0;
    for (int i = 0; i < IL_BLOCKS / 64; ++i) sm += red[i];
    out[f] = sm;
  }
}
size_t intensity_loss_ws(int nf) { return (size_t)nf * IL_BLOCKS * sizeof(double); }
hipError_t intensity_loss(const void* field, const void* target, int dtype, long long per, int nf, double* loss,
                          void* grad, void* part, hipStream_t s) {
  if (nf < 1 || per < 1) return hipSuccess;
  dim3 g(IL_BLOCKS, nf);
  if (dtype == 0)
    hipLaunchKernelGGL((intensity_loss_kernel<float2, float>), g, dim3(IL_NT), 0, s, (const float2*)field,
                       (const float*)target, per, (float2*)grad, (double*)part);
  else
    hipLaunchKernelGGL((intensity_loss_kernel<double2, double>), g, dim3(IL_NT), 0, s, (const double2*)field,
                       (const double*)target, per, (double2*)grad, (double*)part);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(nf), dim3(IL_BLOCKS), 0, s, (const double*)part, loss);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void block_norm_b_kernel(const void* p, int dtype, DimExpr rows, DimExpr cols,
                                                            int rmax, int cmax, long long ld_r, long long ld_c,
                                                            long long s_f, double* out) {
  const int f = blockIdx.x;
  const int nr = min(dim_eval(rows, f), rmax), nc = min(dim_eval(cols, f), cmax);
  const long long tot = (long long)nr * nc;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    long long r = e / nc, c = e - r * nc;
    long long off = f * s_f + r * ld_r + c * ld_c;
    double re, im;
    if (dtype == 0) { float2 v = ((const float2*)p)[off]; re = v.x; im = v.y; }
    else { double2 v = ((const double2*)p)[off]; re = v.x; im = v.y; }
    acc += re * re + im * im;
  }
  __shared__ double red[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    out[f] = sqrt(s);
  }
}
hipError_t block_norm_b(const void* p, int dtype, DimExpr rows, DimExpr cols, int rows_bound, int cols_bound,
                        long long ld_r, long long ld_c, long long s_f, double* out, int nf, hipStream_t s) {
  if (nf < 1) return hipSuccess;
  hipLaunchKernelGGL(block_norm_b_kernel, dim3(nf), dim3(1024), 0, s, p, dtype, rows, cols, rows_bound, cols_bound,
                     ld_r, ld_c, s_f, out);
  return hipGetLastError();
}

__global__ void set_ints_strided_kernel(int* p, int per, long long stride, int val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < per) p[blockIdx.y * stride + i] = val;
}
hipError_t set_ints_strided(int* dev, int per, long long stride, int nf, int val, hipStream_t s) {
  if (per < 1 || nf < 1) return hipSuccess;
  hipLaunchKernelGGL(set_ints_strided_kernel, dim3((per + 255) / 256, nf), dim3(256), 0, s, dev, per, stride, val);
  return hipGetLastError();
}

__global__ void set_one_b_kernel(void* p, long long s_f, int dtype) {
  long long o = (long long)blockIdx.x * s_f;
  if (dtype == 0) ((float2*)p)[o] = make_float2(1.f, 0.f);
  else ((double2*)p)[o] = make_double2(1.0, 0.0);
}
hipError_t set_one_b(void* p, long long s_f, int dtype, int nf, hipStream_t s) {
  if (nf < 1) return hipSuccess;
  hipLaunchKernelGGL(set_one_b_kernel, dim3(nf), dim3(1), 0, s, p, s_f, dtype);
  return hipGetLastError();
}

// Diagonal MPO of an MPS (the element-wise product with that MPS as an
// operator): W[k][w][t][s][w'] = delta_ts A_k[w][s][w'] (conjugated if conj)
// for w, w' inside the MPS's device bonds, 0 elsewhere up to the operator's
// bond bounds D_k = min(cap, 2^k, 2^(m-k)) (the bounds of any m-site MPS of
// capacity cap; zero padding leaves the operator unchanged).  One thread per
// (site, w, t, s, w') of the d_cap-strided operator.
__device__ __forceinline__ int mps_bound(int k, int m, int cap) {
  const int a = k >= 30 ? cap : min(cap, 1 << k);
  const int b = m - k >= 30 ? cap : min(cap, 1 << (m - k));
  return min(a, b);
}

template <typename C>
__global__ void mps_to_diag_mpo_kernel(const C* A, const int* bonds, int cap, int conj, C* W, int dcap, int m) {
  const long long per = (long long)dcap * 4 * dcap;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per * m) return;
  const int k = (int)(e / per);
  const long long r = e - (long long)k * per;
  const int w = (int)(r / (4 * dcap)), ts = (int)((r / dcap) & 3), w2 = (int)(r % dcap);
  const int t = ts >> 1, sb = ts & 1;
  const int dl = mps_bound(k, m, cap), dr = mps_bound(k + 1, m, cap);
  if (w >= dl || w2 >= dr) return;                       // outside this site's operator bonds
  const int bl = min(bonds[k], cap), br = min(bonds[k + 1], cap);
  C v;
  v.x = 0;
  v.y = 0;
  if (t == sb && w < bl && w2 < br) {
    v = A[(long long)k * cap * 2 * cap + (long long)w * 2 * cap + (long long)sb * cap + w2];
    if (conj) v.y = -v.y;
  }
  W[(long long)k * per + ((long long)w * 4 + ts) * dr + w2] = v;
}

hipError_t mps_to_diag_mpo(const void* A, const int* bonds, int cap, int conj, void* W, int dcap, int m, int dtype,
                           hipStream_t s) {
  const long long tot = (long long)dcap * 4 * dcap * m;
  const int blocks = (int)((tot + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(mps_to_diag_mpo_kernel<float2>, dim3(blocks), dim3(256), 0, s, (const float2*)A, bonds, cap,
                       conj, (float2*)W, dcap, m);
  else
    hipLaunchKernelGGL(mps_to_diag_mpo_kernel<double2>, dim3(blocks), dim3(256), 0, s, (const double2*)A, bonds, cap,
                       conj, (double2*)W, dcap, m);
  return hipGetLastError();
}

// Write one complex element (used to seed the zip-up carry with 1).
__global__ void set_one_kernel(void* p, int dtype) {
  if (dtype == 0) ((float2*)p)[0] = make_float2(1.f, 0.f);
  else ((double2*)p)[0] = make_double2(1.0, 0.0);
}
hipError_t set_one(void* p, int dtype, hipStream_t s) {
  hipLaunchKernelGGL(set_one_kernel, dim3(1), dim3(1), 0, s, p, dtype);
  return hipGetLastError();
}

// ---- separable fields: interleave two 1-D MPS (Sec. 3 quantics order)
// Output site 2p (bit p of a) has bonds (ru_p rv_p) -> (ru_(p+1) rv_p) and
// core U_p x identity; site 2p+1 (bit p of b) has (ru_(p+1) rv_p) ->
// (ru_(p+1) rv_(p+1)) and core identity x V_p.  Bond pairs are flattened
// as iu * rv + iv.  Products beyond the output capacity flag the status.
template <typename T>
__global__ void interleave_kernel(const T* U, const int* ub, int ucap, const T* V, const int* vb, int vcap, T* out,
                                  int* ob, int ocap, int* status) {
  const int j = blockIdx.y, p = j >> 1;
  const bool is_a = (j & 1) == 0;
  const int rul = ub[p], rur = ub[p + 1], rvl = vb[p], rvr = vb[p + 1];
  const int L = is_a ? rul * rvl : rur * rvl;
  const int R = is_a ? rur * rvl : rur * rvr;
  if (L > ocap || R > ocap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) set_status(status, -5);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ob[j + 1] = R;
    if (j == 0) ob[0] = 1;
  }
  const T* Up = U + (long long)p * ucap * 2 * ucap;
  const T* Vp = V + (long long)p * vcap * 2 * vcap;
  T* O = out + (long long)j * ocap * 2 * ocap;
  const long long tot = (long long)L * 2 * R;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(e / (2 * R)), rem = (int)(e - (long long)l * 2 * R), s = rem / R, r = rem - s * R;
    T val;
    val.x = 0;
    val.y = 0;
    if (is_a) {
      const int iu = l / rvl, iv = l - iu * rvl, ju = r / rvl, jv = r - ju * rvl;
      if (iv == jv) val = Up[(long long)iu * 2 * ucap + s * ucap + ju];
    } else {
      const int iu = l / rvl, iv = l - iu * rvl, ju = r / rvr, jv = r - ju * rvr;
      if (iu == ju) val = Vp[(long long)iv * 2 * vcap + s * vcap + jv];
    }
    O[(long long)l * 2 * ocap + s * ocap + r] = val;
  }
}
hipError_t interleave(const void* U, const int* ub, int ucap, const void* V, const int* vb, int vcap, void* out,
                      int* ob, int ocap, int n_per_axis, int dtype, int* status, hipStream_t s) {
  dim3 g(256, 2 * n_per_axis);
  if (dtype == 0)
    hipLaunchKernelGGL(interleave_kernel<float2>, g, dim3(256), 0, s, (const float2*)U, ub, ucap, (const float2*)V,
                       vb, vcap, (float2*)out, ob, ocap, status);
  else
    hipLaunchKernelGGL(interleave_kernel<double2>, g, dim3(256), 0, s, (const double2*)U, ub, ucap,
                       (const double2*)V, vb, vcap, (double2*)out, ob, ocap, status);
  return hipGetLastError();
}

// ---- point evaluation: after contracting site k for every point, keep the
// half of C[p][(r', s)] selected by the point's bit at site k.
// Site 2q is bit q (most significant first) of the row a, site 2q+1 of b.
template <typename T>
__global__ void select_bit_kernel(const T* C, long long ldc, T* Lnext, long long ldl, const int* rows,
                                  const int* cols, int count, int site, int n, const int* rbond, int cap) {
  const int p = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (p >= count) return;
  const int q = site >> 1;
  const int coord = (site & 1) ? cols[p] : rows[p];
  const int bit = (coord >> (n - 1 - q)) & 1;
  const int rr = min(rbond[0], cap);
  for (int r = threadIdx.x & 63; r < rr; r += 64) Lnext[(long long)p * ldl + r] = C[(long long)p * ldc + 2 * r + bit];
}
hipError_t select_bit(const void* C, long long ldc, void* Lnext, long long ldl, const int* rows, const int* cols,
                      int count, int site, int n, const int* rbond, int cap, int dtype, hipStream_t s) {
  if (count < 1) return hipSuccess;
  dim3 g((count + 3) / 4);
  if (dtype == 0)
    hipLaunchKernelGGL(select_bit_kernel<float2>, g, dim3(256), 0, s, (const float2*)C, ldc, (float2*)Lnext, ldl,
                       rows, cols, count, site, n, rbond, cap);
  else
    hipLaunchKernelGGL(select_bit_kernel<double2>, g, dim3(256), 0, s, (const double2*)C, ldc, (double2*)Lnext, ldl,
                       rows, cols, count, site, n, rbond, cap);
  return hipGetLastError();
}

// Point p's value: column 0 of its final row vector.
template <typename T>
__global__ void gather_col0_kernel(const T* Lf, long long ldl, T* out, int count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) out[p] = Lf[(long long)p * ldl];
}
hipError_t gather_col0(const void* Lf, long long ldl, void* out, int count, int dtype, hipStream_t s) {
  if (count < 1) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(gather_col0_kernel<float2>, dim3((count + 255) / 256), dim3(256), 0, s, (const float2*)Lf, ldl,
                       (float2*)out, count);
  else
    hipLaunchKernelGGL(gather_col0_kernel<double2>, dim3((count + 255) / 256), dim3(256), 0, s, (const double2*)Lf,
                       ldl, (double2*)out, count);
  return hipGetLastError();
}

// Row vector e_0 (complex 1 at column 0, zeros to the capacity) per point.
template <typename T>
__global__ void unit_rows_kernel(T* L, long long ldl, int count, int cap) {
  const long long tot = (long long)count * cap;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / cap;
    const int r = (int)(e - p * cap);
    T v;
    v.x = r == 0 ? 1 : 0;
    v.y = 0;
    L[p * ldl + r] = v;
  }
}
hipError_t unit_rows(void* L, long long ldl, int count, int cap, int dtype, hipStream_t s) {
  if (count < 1) return hipSuccess;
  long long tot = (long long)count * cap;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 8192);
  if (dtype == 0)
    hipLaunchKernelGGL(unit_rows_kernel<float2>, dim3(blocks), dim3(256), 0, s, (float2*)L, ldl, count, cap);
  else
    hipLaunchKernelGGL(unit_rows_kernel<double2>, dim3(blocks), dim3(256), 0, s, (double2*)L, ldl, count, cap);
  return hipGetLastError();
}

// Write the bit pattern of a block's fixed high bits as point coordinates.
__global__ void fill_point_kernel(int* rows, int* cols, int row, int col) {
  rows[0] = row;
  cols[0] = col;
}
hipError_t fill_point(int* rows, int* cols, int row, int col, hipStream_t s) {
  hipLaunchKernelGGL(fill_point_kernel, dim3(1), dim3(1), 0, s, rows, cols, row, col);
  return hipGetLastError();
}

}  // namespace qtt

namespace qtt {
// ---- direct sum of R MPS (rank terms of a low-rank field): the sum's bond at
// cut k is the sum of the terms' bonds there; core 0 places the terms' row
// vectors side by side, the last core stacks their columns, every other core
// is block-diagonal.  Terms share one capacity tcap and sit back to back
// (term r at element offset r * m * tcap * 2 * tcap, bonds at r * (m + 1)).
template <typename T>
__global__ void direct_sum_kernel(const T* terms, const int* tbonds, int rank, int tcap, int m, T* out, int* ob,
                                  int ocap, int* status) {
  const int k = blockIdx.y;
  const int* b0 = tbonds;
  // offsets of every term's block at cuts k and k + 1 and the sum's bonds
  int lo_off[QTT_MAX_RANK], hi_off[QTT_MAX_RANK];
  int lsum = 0, hsum = 0;
  for (int r = 0; r < rank; ++r) {
    const int* b = b0 + r * (m + 1);
    const int bl = k == 0 ? 1 : min(b[k], tcap), bh = k == m - 1 ? 1 : min(b[k + 1], tcap);
    lo_off[r] = k == 0 ? 0 : lsum;
    hi_off[r] = k == m - 1 ? 0 : hsum;
    lsum += bl;
    hsum += bh;
  }
  const int L = k == 0 ? 1 : lsum, R = k == m - 1 ? 1 : hsum;
  if (L > ocap || R > ocap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) set_status(status, ST_CAPACITY);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) ob[0] = 1;
    ob[k + 1] = R;
  }
  T* O = out + (long long)k * ocap * 2 * ocap;
  const long long tot = (long long)ocap * 2 * ocap;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(e / (2 * ocap)), rem = (int)(e - (long long)l * 2 * ocap), s = rem / ocap, c = rem - s * ocap;
    T val;
    val.x = 0;
    val.y = 0;
    if (l < L && c < R) {
      for (int r = 0; r < rank; ++r) {
        const int* b = b0 + r * (m + 1);
        const int bl = k == 0 ? 1 : min(b[k], tcap), bh = k == m - 1 ? 1 : min(b[k + 1], tcap);
        const int li = k == 0 ? l : l - lo_off[r], ci = k == m - 1 ? c : c - hi_off[r];
        if (li >= 0 && li < bl && ci >= 0 && ci < bh) {
          val = terms[(long long)r * m * tcap * 2 * tcap + (long long)k * tcap * 2 * tcap + (long long)li * 2 * tcap +
                      s * tcap + ci];
          break;
        }
      }
    }
    O[e] = val;
  }
}
hipError_t direct_sum(const void* terms, const int* tbonds, int rank, int tcap, int m, void* out, int* ob, int ocap,
                      int dtype, int* status, hipStream_t s) {
  if (rank < 1 || rank > QTT_MAX_RANK) return hipErrorInvalidValue;
  dim3 g(64, m);
  if (dtype == 0)
    hipLaunchKernelGGL(direct_sum_kernel<float2>, g, dim3(256), 0, s, (const float2*)terms, tbonds, rank, tcap, m,
                       (float2*)out, ob, ocap, status);
  else
    hipLaunchKernelGGL(direct_sum_kernel<double2>, g, dim3(256), 0, s, (const double2*)terms, tbonds, rank, tcap, m,
                       (double2*)out, ob, ocap, status);
  return hipGetLastError();
}
}  // namespace qtt

namespace qtt {
// ---- perfect sampling: one bit per sample at site k.  C[p][2 r + s] holds
// (A_k[s] R_p)[r] for this sample's boundary vector R_p (right of site k);
// with the sites left of k an isometry, the probability of bit s given the
// bits already drawn is |C[p][2 . + s]|^2 / (|C[p][2 . + 0]|^2 + |C[p][2 . + 1]|^2).
// The bit is s = 0 when u * (p0 + p1) < p0 (u the sample's uniform for this
// site), the new boundary vector C[p][2 . + s] / sqrt(p_s), and the bit is
// written into the row (even site) or column (odd site) coordinate, most
// significant bit first.  One wave per sample; sums in FP64.
template <typename T>
__global__ void sample_select_kernel(const T* C, long long ldc, T* Rn, long long ldr, const double* uni, int m,
                                     int site, const int* bond, int cap, int* rows, int* cols, int count) {
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= count) return;
  const int lane = threadIdx.x & 63;
  const int bk = min(max(bond[0], 1), cap);
  const T* Cp = C + (long long)p * ldc;
  double s0 = 0.0, s1 = 0.0;
  for (int r = lane; r < bk; r += 64) {
    const T a = Cp[2 * r], b = Cp[2 * r + 1];
    s0 += (double)a.x * a.x + (double)a.y * a.y;
    s1 += (double)b.x * b.x + (double)b.y * b.y;
  }
  s0 = wave_sum_u(s0);
  s1 = wave_sum_u(s1);
  const double u = uni[(long long)p * m + site];
  const int bit = (s0 + s1 > 0.0 && !(u * (s0 + s1) < s0)) ? 1 : 0;
  const double ps = bit ? s1 : s0;
  const double sc = ps > 0.0 ? 1.0 / sqrt(ps) : 0.0;
  for (int r = lane; r < cap; r += 64) {
    T v;
    v.x = 0;
    v.y = 0;
    if (r < bk) {
      const T a = Cp[2 * r + bit];
      v.x = (decltype(v.x))(a.x * sc);
      v.y = (decltype(v.y))(a.y * sc);
    }
    Rn[(long long)p * ldr + r] = v;
  }
  if (lane == 0) {
    const int n = m >> 1, q = site >> 1, sh = n - 1 - q;
    int* dst = (site & 1) ? cols : rows;
    const int prev = site == m - 1 || site == m - 2 ? 0 : dst[p];   // the first bit of each coordinate starts it
    dst[p] = prev | (bit << sh);
  }
}
hipError_t sample_select(const void* C, long long ldc, void* Rn, long long ldr, const double* uni, int m, int site,
                         const int* bond, int cap, int* rows, int* cols, int count, int dtype, hipStream_t s) {
  if (count < 1) return hipSuccess;
  dim3 g((count + 3) / 4);
  if (dtype == 0)
    hipLaunchKernelGGL(sample_select_kernel<float2>, g, dim3(256), 0, s, (const float2*)C, ldc, (float2*)Rn, ldr, uni,
                       m, site, bond, cap, rows, cols, count);
  else
    hipLaunchKernelGGL(sample_select_kernel<double2>, g, dim3(256), 0, s, (const double2*)C, ldc, (double2*)Rn, ldr,
                       uni, m, site, bond, cap, rows, cols, count);
  return hipGetLastError();
}
}  // namespace qtt
