// Shared device-side helpers of libqtt (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// A problem dimension known only on the device: for batch entry (field) f,
// value = c * p0[f*bs] * p1[f*bs], a NULL pointer contributing 1.  Bond
// dimensions chosen by the eigensolver are written to device memory and read
// back through these by later kernels in the same stream, so the host never
// waits for them; bs is the per-field stride of the bond arrays.
struct DimExpr {
  int c;
  const int* p0;
  const int* p1;
  int bs;
};

__device__ __forceinline__ int dim_eval(const DimExpr& d, int f = 0) {
  int v = d.c;
  if (d.p0) v *= d.p0[(long long)f * d.bs];
  if (d.p1) v *= d.p1[(long long)f * d.bs];
  return v;
}

// Division by a run-time constant d >= 1 for n < 2^31 (Granlund-Montgomery
// round-up method): q = (umulhi(n, mul) + n) >> shift.
struct FastDiv {
  uint32_t d, mul, shift;
};

__device__ __forceinline__ uint32_t fdiv(const FastDiv& f, uint32_t n) {
  uint64_t t = (uint64_t)__umulhi(n, f.mul) + n;
  return (uint32_t)(t >> f.shift);
}

// One operand (or the result) of a batched complex contraction.  A logical
// matrix index pair (x, y) is split as x = xh * Lx + xl, y = yh * Ly + yl
// (Lx, Ly given by FastDiv of the owning dimension) and addressed at
//   ptr + batch * sb + xh * sxh + xl * sxl + yh * syh + yl * syl
// in complex elements.  This expresses every reshape/permutation the zip-up,
// sweep, encode and decompression steps need without copies.
// sb: stride between fields (outer batch), sb2: stride of the inner batch index.
struct Operand {
  void* ptr;
  long long sxh, sxl, syh, syl, sb, sb2;
  int conj;
};

// Two-level batch: blockIdx.z = f * b2cap + a, f the field, a an inner
// batch index bounded by the device value batch(f).
struct GemmArgs {
  DimExpr M, N, K, batch;
  int b2cap;
  FastDiv fm, fn, fk;     // low extents of the split M, N, K indices
  Operand A, B, C;        // A: (M, K); B: (K, N); C: (M, N)
  int accumulate;         // C += A.B instead of C = A.B
  int lower;              // Hermitian result: tiles wholly above the diagonal are skipped
  int ksplit;             // >1: blockIdx.y selects a K chunk; C gets batch stride csplit
  long long csplit;       // complex-element stride between K-chunk partial results
  int tiles_n;            // tile-grid width used to decode blockIdx.x
  int Mmax, Nmax, Kmax, Bmax;   // host bounds: device sizes are clamped to these
};

// Device status word (first 4 bytes of every workspace).
enum { ST_OK = 0, ST_NONFINITE = -7, ST_NOCONVERGE = -8 };

__device__ __forceinline__ void set_status(int* st, int code) {
  if (st) atomicCAS(st, 0, code);
}

// Cross-lane sums through DPP moves (a few cycles each) instead of LDS
// permutes.  row16_sum: every lane gets the sum over its 16-lane row (lanes
// of one row may differ in the last bit: the association depends on the
// quad).  wave_sum_u: the wave's sum from rows 0..3 in a fixed order,
// identical in every lane.  seg_sum<TPC>: sum over aligned segments of TPC
// lanes (32 or 64), valid in the segment's last lane.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, RM, 0xf, false);
  return __hiloint2double(h2, l2);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1, 0xf>(v);      // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xf>(v);      // quad_perm [2,3,0,1]
  v += dpp_d<0x124, 0xf>(v);     // row_ror:4
  v += dpp_d<0x128, 0xf>(v);     // row_ror:8
  return v;
}
__device__ __forceinline__ double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double wave_sum_u(double v) {
  v = row16_sum(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}
// Uniform wave sums of two values for about the price of one: a v_permlane32_swap
// gives lanes 0..31 a[l] + a[l + 32] and lanes 32..63 b[l - 32] + b[l], a
// v_permlane16_swap folds each half onto its two rows, and one row16_sum
// finishes both; a is then read from lane 0 and b from lane 32.
__device__ __forceinline__ void wave_sum2_u(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  double v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  const auto l16 = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false,
                                                    false);
  const auto h16 = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false,
                                                    false);
  v = __hiloint2double((int)h16[0], (int)l16[0]) + __hiloint2double((int)h16[1], (int)l16[1]);
  v = row16_sum(v);
  a = lane_d(v, 0);
  b = lane_d(v, 32);
}
// Uniform wave sums of three complex values (six reals) in one pass: the
// permlane32 swaps fold the pairs (a.x, a.y), (b.x, b.y), (c.x, c.y) onto the
// wave halves; a permlane16 swap then folds the first two results onto rows
// (a.x, b.x, a.y, b.y) and the third onto (c.x, c.x, c.y, c.y); two row16_sums
// finish them and readlane picks each row's total.
__device__ __forceinline__ double2 pl32_fold(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return make_double2(__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1]));
}
__device__ __forceinline__ double2 pl16_fold(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return make_double2(__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1]));
}
__device__ __forceinline__ void wave_sum3c_u(double2& a, double2& b, double2& c) {
  const double2 p = pl32_fold(a.x, a.y), q = pl32_fold(b.x, b.y), r = pl32_fold(c.x, c.y);
  const double2 s2 = pl16_fold(p.x + p.y, q.x + q.y), t2 = pl16_fold(r.x + r.y, r.x + r.y);
  const double s = row16_sum(s2.x + s2.y), t = row16_sum(t2.x + t2.y);
  a = make_double2(lane_d(s, 0), lane_d(s, 32));
  b = make_double2(lane_d(s, 16), lane_d(s, 48));
  c = make_double2(lane_d(t, 0), lane_d(t, 32));
}
// Sums of two values over each 32-lane half of the wave, valid in lanes 31 and
// 63: a permlane16 fold leaves x's 16-lane partials on rows 0 and 2 and y's on
// rows 1 and 3, one row16_sum finishes both, and row_bcast:15 brings each
// half's x total to the row that holds its y total.
__device__ __forceinline__ void seg32_sum2(double& x, double& y) {
  const double2 f = pl16_fold(x, y);
  const double v = row16_sum(f.x + f.y);
  y = v;
  x = dpp_d<0x142, 0xA>(v);
}
template <int TPC>
__device__ __forceinline__ double seg_sum(double v) {
  static_assert(TPC == 32 || TPC == 64, "segments of 32 or 64 lanes");
  if constexpr (TPC == 64) {
    return wave_sum_u(v);
  } else {
    v = row16_sum(v);
    return v + dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  }
}
