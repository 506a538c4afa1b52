// Batched complex contraction on CDNA4 matrix cores.
//
// Every tensor contraction of the zip-up, the truncation sweep, the encode
// projections and the decompression is a batched complex matrix product
// C = op(A) . op(B) over reshaped/permuted views of the cores (Operand
// strides).  A complex product is run as ONE real product on the embedding
//   [Re C | Im C] = [Re A | Im A] . [[Re B, Im B], [-Im B, Re B]],
// i.e. the interleaved complex rows of A are already the real operand and the
// 2x2 real block of each B element is written out when B's tile is stored to
// LDS.  This keeps complex64/complex128 interleaved in HBM and in the output
// with no separate real/imaginary planes and no extra passes.
//
// Tiles: 64x64 complex outputs per 256-thread workgroup by default (32x64,
// 32x32 and, for FP32, 128x64 and 128x128 picked per call shape by the
// autotuner), 16 complex of depth per LDS stage, 4 waves in a 2x2
// arrangement, each wave a (BM/2)x(BN) real block made of 16x16 MFMA tiles
// (v_mfma_f32_16x16x4f32 for FP32,
// v_mfma_f64_16x16x4f64 for FP64 Gram matrices and the FP64 path).  The
// BF16 precision forms (operands rounded to bfloat16, or split into two
// bfloat16 terms with three products, FP32 accumulation) run a separate
// kernel on v_mfma_f32_16x16x32_bf16 with operands converted on their way
// into LDS.  Global
// loads of the next stage are issued into registers before the MFMAs of the
// current stage (software pipelining).  Dimensions are read from the device
// (DimExpr), so tiles beyond the actual bond dimensions exit at once.
#include <map>
#include <set>

#include "common.h"
#include "kernels.h"

namespace qtt {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Round an FP32 value to the nearest bfloat16 (ties to even) and return it
// as FP32 (low 16 bits zero); finite inputs only.
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(x) >> 16); }

template <typename TC> struct Mfma;
template <> struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float2 t; };
template <> struct Vec2<double> { typedef double2 t; };

constexpr int BKC = 16;                     // complex depth per LDS stage
constexpr int PADA = 4, PADB = 4;
constexpr int NT = 256;
// Output tile variants (complex rows x complex columns per workgroup); the
// autotuner picks one per call shape, 64 x 64 by default.  The two wide
// variants (FP32 operands and accumulation only) halve the operand bytes per
// flop of the 64 x 64 tile: at 16 complex of depth per stage a 64 x 64 tile
// reads 32 flops' worth of operands per byte, which at the FP32 matrix peak
// is more L2 traffic than the chip serves.
constexpr int N_TILES = 5;
constexpr int N_TILES_NARROW = 3;            // variants of the FP64-accumulating and bfloat16 forms
constexpr int TILE_M[N_TILES] = {64, 32, 32, 128, 128};
constexpr int TILE_N[N_TILES] = {64, 64, 32, 64, 128};

__device__ __forceinline__ long long split_off(const FastDiv& f, uint32_t x, long long sh, long long sl) {
  uint32_t h = fdiv(f, x);
  uint32_t l = x - h * f.d;
  return (long long)h * sh + (long long)l * sl;
}

// FP32 / FP64 operands (the bfloat16 forms have a kernel of their own below).
template <typename TIn, typename TC, typename TOut, bool AKM, bool BKM, int BM, int BN>
__global__ __launch_bounds__(NT) void cgemm_kernel(GemmArgs g) {
  constexpr int A_PER_T = BM * BKC / NT;      // complex elements of A per thread per stage
  constexpr int B_PER_T = BKC * BN / NT;
  typedef typename Vec2<TIn>::t in2;
  typedef typename Mfma<TC>::acc_t acc_t;
  const int f = blockIdx.z / g.b2cap;
  const int bz = blockIdx.z - f * g.b2cap;
  if (bz >= min(dim_eval(g.batch, f), g.Bmax)) return;
  const int M = min(dim_eval(g.M, f), g.Mmax), N = min(dim_eval(g.N, f), g.Nmax), K = min(dim_eval(g.K, f), g.Kmax);
  const int tm = blockIdx.x / g.tiles_n, tn = blockIdx.x % g.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  if (g.lower && m0 + BM <= n0) return;
  int kbeg = 0, kend = K;
  if (g.ksplit > 1) {
    int chunk = (K + g.ksplit - 1) / g.ksplit;
    chunk = (chunk + BKC - 1) / BKC * BKC;
    kbeg = blockIdx.y * chunk;
    kend = min(K, kbeg + chunk);
  }

  // FP32 operands: two LDS buffers (one barrier per stage, the next stage
  // stored while this one's products run); FP64 keeps one (occupancy)
  constexpr int NBUF = sizeof(TC) == 4 ? 2 : 1;
  // FP32 A tile without padding, its columns XOR-swizzled per row: the MFMA
  // reads (4 k-rows x 16 columns) and the k-major stores (16 even or odd
  // k-rows x 4 columns) then touch every bank exactly twice, the minimum for
  // 64 four-byte accesses (a 4-float pad gave 4-way conflicts on both).
  // B is stored as the real right operand of the embedding: complex row k
  // becomes real rows 2k = [re, im] and 2k + 1 = [-im, re] per column, so an
  // MFMA operand is one plain LDS read with no sign select after it (a select
  // per value made every read wait for its own data).  FP32 rows are padded
  // by 16 floats (8 when stored k-major) so the four k-rows of a read cover
  // the banks twice.
  constexpr bool SWZ = sizeof(TC) == 4;
  constexpr int SA = SWZ ? BM : BM + PADA;
  constexpr int SB = 2 * BN + (SWZ ? (BKM ? 8 : 16) : PADB);
  __shared__ TC Asb[NBUF][2 * BKC][SA];
  __shared__ __align__(16) TC Bsb[NBUF][2 * BKC][SB];
  auto acol = [](int row, int col) -> int {
    if constexpr (SWZ) return col ^ ((((row >> 1) & 3) << 2) | ((((row >> 3) ^ row) & 1) << 4));
    else return col;
  };
  int cur = 0;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const TIn* Ap = (const TIn*)g.A.ptr + 2 * ((long long)f * g.A.sb + (long long)bz * g.A.sb2);
  const TIn* Bp = (const TIn*)g.B.ptr + 2 * ((long long)f * g.B.sb + (long long)bz * g.B.sb2);

  // ---- per-thread fixed parts of the load addresses
  int a_i[A_PER_T], a_k[A_PER_T];
  long long a_rowoff[A_PER_T];
  int b_k[B_PER_T], b_j[B_PER_T];
  long long b_coloff[B_PER_T];
#pragma unroll
  for (int r = 0; r < A_PER_T; ++r) {
    int e = t + r * NT;
    if (AKM) { a_k[r] = e % BKC; a_i[r] = e / BKC; }
    else     { a_i[r] = e % BM;  a_k[r] = e / BM; }
    int gi = m0 + a_i[r];
    a_rowoff[r] = gi < M ? split_off(g.fm, gi, g.A.sxh, g.A.sxl) : -1;
  }
#pragma unroll
  for (int r = 0; r < B_PER_T; ++r) {
    int e = t + r * NT;
    if (BKM) { b_k[r] = e % BKC; b_j[r] = e / BKC; }
    else     { b_j[r] = e % BN;  b_k[r] = e / BN; }
    int gj = n0 + b_j[r];
    b_coloff[r] = gj < N ? split_off(g.fn, gj, g.B.syh, g.B.syl) : -1;
  }

  in2 ra[A_PER_T], rb[B_PER_T];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      int gk = k0 + a_k[r];
      in2 v; v.x = 0; v.y = 0;
      if (a_rowoff[r] >= 0 && gk < kend) {
        long long o = a_rowoff[r] + split_off(g.fk, gk, g.A.syh, g.A.syl);
        v = *(const in2*)(Ap + 2 * o);
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      int gk = k0 + b_k[r];
      in2 v; v.x = 0; v.y = 0;
      if (b_coloff[r] >= 0 && gk < kend) {
        long long o = b_coloff[r] + split_off(g.fk, gk, g.B.sxh, g.B.sxl);
        v = *(const in2*)(Bp + 2 * o);
      }
      rb[r] = v;
    }
  };
  auto store_stage = [&](int bi) {
    typedef typename Vec2<TC>::t tc2;
    TC (*As)[SA] = Asb[bi];
    TC (*Bs)[SB] = Bsb[bi];
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      TC re = (TC)ra[r].x, im = (TC)ra[r].y;
      As[2 * a_k[r]][acol(2 * a_k[r], a_i[r])] = re;
      As[2 * a_k[r] + 1][acol(2 * a_k[r] + 1, a_i[r])] = g.A.conj ? -im : im;
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      TC re = (TC)rb[r].x, im = (TC)rb[r].y;
      if (g.B.conj) im = -im;
      tc2 top, bot;
      top.x = re; top.y = im;
      bot.x = -im; bot.y = re;
      *(tc2*)&Bs[2 * b_k[r]][2 * b_j[r]] = top;
      *(tc2*)&Bs[2 * b_k[r] + 1][2 * b_j[r]] = bot;
    }
  };

  constexpr int MI = BM / 32;   // 16-row MFMA blocks per wave
  constexpr int NJ = BN / 16;   // 16-real-column MFMA blocks per wave (BN real cols)
  acc_t acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const int l16 = lane & 15, lq = lane >> 4;

  if (kbeg < kend) {
    load_stage(kbeg);
    if constexpr (NBUF == 2) {
      store_stage(0);
      __syncthreads();
    }
    for (int k0 = kbeg; k0 < kend; k0 += BKC) {
      if constexpr (NBUF == 1) {
        __syncthreads();
        store_stage(0);
        __syncthreads();
      }
      const bool more = k0 + BKC < kend;
      if (more) load_stage(k0 + BKC);
      TC (*As)[SA] = Asb[cur];
      TC (*Bs)[SB] = Bsb[cur];
#pragma unroll
      for (int ks = 0; ks < BKC / 2; ++ks) {
        TC af[MI], bf[NJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) af[i] = As[ks * 4 + lq][acol(ks * 4 + lq, wm * (BM / 2) + i * 16 + l16)];
#pragma unroll
        for (int j = 0; j < NJ; ++j) bf[j] = Bs[ks * 4 + lq][wn * BN + j * 16 + l16];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[i][j] = Mfma<TC>::op(af[i], bf[j], acc[i][j]);
      }
      if constexpr (NBUF == 2) {
        if (more) store_stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
      }
    }
  }

  // ---- epilogue: lanes (l, l^1) hold (re, im) of one complex output
  TOut* Cp = (TOut*)g.C.ptr + 2 * ((long long)f * g.C.sb + (long long)bz * g.C.sb2 +
                                   (long long)blockIdx.y * g.csplit);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    int jr = wn * BN + j * 16 + l16;
    int gj = n0 + (jr >> 1);
    long long coff = gj < N ? split_off(g.fn, gj, g.C.syh, g.C.syl) : -1;
#pragma unroll
    for (int i = 0; i < MI; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        TC v = acc[i][j][r];
        TC pv = __shfl_xor(v, 1);
        // output row of accumulator element r: the f32 16x16x4 MFMA gives lane
        // group lq rows 4*lq + r, the f64 one rows 4*r + lq
        const int row = sizeof(TC) == 8 ? (4 * r + lq) : (lq * 4 + r);
        int gi = m0 + wm * (BM / 2) + i * 16 + row;
        if (!(lane & 1) && coff >= 0 && gi < M) {
          long long o = split_off(g.fm, gi, g.C.sxh, g.C.sxl) + coff;
          typename Vec2<TOut>::t* dst = (typename Vec2<TOut>::t*)(Cp + 2 * o);
          typename Vec2<TOut>::t w;
          w.x = (TOut)v;
          w.y = (TOut)pv;
          if (g.accumulate) {
            typename Vec2<TOut>::t old = *dst;
            w.x += old.x;
            w.y += old.y;
          }
          *dst = w;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- bfloat16 forms
// The same complex product on gfx950's v_mfma_f32_16x16x32_bf16 (32 real k
// per instruction, FP32 accumulation).  Operands are converted once, on their
// way into LDS, into bfloat16 planes laid out as the instruction reads them:
// A as [row i][real k] (k = 2 kc + {re, im}), B as [real column jr][real k]
// with the 2 x 2 real block of every complex element,
//   rows 2kc, 2kc+1 x columns 2jc, 2jc+1 = [[re, im], [-im, re]],
// already expanded, so a lane's 8 consecutive k are one 16-byte LDS read and
// the MFMA loop does no conversions.  BF = 1: each operand rounded to
// bfloat16 (one product per 32-k stage).  BF = 3: x = hi + lo with hi, lo
// bfloat16 and the product hi.hi + hi.lo + lo.hi (three per stage; the lo.lo
// term, below FP32 rounding, is left out).  Global loads and the epilogue are
// those of cgemm_kernel.
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BKR = 2 * BKC;                 // real k per stage (32: one x32 MFMA)
constexpr int BROW = BKR + 8;                // bfloat16 per LDS row (16-byte aligned rows, staggered banks)

__device__ __forceinline__ uint32_t bf16_pair(float lo_k, float hi_k) {
  return (uint32_t)(uint16_t)bf16_bits(lo_k) | ((uint32_t)(uint16_t)bf16_bits(hi_k) << 16);
}

template <bool AKM, bool BKM, int BF, int BM, int BN>
__global__ __launch_bounds__(NT) void cgemm_bf16_kernel(GemmArgs g) {
  constexpr int A_PER_T = BM * BKC / NT;
  constexpr int B_PER_T = BKC * BN / NT;
  constexpr int NP = BF == 3 ? 2 : 1;         // bfloat16 planes per operand (hi[, lo])
  typedef floatx4 acc_t;
  const int f = blockIdx.z / g.b2cap;
  const int bz = blockIdx.z - f * g.b2cap;
  if (bz >= min(dim_eval(g.batch, f), g.Bmax)) return;
  const int M = min(dim_eval(g.M, f), g.Mmax), N = min(dim_eval(g.N, f), g.Nmax), K = min(dim_eval(g.K, f), g.Kmax);
  const int tm = blockIdx.x / g.tiles_n, tn = blockIdx.x % g.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  if (g.lower && m0 + BM <= n0) return;
  int kbeg = 0, kend = K;
  if (g.ksplit > 1) {
    int chunk = (K + g.ksplit - 1) / g.ksplit;
    chunk = (chunk + BKC - 1) / BKC * BKC;
    kbeg = blockIdx.y * chunk;
    kend = min(K, kbeg + chunk);
  }
  __shared__ __attribute__((aligned(16))) uint16_t Asb[2][NP][BM][BROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bsb[2][NP][2 * BN][BROW];
  int cur = 0;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const float* Ap = (const float*)g.A.ptr + 2 * ((long long)f * g.A.sb + (long long)bz * g.A.sb2);
  const float* Bp = (const float*)g.B.ptr + 2 * ((long long)f * g.B.sb + (long long)bz * g.B.sb2);

  int a_i[A_PER_T], a_k[A_PER_T];
  long long a_rowoff[A_PER_T];
  int b_k[B_PER_T], b_j[B_PER_T];
  long long b_coloff[B_PER_T];
#pragma unroll
  for (int r = 0; r < A_PER_T; ++r) {
    int e = t + r * NT;
    if (AKM) { a_k[r] = e % BKC; a_i[r] = e / BKC; }
    else     { a_i[r] = e % BM;  a_k[r] = e / BM; }
    int gi = m0 + a_i[r];
    a_rowoff[r] = gi < M ? split_off(g.fm, gi, g.A.sxh, g.A.sxl) : -1;
  }
#pragma unroll
  for (int r = 0; r < B_PER_T; ++r) {
    int e = t + r * NT;
    if (BKM) { b_k[r] = e % BKC; b_j[r] = e / BKC; }
    else     { b_j[r] = e % BN;  b_k[r] = e / BN; }
    int gj = n0 + b_j[r];
    b_coloff[r] = gj < N ? split_off(g.fn, gj, g.B.syh, g.B.syl) : -1;
  }

  float2 ra[A_PER_T], rb[B_PER_T];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      int gk = k0 + a_k[r];
      float2 v = make_float2(0.f, 0.f);
      if (a_rowoff[r] >= 0 && gk < kend) v = *(const float2*)(Ap + 2 * (a_rowoff[r] + split_off(g.fk, gk, g.A.syh, g.A.syl)));
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      int gk = k0 + b_k[r];
      float2 v = make_float2(0.f, 0.f);
      if (b_coloff[r] >= 0 && gk < kend) v = *(const float2*)(Bp + 2 * (b_coloff[r] + split_off(g.fk, gk, g.B.sxh, g.B.sxl)));
      rb[r] = v;
    }
  };
  // hi (and lo) bfloat16 values of x
  auto split2 = [&](float x, float& hi, float& lo) {
    hi = round_bf16(x);
    lo = BF == 3 ? round_bf16(x - hi) : 0.f;
  };
  auto store_stage = [&](int bi) {
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      float re = ra[r].x, im = g.A.conj ? -ra[r].y : ra[r].y;
      float rh, rl, ih, il;
      split2(re, rh, rl);
      split2(im, ih, il);
      *(uint32_t*)&Asb[bi][0][a_i[r]][2 * a_k[r]] = bf16_pair(rh, ih);
      if constexpr (BF == 3) *(uint32_t*)&Asb[bi][1][a_i[r]][2 * a_k[r]] = bf16_pair(rl, il);
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      float re = rb[r].x, im = g.B.conj ? -rb[r].y : rb[r].y;
      float rh, rl, ih, il;
      split2(re, rh, rl);
      split2(im, ih, il);
      // column 2 jc: (k = 2kc, 2kc+1) = (re, -im); column 2 jc + 1: (im, re)
      *(uint32_t*)&Bsb[bi][0][2 * b_j[r]][2 * b_k[r]] = bf16_pair(rh, -ih);
      *(uint32_t*)&Bsb[bi][0][2 * b_j[r] + 1][2 * b_k[r]] = bf16_pair(ih, rh);
      if constexpr (BF == 3) {
        *(uint32_t*)&Bsb[bi][1][2 * b_j[r]][2 * b_k[r]] = bf16_pair(rl, -il);
        *(uint32_t*)&Bsb[bi][1][2 * b_j[r] + 1][2 * b_k[r]] = bf16_pair(il, rl);
      }
    }
  };

  constexpr int MI = BM / 32;
  constexpr int NJ = BN / 16;
  acc_t acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.f;
  const int l16 = lane & 15, lq = lane >> 4;

  if (kbeg < kend) {
    load_stage(kbeg);
    store_stage(0);
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += BKC) {
      const bool more = k0 + BKC < kend;
      if (more) load_stage(k0 + BKC);
      // lane (l16, lq) supplies A[row l16][k = 8 lq .. 8 lq + 7] and
      // B[k = 8 lq .. 8 lq + 7][column l16]
      shortx8 ah[MI], bh[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) ah[i] = *(const shortx8*)&Asb[cur][0][wm * (BM / 2) + i * 16 + l16][8 * lq];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bh[j] = *(const shortx8*)&Bsb[cur][0][wn * BN + j * 16 + l16][8 * lq];
      if constexpr (BF == 3) {
        shortx8 al[MI], bl[NJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) al[i] = *(const shortx8*)&Asb[cur][1][wm * (BM / 2) + i * 16 + l16][8 * lq];
#pragma unroll
        for (int j = 0; j < NJ; ++j) bl[j] = *(const shortx8*)&Bsb[cur][1][wn * BN + j * 16 + l16][8 * lq];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                                __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                                __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
          }
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                              __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
      if (more) store_stage(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }

  float* Cp = (float*)g.C.ptr + 2 * ((long long)f * g.C.sb + (long long)bz * g.C.sb2 + (long long)blockIdx.y * g.csplit);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    int jr = wn * BN + j * 16 + l16;
    int gj = n0 + (jr >> 1);
    long long coff = gj < N ? split_off(g.fn, gj, g.C.syh, g.C.syl) : -1;
#pragma unroll
    for (int i = 0; i < MI; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[i][j][r];
        float pv = __shfl_xor(v, 1);
        int gi = m0 + wm * (BM / 2) + i * 16 + lq * 4 + r;
        if (!(lane & 1) && coff >= 0 && gi < M) {
          long long o = split_off(g.fm, gi, g.C.sxh, g.C.sxl) + coff;
          float2* dst = (float2*)(Cp + 2 * o);
          float2 w = make_float2(v, pv);
          if (g.accumulate) {
            float2 old = *dst;
            w.x += old.x;
            w.y += old.y;
          }
          *dst = w;
        }
      }
    }
  }
}

// Sum of K-chunk partial results: out[i][j] = sum_c part[c][i][j], i, j < n
// (j <= i only when `lower`); partials have leading dimension ldp, out ld.
__global__ void ksplit_reduce_kernel(const double2* __restrict__ part, long long cstride, int nsplit, int ldp,
                                     double2* __restrict__ out, int ld, DimExpr nrows, DimExpr ncols,
                                     long long bstride_part, long long bstride_out, int lower) {
  const int b = blockIdx.z;
  const int nr = min(dim_eval(nrows, b), (int)gridDim.y);
  const int i = blockIdx.y;
  if (i >= nr) return;
  const int nc = min(min(dim_eval(ncols, b), min(ld, ldp)), lower ? i + 1 : ld);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += gridDim.x * blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    const double2* p = part + b * bstride_part + (long long)i * ldp + j;
    for (int c = 0; c < nsplit; ++c) {
      double2 v = p[c * cstride];
      s.x += v.x;
      s.y += v.y;
    }
    out[b * bstride_out + (long long)i * ld + j] = s;
  }
}

// Products with at most SM_M output rows and SM_K depth (the encode's
// projections R_{k+1} = U^H M at the first sites: 2-16 rows, 2-16 deep, up to
// 2^21 columns per field).  MFMA tiles would be almost all padding and the
// work is a single pass over B and C, so each thread streams whole output
// columns: op(A) (at most 16 x 16) sits in LDS, the thread loads its column
// of op(B) and writes its column of C.  FP32 or FP64 arithmetic as the
// inputs (no bfloat16 rounding: only the plain precision forms come here).
constexpr int SM_M = 16, SM_K = 16, SM_NT = 256;

template <typename T>
__global__ __launch_bounds__(SM_NT) void gemm_smallmk_kernel(GemmArgs g) {
  typedef typename Vec2<T>::t t2;
  const int f = blockIdx.z;
  const int M = min(min(dim_eval(g.M, f), g.Mmax), SM_M), N = min(dim_eval(g.N, f), g.Nmax);
  const int K = min(min(dim_eval(g.K, f), g.Kmax), SM_K);
  __shared__ t2 As[SM_M][SM_K];
  const T* Ap = (const T*)g.A.ptr + 2 * ((long long)f * g.A.sb);
  const T* Bp = (const T*)g.B.ptr + 2 * ((long long)f * g.B.sb);
  T* Cp = (T*)g.C.ptr + 2 * ((long long)f * g.C.sb);
  for (int e = threadIdx.x; e < SM_M * SM_K; e += SM_NT) {
    const int i = e / SM_K, p = e - i * SM_K;
    t2 v;
    v.x = 0; v.y = 0;
    if (i < M && p < K) {
      v = *(const t2*)(Ap + 2 * (split_off(g.fm, i, g.A.sxh, g.A.sxl) + split_off(g.fk, p, g.A.syh, g.A.syl)));
      if (g.A.conj) v.y = -v.y;
    }
    As[i][p] = v;
  }
  __syncthreads();
  long long boff[SM_K];
#pragma unroll
  for (int p = 0; p < SM_K; ++p) boff[p] = p < K ? split_off(g.fk, p, g.B.sxh, g.B.sxl) : 0;
  for (int j = blockIdx.x * SM_NT + threadIdx.x; j < N; j += gridDim.x * SM_NT) {
    const long long bc = split_off(g.fn, j, g.B.syh, g.B.syl);
    const long long cc = split_off(g.fn, j, g.C.syh, g.C.syl);
    t2 b[SM_K];
#pragma unroll
    for (int p = 0; p < SM_K; ++p) {
      b[p].x = 0; b[p].y = 0;
      if (p < K) {
        b[p] = *(const t2*)(Bp + 2 * (boff[p] + bc));
        if (g.B.conj) b[p].y = -b[p].y;
      }
    }
#pragma unroll
    for (int i = 0; i < SM_M; ++i) {
      if (i >= M) break;
      T re = 0, im = 0;
#pragma unroll
      for (int p = 0; p < SM_K; ++p) {
        const t2 a = As[i][p];
        re = fma(a.x, b[p].x, fma(-a.y, b[p].y, re));
        im = fma(a.x, b[p].y, fma(a.y, b[p].x, im));
      }
      t2* dst = (t2*)(Cp + 2 * (split_off(g.fm, i, g.C.sxh, g.C.sxl) + cc));
      if (g.accumulate) {
        const t2 o = *dst;
        re += o.x;
        im += o.y;
      }
      t2 w;
      w.x = re;
      w.y = im;
      *dst = w;
    }
  }
}

// Gram matrices of very few rows: G = X X^H (lower triangle) for an n x K
// operand X with n <= SK_N and K large (the first encode sites: 2, 4, 8
// rows against up to 2^21 columns).  A tile-based MFMA product would waste
// almost all of its work on padding here, and the data is read once, so
// this is a streaming reduction: each thread takes columns k = kbeg + t,
// kbeg + t + 256, ... of one K chunk, accumulates the n(n+1)/2 products
// x_i conj(x_j) in FP64 registers, and the workgroup's sums (DPP within
// waves, LDS across them) go to its own partial n x n block; the K-chunk
// partials are summed by ksplit_reduce.  Grid: (K chunks, 1, fields).
constexpr int SK_N = 8;
constexpr int SK_NT = 256;
constexpr int SK_P = SK_N * (SK_N + 1) / 2;


template <typename TIn>
__global__ __launch_bounds__(SK_NT) void gram_skinny_kernel(Operand A, DimExpr Mexp, DimExpr Kexp, FastDiv fm,
                                                            FastDiv fk, int kmax, int nsplit, double2* part,
                                                            int ldp) {
  typedef typename Vec2<TIn>::t in2;
  const int f = blockIdx.z, sp = blockIdx.x;
  const int n = min(dim_eval(Mexp, f), SK_N);
  const int K = min(dim_eval(Kexp, f), kmax);
  int chunk = (K + nsplit - 1) / nsplit;
  const int kbeg = sp * chunk, kend = min(K, kbeg + chunk);
  const TIn* Ap = (const TIn*)A.ptr + 2 * ((long long)f * A.sb);
  long long ro[SK_N];
#pragma unroll
  for (int i = 0; i < SK_N; ++i) ro[i] = i < n ? split_off(fm, i, A.sxh, A.sxl) : 0;
  double ar[SK_P], ai[SK_P];
#pragma unroll
  for (int q = 0; q < SK_P; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
  const double cs = A.conj ? -1.0 : 1.0;
  for (int k = kbeg + (int)threadIdx.x; k < kend; k += SK_NT) {
    const long long ko = split_off(fk, k, A.syh, A.syl);
    double xr[SK_N], xi[SK_N];
#pragma unroll
    for (int i = 0; i < SK_N; ++i) {
      in2 v;
      v.x = 0; v.y = 0;
      if (i < n) v = *(const in2*)(Ap + 2 * (ro[i] + ko));
      xr[i] = (double)v.x;
      xi[i] = cs * (double)v.y;
    }
    int q = 0;
#pragma unroll
    for (int i = 0; i < SK_N; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j, ++q) {
        // x_i conj(x_j)
        ar[q] = fma(xr[i], xr[j], fma(xi[i], xi[j], ar[q]));
        ai[q] = fma(xi[i], xr[j], fma(-xr[i], xi[j], ai[q]));
      }
  }
  __shared__ double red[SK_NT / 64][2 * SK_P];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int q = 0;
#pragma unroll
  for (int i = 0; i < SK_N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++q) {
      if (i < n) {
        double sr = ar[q], si = ai[q];
        wave_sum2_u(sr, si);
        if (lane == 0) { red[wv][2 * q] = sr; red[wv][2 * q + 1] = si; }
      }
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < SK_P) {
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    const int j = t - i * (i + 1) / 2;
    if (i < n) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int w = 0; w < SK_NT / 64; ++w) { sr += red[w][2 * t]; si += red[w][2 * t + 1]; }
      part[((long long)f * nsplit + sp) * ldp * ldp + (long long)i * ldp + j] = make_double2(sr, si);
    }
  }
}

// ---------------------------------------------------------------- host side

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d < 1 ? 1 : d;
  uint32_t l = 0;
  while ((1ull << l) < f.d) ++l;
  f.shift = l;
  f.mul = (uint32_t)(((1ull << 32) * ((1ull << l) - f.d)) / f.d + 1);
  return f;
}

template <typename TIn, typename TC, typename TOut, int BF, int BM, int BN>
static hipError_t launch_tile(const GemmArgs& g, dim3 grid, bool akm, bool bkm, hipStream_t s) {
  if constexpr (BF != 0) {
    if (akm && bkm) hipLaunchKernelGGL((cgemm_bf16_kernel<true, true, BF, BM, BN>), grid, dim3(NT), 0, s, g);
    else if (akm) hipLaunchKernelGGL((cgemm_bf16_kernel<true, false, BF, BM, BN>), grid, dim3(NT), 0, s, g);
    else if (bkm) hipLaunchKernelGGL((cgemm_bf16_kernel<false, true, BF, BM, BN>), grid, dim3(NT), 0, s, g);
    else hipLaunchKernelGGL((cgemm_bf16_kernel<false, false, BF, BM, BN>), grid, dim3(NT), 0, s, g);
    return hipGetLastError();
  }
  if (akm && bkm) hipLaunchKernelGGL((cgemm_kernel<TIn, TC, TOut, true, true, BM, BN>), grid, dim3(NT), 0, s, g);
  else if (akm) hipLaunchKernelGGL((cgemm_kernel<TIn, TC, TOut, true, false, BM, BN>), grid, dim3(NT), 0, s, g);
  else if (bkm) hipLaunchKernelGGL((cgemm_kernel<TIn, TC, TOut, false, true, BM, BN>), grid, dim3(NT), 0, s, g);
  else hipLaunchKernelGGL((cgemm_kernel<TIn, TC, TOut, false, false, BM, BN>), grid, dim3(NT), 0, s, g);
  return hipGetLastError();
}

template <typename TIn, typename TC, typename TOut, int BF = 0>
static hipError_t launch_typed(const GemmArgs& g, dim3 grid, bool akm, bool bkm, int tile, hipStream_t s) {
  constexpr bool wide = sizeof(TIn) == 4 && sizeof(TC) == 4 && BF == 0;
  switch (tile) {
    case 1: return launch_tile<TIn, TC, TOut, BF, 32, 64>(g, grid, akm, bkm, s);
    case 2: return launch_tile<TIn, TC, TOut, BF, 32, 32>(g, grid, akm, bkm, s);
    case 3:
      if constexpr (wide) return launch_tile<TIn, TC, TOut, BF, 128, 64>(g, grid, akm, bkm, s);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (wide) return launch_tile<TIn, TC, TOut, BF, 128, 128>(g, grid, akm, bkm, s);
      return hipErrorInvalidValue;
    default: return launch_tile<TIn, TC, TOut, BF, 64, 64>(g, grid, akm, bkm, s);
  }
}

// Tile variants available to one element-type combination.
static int tile_count(int types) { return types == GEMM_F32 ? N_TILES : N_TILES_NARROW; }

// ---------------------------------------------------------------- autotuner
// Per call shape (element types, host bounds of M and N, grid depth = inner
// batch x fields, operand access pattern) the tile variant measured fastest
// on this device.  Shapes are collected while recording is on, each with the
// largest depth one workgroup reduces over (K, or its K-split chunk); tuning
// times every variant on synthetic operands of that shape and depth.
namespace {
struct TileKey {
  int types, mb, nb, zb, pat;
  bool operator<(const TileKey& o) const {
    if (types != o.types) return types < o.types;
    if (mb != o.mb) return mb < o.mb;
    if (nb != o.nb) return nb < o.nb;
    if (zb != o.zb) return zb < o.zb;
    return pat < o.pat;
  }
};
std::map<TileKey, int> g_tiles;
std::map<TileKey, int> g_seen;       // recorded shapes -> largest depth per workgroup
bool g_record = false;
constexpr int TUNE_KMIN = 16, TUNE_KMAX = 1024;  // synthetic depth range
constexpr int TUNE_ZMAX = 2048;      // grid depth used for timing (larger grids all saturate)
constexpr long long TUNE_MN_MAX = 4096ll * 4096;  // larger outputs keep the 64 x 64 tile
constexpr size_t TUNE_BYTES = 256ull << 20;     // synthetic operands per shape

// Synthetic depth for a recorded depth: rounded up to a whole stage, clamped.
int tune_k(int kd) {
  const int k = (kd + BKC - 1) / BKC * BKC;
  return std::min(std::max(k, TUNE_KMIN), TUNE_KMAX);
}

// Grid depth used to time shape k at depth kk (0: not tuned).
int tune_depth(const TileKey& k, int kk) {
  if ((long long)k.mb * k.nb > TUNE_MN_MAX) return 0;
  const size_t esz = k.types == GEMM_F64 ? 16 : 8;
  const size_t csz = (k.types == GEMM_F64 || k.types == GEMM_F32_GRAM64) ? 16 : 8;
  const size_t per = (size_t)k.mb * kk * esz + (size_t)kk * k.nb * esz + (size_t)k.mb * k.nb * csz + 768;
  size_t z = std::min<size_t>({(size_t)k.zb, (size_t)TUNE_ZMAX, TUNE_BYTES / per});
  return (int)z;
}
}  // namespace

static TileKey make_key(const GemmSpec& sp, bool akm, bool bkm) {
  TileKey k;
  k.types = sp.types;
  k.mb = sp.m_bound;
  k.nb = sp.n_bound;
  k.zb = (sp.batch_bound < 1 ? 1 : sp.batch_bound) * (sp.nfield < 1 ? 1 : sp.nfield) * (sp.ksplit < 1 ? 1 : sp.ksplit);
  k.pat = (akm ? 1 : 0) | (bkm ? 2 : 0);
  return k;
}

static hipError_t launch_variant(const GemmArgs& g0, int types, bool akm, bool bkm, int tile, int m_bound,
                                 int n_bound, int zdim, int ksplit, hipStream_t s) {
  GemmArgs g = g0;
  const int bm = TILE_M[tile], bn = TILE_N[tile];
  int tiles_m = (m_bound + bm - 1) / bm;
  int tiles_n = (n_bound + bn - 1) / bn;
  if (tiles_m < 1 || tiles_n < 1 || zdim < 1) return hipSuccess;
  g.tiles_n = tiles_n;
  dim3 grid(tiles_m * tiles_n, ksplit, zdim);
  switch (types) {
    case GEMM_F32: return launch_typed<float, float, float>(g, grid, akm, bkm, tile, s);
    case GEMM_F32_GRAM64: return launch_typed<float, double, double>(g, grid, akm, bkm, tile, s);
    case GEMM_F64: return launch_typed<double, double, double>(g, grid, akm, bkm, tile, s);
    case GEMM_BF16: return launch_typed<float, float, float, 1>(g, grid, akm, bkm, tile, s);
    case GEMM_BF16X3: return launch_typed<float, float, float, 3>(g, grid, akm, bkm, tile, s);
  }
  return hipErrorInvalidValue;
}

__global__ void gemm_flops_kernel(DimExpr M, DimExpr N, DimExpr K, DimExpr batch, int mb, int nb, int kb, int bb,
                                  int nf, double scale, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int f = 0; f < nf; ++f) {
    const double m = min(dim_eval(M, f), mb), n = min(dim_eval(N, f), nb), k = min(dim_eval(K, f), kb);
    s += m * n * k * (double)min(dim_eval(batch, f), bb);
  }
  out[0] += scale * s;
}

hipError_t gemm_flops(const GemmSpec& sp, double scale, double* out, hipStream_t s) {
  const int slot = sp.types == GEMM_F32_GRAM64 || sp.types == GEMM_F64 ? 1 : 0;
  hipLaunchKernelGGL(gemm_flops_kernel, dim3(1), dim3(64), 0, s, sp.M, sp.N, sp.K, sp.batch, sp.m_bound,
                     sp.n_bound, sp.k_bound, sp.batch_bound, sp.nfield, scale, out + slot);
  return hipGetLastError();
}

hipError_t gemm_launch(const GemmSpec& sp, hipStream_t s) {
  GemmArgs g;
  g.M = sp.M; g.N = sp.N; g.K = sp.K; g.batch = sp.batch;
  g.b2cap = sp.batch_bound < 1 ? 1 : sp.batch_bound;
  g.fm = make_fastdiv(sp.mlo); g.fn = make_fastdiv(sp.nlo); g.fk = make_fastdiv(sp.klo);
  g.A = sp.A; g.B = sp.B; g.C = sp.C;
  g.accumulate = sp.accumulate;
  g.lower = sp.lower;
  g.ksplit = sp.ksplit < 1 ? 1 : sp.ksplit;
  g.csplit = sp.csplit;
  if (sp.m_bound < 1 || sp.n_bound < 1 || sp.batch_bound < 1 || sp.nfield < 1) return hipSuccess;
  g.Mmax = sp.m_bound; g.Nmax = sp.n_bound; g.Kmax = sp.k_bound; g.Bmax = sp.batch_bound;
  // coalescing pattern: which index is unit-stride in memory
  if (sp.m_bound <= SM_M && sp.k_bound <= SM_K && g.ksplit == 1 && sp.batch_bound == 1 &&
      (sp.types == GEMM_F32 || sp.types == GEMM_F64)) {
    g.Mmax = sp.m_bound; g.Nmax = sp.n_bound; g.Kmax = sp.k_bound; g.Bmax = 1;
    const int gx = (int)std::min<long long>(((long long)sp.n_bound + SM_NT - 1) / SM_NT, 64);
    const dim3 grid(gx, 1, sp.nfield);
    if (sp.types == GEMM_F32) hipLaunchKernelGGL(gemm_smallmk_kernel<float>, grid, dim3(SM_NT), 0, s, g);
    else hipLaunchKernelGGL(gemm_smallmk_kernel<double>, grid, dim3(SM_NT), 0, s, g);
    return hipGetLastError();
  }
  bool akm = (sp.A.syl == 1 && sp.klo > 1) || (sp.klo == 1 && sp.A.syh == 1);
  bool bkm = (sp.B.sxl == 1 && sp.klo > 1) || (sp.klo == 1 && sp.B.sxh == 1);
  TileKey key = make_key(sp, akm, bkm);
  // every product is recorded, the FP64-accumulating Gram matrices included:
  // their K-split chunks are short enough for the tuner's synthetic K
  if (g_record) {
    const int kd = (sp.k_bound + g.ksplit - 1) / g.ksplit;
    int& rec = g_seen[key];
    rec = std::max(rec, kd);
  }
  auto it = g_tiles.find(key);
  // untuned default: 32-row tiles when the rows (or both sides) are that small
  const int tile = it != g_tiles.end() ? it->second
                                       : (sp.m_bound <= 32 ? (sp.n_bound <= 32 ? 2 : 1) : 0);
  return launch_variant(g, sp.types, akm, bkm, tile, sp.m_bound, sp.n_bound, sp.batch_bound * sp.nfield, g.ksplit,
                        s);
}

hipError_t gram_skinny(const GemmSpec& sp, int nsplit, double* part, int ldp, hipStream_t s) {
  if (sp.m_bound < 1 || sp.nfield < 1 || nsplit < 1) return hipSuccess;
  if (sp.m_bound > SK_N || ldp < sp.m_bound) return hipErrorInvalidValue;
  const dim3 grid(nsplit, 1, sp.nfield);
  const FastDiv fm = make_fastdiv(sp.mlo), fk = make_fastdiv(sp.klo);
  if (sp.types == GEMM_F32_GRAM64)
    hipLaunchKernelGGL(gram_skinny_kernel<float>, grid, dim3(SK_NT), 0, s, sp.A, sp.M, sp.K, fm, fk, sp.k_bound,
                       nsplit, (double2*)part, ldp);
  else if (sp.types == GEMM_F64)
    hipLaunchKernelGGL(gram_skinny_kernel<double>, grid, dim3(SK_NT), 0, s, sp.A, sp.M, sp.K, fm, fk, sp.k_bound,
                       nsplit, (double2*)part, ldp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

void autotune_record(bool on) {
  g_record = on;
  if (on) g_seen.clear();
}

size_t autotune_ws_bytes() {
  size_t need = 0;
  for (const auto& kv : g_seen) {
    const TileKey& k = kv.first;
    const int kk = tune_k(kv.second);
    const size_t esz = k.types == GEMM_F64 ? 16 : 8;
    const size_t csz = (k.types == GEMM_F64 || k.types == GEMM_F32_GRAM64) ? 16 : 8;
    const size_t z = (size_t)tune_depth(k, kk);
    if (z == 0) continue;
    size_t a = z * k.mb * kk * esz, b = z * kk * k.nb * esz;
    size_t c = z * k.mb * k.nb * csz;
    need = std::max(need, ((a + 255) / 256 + (b + 255) / 256 + (c + 255) / 256) * 256);
  }
  return need;
}

hipError_t autotune_run(void* ws, size_t ws_bytes, hipStream_t s, int* n_tuned) {
  int tuned = 0;
  if (ws_bytes < autotune_ws_bytes()) return hipErrorInvalidValue;
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) { hipEventDestroy(e0); return err; }
  for (const auto& kv : g_seen) {
    const TileKey& k = kv.first;
    const int kk = tune_k(kv.second);
    const size_t esz = k.types == GEMM_F64 ? 16 : 8;
    char* base = (char*)ws;
    const int zt = tune_depth(k, kk);
    if (zt == 0) continue;
    const size_t a = ((size_t)zt * k.mb * kk * esz + 255) / 256 * 256;
    const size_t b = ((size_t)zt * kk * k.nb * esz + 255) / 256 * 256;
    // plain row-major operands with the recorded access pattern: A [z][M][K]
    // (K unit stride if pat bit 0) or [z][K][M]; B likewise
    GemmArgs g;
    g.M = DimExpr{k.mb, nullptr, nullptr, 0};
    g.N = DimExpr{k.nb, nullptr, nullptr, 0};
    g.K = DimExpr{kk, nullptr, nullptr, 0};
    g.batch = DimExpr{1, nullptr, nullptr, 0};
    g.b2cap = 1;
    g.fm = make_fastdiv(1); g.fn = make_fastdiv(1); g.fk = make_fastdiv(1);
    const bool akm = k.pat & 1, bkm = (k.pat >> 1) & 1;
    g.A = Operand{base, akm ? kk : 1, 0, akm ? 1 : k.mb, 0, (long long)k.mb * kk, 0, 0};
    g.B = Operand{base + a, bkm ? 1 : k.nb, 0, bkm ? kk : 1, 0, (long long)kk * k.nb, 0, 0};
    g.C = Operand{base + a + b, k.nb, 0, 1, 0, (long long)k.mb * k.nb, 0, 0};
    g.accumulate = 0;
    g.lower = 0;
    g.ksplit = 1;
    g.csplit = 0;
    g.Mmax = k.mb; g.Nmax = k.nb; g.Kmax = kk; g.Bmax = 1;
    float best = 1e30f;
    int best_t = 0;
    for (int t = 0; t < tile_count(k.types); ++t) {
      // warm-up, then the mean of three launches
      err = launch_variant(g, k.types, akm, bkm, t, k.mb, k.nb, zt, 1, s);
      if (err != hipSuccess) break;
      hipEventRecord(e0, s);
      for (int r = 0; r < 3; ++r) launch_variant(g, k.types, akm, bkm, t, k.mb, k.nb, zt, 1, s);
      hipEventRecord(e1, s);
      err = hipEventSynchronize(e1);
      if (err != hipSuccess) break;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_t = t; }
    }
    if (err != hipSuccess) break;
    g_tiles[k] = best_t;
    ++tuned;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (n_tuned) *n_tuned = tuned;
  return err;
}

int autotune_export(int* out, int max_entries) {
  int n = 0;
  for (const auto& kv : g_tiles) {
    if (n < max_entries && out) {
      int* e = out + 6 * n;
      e[0] = kv.first.types; e[1] = kv.first.mb; e[2] = kv.first.nb; e[3] = kv.first.zb; e[4] = kv.first.pat;
      e[5] = kv.second;
    }
    ++n;
  }
  return n;
}

int autotune_import(const int* entries, int n) {
  int bad = 0;
  for (int i = 0; i < n; ++i) {
    const int* e = entries + 6 * i;
    if (e[5] < 0 || e[5] >= tile_count(e[0]) || e[1] < 1 || e[2] < 1 || e[3] < 1) { ++bad; continue; }
    TileKey k;
    k.types = e[0]; k.mb = e[1]; k.nb = e[2]; k.zb = e[3]; k.pat = e[4];
    g_tiles[k] = e[5];
  }
  return bad;
}

void autotune_clear() {
  g_tiles.clear();
  g_seen.clear();
}

hipError_t ksplit_reduce(const void* part, long long cstride, int nsplit, int ldp, void* out, int ld,
                         DimExpr nrows, DimExpr ncols, int rows_bound, int cols_bound,
                         long long bstride_part, long long bstride_out, int batch_bound, int lower,
                         hipStream_t s) {
  int bx = (cols_bound + 255) / 256;
  if (bx < 1 || rows_bound < 1 || batch_bound < 1) return hipSuccess;
  hipLaunchKernelGGL(ksplit_reduce_kernel, dim3(bx, rows_bound, batch_bound), dim3(256), 0, s,
                     (const double2*)part, cstride, nsplit, ldp, (double2*)out, ld, nrows, ncols,
                     bstride_part, bstride_out, lower);
  return hipGetLastError();
}

}  // namespace qtt
