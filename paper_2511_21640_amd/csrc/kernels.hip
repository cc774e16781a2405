// Device kernels of the sigma build (gfx950 / CDNA4).
//
// Complex tensors are interleaved (re, im) float64.  Contractions run on the
// matrix cores: the complex product is split into real/imaginary planes in LDS
// and formed with four real MFMA products per k-step (Re*Re - Im*Im into the
// real accumulator, Re*Im + Im*Re into the imaginary one).
#include "internal.h"

#include <hip/hip_bf16.h>
#include <mutex>
#include <stdexcept>

namespace adc {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

static inline unsigned nblocks(int64_t n, int t) {
  int64_t b = (n + t - 1) / t;
  if (b > 65535LL * 16) b = 65535LL * 16;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// C offset of a row (or column) index under an OutMap group (see internal.h)
__device__ __forceinline__ int64_t omap(int64_t x, int n, const int64_t* d, const int64_t* st, int64_t s1) {
  if (n == 0) return x * s1;
  uint32_t u = (uint32_t)x;
  int64_t off = 0;
  for (int q = n - 1; q > 0; --q) {
    const uint32_t dq = (uint32_t)d[q];
    const uint32_t v = u / dq;
    off += (int64_t)(u - v * dq) * st[q];
    u = v;
  }
  return off + (int64_t)u * st[0];
}

typedef double d2v __attribute__((ext_vector_type(2)));

// Epilogue of a complex GEMM tile held in MFMA accumulators: register r of
// block (i, j) of this lane is element (rows[i][r], cols[j]).  The output
// offsets of the rows and columns are computed once; with beta != 0 the old
// values of a block row are all loaded before any of them is stored, so that
// the loads are in flight together; every access is one 16-byte vector.  P
// (split-K partials of this split, row-major M x N) replaces the output when
// given.
typedef float f2v __attribute__((ext_vector_type(2)));

template <int WM, int WN, class AccT>
__device__ __forceinline__ void store_tile(int64_t M, int64_t N, double2* C, double2* P, const OutMap& om,
                                           int64_t scm, int64_t scn, cplx alpha, cplx beta,
                                           const int64_t (&rows)[WM][4], const int64_t (&cols)[WN],
                                           const AccT (&accR)[WM][WN], const AccT (&accI)[WM][WN], int c32) {
  if (P) {
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (rows[i][r] < M && cols[j] < N)
            *(d2v*)(P + rows[i][r] * N + cols[j]) = d2v{(double)accR[i][j][r], (double)accI[i][j][r]};
    return;
  }
  const bool has_beta = (beta.re != 0.0 || beta.im != 0.0);
  int64_t coff[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) coff[j] = cols[j] < N ? omap(cols[j], om.nn, om.nd, om.ns, scn) : 0;
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    int64_t roff[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) roff[r] = rows[i][r] < M ? omap(rows[i][r], om.nm, om.md, om.ms, scm) : 0;
    d2v old[WN][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        old[j][r] = d2v{0.0, 0.0};
        if (has_beta && rows[i][r] < M && cols[j] < N) {
          if (c32) {
            const f2v f = *((const f2v*)C + roff[r] + coff[j]);
            old[j][r] = d2v{(double)f.x, (double)f.y};
          } else {
            old[j][r] = *(const d2v*)(C + roff[r] + coff[j]);
          }
        }
      }
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (rows[i][r] < M && cols[j] < N) {
          const double cr = accR[i][j][r], ci = accI[i][j][r];
          d2v o;
          o.x = alpha.re * cr - alpha.im * ci + beta.re * old[j][r].x - beta.im * old[j][r].y;
          o.y = alpha.re * ci + alpha.im * cr + beta.re * old[j][r].y + beta.im * old[j][r].x;
          if (c32) *((f2v*)C + roff[r] + coff[j]) = f2v{(float)o.x, (float)o.y};
          else *(d2v*)(C + roff[r] + coff[j]) = o;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Complex GEMM on the matrix cores.
//
// One 256-thread workgroup (4 waves in a 2x2 arrangement) computes a
// (32*WM) x (32*WN) tile; each wave owns WM x WN blocks of 16x16.  Per k-step
// of 4 a wave issues four real MFMA per block (Re*Re, -Im*Im into the real
// accumulator, Re*Im, Im*Re into the imaginary one).  The K loop is register
// double-buffered: the next 16-deep slice is fetched from global memory into
// registers while the MFMAs consume the current slice from LDS.  Tiles are
// handed out so that each of the 8 XCDs (workgroups are dispatched round-robin
// over them) works on a contiguous range of tiles and reuses row blocks in its
// own L2.
// ---------------------------------------------------------------------------
constexpr int TK = 16;

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma16(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<double> { typedef dbl4 type; };
template <> struct Acc<float> { typedef flt4 type; };

// row of register r in a 16x16 MFMA result held by lane l
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T, int WM, int WN, int TAG>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmDesc p) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int RA = BM * TK / 256, RB = BN * TK / 256;   // elements per thread
  typedef typename Acc<T>::type acc_t;
  __shared__ T sAr[TK][BM + 1], sAi[TK][BM + 1], sBr[TK][BN + 1], sBi[TK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // XCD-aware tile index
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN, ntile = tilesM * tilesN;
  const int64_t L = blockIdx.x;
  int64_t tile = L;
  {
    const int64_t q = ntile / 8, r = ntile % 8, x = L % 8, slot = L / 8;
    tile = x * q + (x < r ? x : r) + slot;
  }
  const int64_t m0 = (tile / tilesN) * BM, n0 = (tile % tilesN) * BN;
  const int64_t zz = blockIdx.y;
  const int64_t sidx = zz / p.batch, bz = zz - sidx * p.batch;
  const int64_t kbeg = sidx * p.kchunk;
  const int64_t kend = (kbeg + p.kchunk < p.K) ? kbeg + p.kchunk : p.K;
  const double2* A = p.A + bz * p.sab;
  const double2* B = p.B + bz * p.sbb;
  double2* C = p.c32 ? (double2*)((float2*)p.C + bz * p.scb) : p.C + bz * p.scb;
  const int wr = wave >> 1, wc = wave & 1;
  const bool aK = (p.sak == 1), bK = (p.sbk == 1);
  const T sa = p.conjA ? T(-1) : T(1), sb = p.conjB ? T(-1) : T(1);

  acc_t accR[WM][WN], accI[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      accR[i][j] = acc_t{0, 0, 0, 0};
      accI[i][j] = acc_t{0, 0, 0, 0};
    }
  double2 ra[RA], rb[RB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int m, k;
      if (aK) { m = (tid >> 4) + 16 * r; k = tid & 15; }
      else    { m = tid % BM; k = tid / BM + (256 / BM) * r; }
      const int64_t gm = m0 + m, gk = k0 + k;
      ra[r] = (gm < p.M && gk < kend) ? A[gm * p.sam + gk * p.sak] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int n, k;
      if (bK) { n = (tid >> 4) + 16 * r; k = tid & 15; }
      else    { n = tid % BN; k = tid / BN + (256 / BN) * r; }
      const int64_t gn = n0 + n, gk = k0 + k;
      rb[r] = (gn < p.N && gk < kend) ? B[gk * p.sbk + gn * p.sbn] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int m, k;
      if (aK) { m = (tid >> 4) + 16 * r; k = tid & 15; }
      else    { m = tid % BM; k = tid / BM + (256 / BM) * r; }
      sAr[k][m] = (T)ra[r].x;
      sAi[k][m] = sa * (T)ra[r].y;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int n, k;
      if (bK) { n = (tid >> 4) + 16 * r; k = tid & 15; }
      else    { n = tid % BN; k = tid / BN + (256 / BN) * r; }
      sBr[k][n] = (T)rb[r].x;
      sBi[k][n] = sb * (T)rb[r].y;
    }
  };
  if (kbeg < kend) {
    gload(kbeg);
    sstore();
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
    const bool more = k0 + TK < kend;
    if (more) gload(k0 + TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[WM], ai[WM], nai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ar[i] = sAr[kr][32 * WM / 2 * wr + 16 * i + (lane & 15)];
        ai[i] = sAi[kr][32 * WM / 2 * wr + 16 * i + (lane & 15)];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = sBr[kr][32 * WN / 2 * wc + 16 * j + (lane & 15)];
        bi[j] = sBi[kr][32 * WN / 2 * wc + 16 * j + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          accR[i][j] = mfma16(ar[i], br[j], accR[i][j]);
          accR[i][j] = mfma16(nai[i], bi[j], accR[i][j]);
          accI[i][j] = mfma16(ar[i], bi[j], accI[i][j]);
          accI[i][j] = mfma16(ai[i], br[j], accI[i][j]);
        }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }
  {
    int64_t rows[WM][4], cols[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[i][r] = m0 + 32 * WM / 2 * wr + 16 * i + acc_row<T>(lane, r);
#pragma unroll
    for (int j = 0; j < WN; ++j) cols[j] = n0 + 32 * WN / 2 * wc + 16 * j + (lane & 15);
    double2* P = p.nsplit > 1 ? p.P + (sidx * p.batch + bz) * p.M * p.N : nullptr;
    store_tile<WM, WN>(p.M, p.N, C, P, p.om, p.scm, p.scn, p.alpha, p.beta, rows, cols, accR, accI, p.c32);
  }
}

// Split-K reduction: out = alpha * sum_s P[s][idx] + beta * out for the
// outputs idx = (batch, m, n).  64 outputs per block; the splits of each are
// spread over four thread rows (independent loads in flight) and summed in LDS.
struct ReduceArgs {
  const double2* P;
  int64_t total, MN, N;
  int nsplit;
  double2* C;
  int64_t scb, scm, scn;
  OutMap om;
  cplx alpha, beta;
  int c32;
};
__global__ __launch_bounds__(256) void splitk_reduce_kernel(ReduceArgs a) {
  __shared__ double2 red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + tx;
  double sr = 0.0, si = 0.0;
  if (idx < a.total) {
#pragma unroll 4
    for (int s = ty; s < a.nsplit; s += 4) {
      const double2 v = a.P[(int64_t)s * a.total + idx];
      sr += v.x;
      si += v.y;
    }
  }
  red[ty][tx] = make_double2(sr, si);
  __syncthreads();
  if (ty != 0 || idx >= a.total) return;
  sr = (red[0][tx].x + red[1][tx].x) + (red[2][tx].x + red[3][tx].x);
  si = (red[0][tx].y + red[1][tx].y) + (red[2][tx].y + red[3][tx].y);
  const int64_t b = idx / a.MN, r = idx - b * a.MN, m = r / a.N, n = r - m * a.N;
  const int64_t off = b * a.scb + omap(m, a.om.nm, a.om.md, a.om.ms, a.scm) + omap(n, a.om.nn, a.om.nd, a.om.ns, a.scn);
  double ox = a.alpha.re * sr - a.alpha.im * si, oy = a.alpha.re * si + a.alpha.im * sr;
  if (a.beta.re != 0.0 || a.beta.im != 0.0) {
    double px, py;
    if (a.c32) {
      const float2 f = ((const float2*)a.C)[off];
      px = f.x; py = f.y;
    } else {
      const double2 d = a.C[off];
      px = d.x; py = d.y;
    }
    ox += a.beta.re * px - a.beta.im * py;
    oy += a.beta.re * py + a.beta.im * px;
  }
  if (a.c32) ((float2*)a.C)[off] = make_float2((float)ox, (float)oy);
  else a.C[off] = make_double2(ox, oy);
}
static void launch_reduce(const ReduceArgs& a, hipStream_t s) {
  if (a.total <= 0) return;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((a.total + 63) / 64)), dim3(256), 0, s, a);
}

void launch_splitk_reduce(const GemmDesc& g, hipStream_t s) {
  ReduceArgs a{g.P, g.batch * g.M * g.N, g.M * g.N, g.N, g.nsplit, g.C, g.scb, g.scm, g.scn, g.om, g.alpha, g.beta,
               g.c32};
  launch_reduce(a, s);
}

// ---------------------------------------------------------------------------
// Split-bf16 complex GEMM.  Each operand value is rounded to fp32 and split
// into bf16 hi = RNE(x) and lo = RNE(x - hi) when it is staged in LDS (four
// planes: re hi/lo, im hi/lo, k contiguous).  A real product x*y is formed as
// xh*yh + xh*yl + xl*yh with v_mfma_f32_16x16x32_bf16 (fp32 accumulation), so
// a complex 16x16x32 block costs 12 MFMA.  64x64 tile, 4 waves, k-slices of
// 32, register double buffering, XCD-aware tile order and split-K as above.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
constexpr int TKB = 32, PADB = 8;

__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  const __hip_bfloat16 h = __float2bfloat16(x);
  const __hip_bfloat16 l = __float2bfloat16(x - __bfloat162float(h));
  hi = __bfloat16_as_ushort(h);
  lo = __bfloat16_as_ushort(l);
}

__device__ __forceinline__ flt4 mfma_bf16(us8 a, us8 b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

template <int TAG>
__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(GemmDesc p) {
  constexpr int BM = 64, BN = 64, RA = BM * TKB / 256, RB = BN * TKB / 256;
  __shared__ __attribute__((aligned(16))) unsigned short sA[4][BM][TKB + PADB];
  __shared__ __attribute__((aligned(16))) unsigned short sB[4][BN][TKB + PADB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN, ntile = tilesM * tilesN;
  const int64_t L = blockIdx.x;
  int64_t tile;
  {
    const int64_t q = ntile / 8, r = ntile % 8, x = L % 8, slot = L / 8;
    tile = x * q + (x < r ? x : r) + slot;
  }
  const int64_t m0 = (tile / tilesN) * BM, n0 = (tile % tilesN) * BN;
  const int64_t zz = blockIdx.y;
  const int64_t sidx = zz / p.batch, bz = zz - sidx * p.batch;
  const int64_t kbeg = sidx * p.kchunk;
  const int64_t kend = (kbeg + p.kchunk < p.K) ? kbeg + p.kchunk : p.K;
  const double2* A = p.A + bz * p.sab;
  const double2* B = p.B + bz * p.sbb;
  double2* C = p.c32 ? (double2*)((float2*)p.C + bz * p.scb) : p.C + bz * p.scb;
  const int wr = wave >> 1, wc = wave & 1;
  const bool aK = (p.sak == 1), bK = (p.sbk == 1);
  const float sa = p.conjA ? -1.f : 1.f, sb = p.conjB ? -1.f : 1.f;
  flt4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  double2 ra[RA], rb[RB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int m, k;
      if (aK) { m = (tid >> 5) + 8 * r; k = tid & 31; }
      else    { m = tid & 63; k = (tid >> 6) + 4 * r; }
      const int64_t gm = m0 + m, gk = k0 + k;
      ra[r] = (gm < p.M && gk < kend) ? A[gm * p.sam + gk * p.sak] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int n, k;
      if (bK) { n = (tid >> 5) + 8 * r; k = tid & 31; }
      else    { n = tid & 63; k = (tid >> 6) + 4 * r; }
      const int64_t gn = n0 + n, gk = k0 + k;
      rb[r] = (gn < p.N && gk < kend) ? B[gk * p.sbk + gn * p.sbn] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int m, k;
      if (aK) { m = (tid >> 5) + 8 * r; k = tid & 31; }
      else    { m = tid & 63; k = (tid >> 6) + 4 * r; }
      unsigned short h0, l0, h1, l1;
      split_bf16((float)ra[r].x, h0, l0);
      split_bf16(sa * (float)ra[r].y, h1, l1);
      sA[0][m][k] = h0; sA[1][m][k] = l0; sA[2][m][k] = h1; sA[3][m][k] = l1;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int n, k;
      if (bK) { n = (tid >> 5) + 8 * r; k = tid & 31; }
      else    { n = tid & 63; k = (tid >> 6) + 4 * r; }
      unsigned short h0, l0, h1, l1;
      split_bf16((float)rb[r].x, h0, l0);
      split_bf16(sb * (float)rb[r].y, h1, l1);
      sB[0][n][k] = h0; sB[1][n][k] = l0; sB[2][n][k] = h1; sB[3][n][k] = l1;
    }
  };
  if (kbeg < kend) {
    gload(kbeg);
    sstore();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);
  const us8 sgn = us8{0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000};
  for (int64_t k0 = kbeg; k0 < kend; k0 += TKB) {
    const bool more = k0 + TKB < kend;
    if (more) gload(k0 + TKB);
    us8 a[2][4], b[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[i][q] = *(const us8*)&sA[q][32 * wr + 16 * i + (lane & 15)][kq];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = *(const us8*)&sB[q][32 * wc + 16 * j + (lane & 15)][kq];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const us8 nih = a[i][2] ^ sgn, nil = a[i][3] ^ sgn;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        flt4 cr = accR[i][j], ci = accI[i][j];
        cr = mfma_bf16(a[i][0], b[j][0], cr);
        cr = mfma_bf16(a[i][0], b[j][1], cr);
        cr = mfma_bf16(a[i][1], b[j][0], cr);
        cr = mfma_bf16(nih, b[j][2], cr);
        cr = mfma_bf16(nih, b[j][3], cr);
        cr = mfma_bf16(nil, b[j][2], cr);
        ci = mfma_bf16(a[i][0], b[j][2], ci);
        ci = mfma_bf16(a[i][0], b[j][3], ci);
        ci = mfma_bf16(a[i][1], b[j][2], ci);
        ci = mfma_bf16(a[i][2], b[j][0], ci);
        ci = mfma_bf16(a[i][2], b[j][1], ci);
        ci = mfma_bf16(a[i][3], b[j][0], ci);
        accR[i][j] = cr;
        accI[i][j] = ci;
      }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }
  {
    // v_mfma_f32_16x16x32_bf16 result: lane l, register r holds row 4(l/16) + r, column l%16
    int64_t rows[2][4], cols[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[i][r] = m0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
#pragma unroll
    for (int j = 0; j < 2; ++j) cols[j] = n0 + 32 * wc + 16 * j + (lane & 15);
    double2* P = p.nsplit > 1 ? p.P + (sidx * p.batch + bz) * p.M * p.N : nullptr;
    store_tile<2, 2>(p.M, p.N, C, P, p.om, p.scm, p.scn, p.alpha, p.beta, rows, cols, accR, accI, p.c32);
  }
}

static void launch_bf16x3(const GemmDesc& g, hipStream_t s) {
  const int64_t tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  dim3 grid((unsigned)tiles, (unsigned)(g.batch * g.nsplit));
  if (g.tag == 1) hipLaunchKernelGGL(zgemm_bf16x3_kernel<1>, grid, dim3(256), 0, s, g);
  else if (g.tag == 2) hipLaunchKernelGGL(zgemm_bf16x3_kernel<2>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(zgemm_bf16x3_kernel<0>, grid, dim3(256), 0, s, g);
}

// ---------------------------------------------------------------------------
// Split-bf16 GEMM on pre-split operands.  A and B are given as four planes
// (re hi, re lo, im hi, im lo) of bf16, [plane][rows][Kp] with K contiguous
// and zero-padded to Kp (a multiple of 32).  Tiles are streamed into LDS with
// 16-byte loads; there is no per-element arithmetic before the MFMAs.
// ---------------------------------------------------------------------------
__global__ void split_planes_kernel(const double2* src, int64_t rows, int64_t K, int64_t srow, int64_t sk, int conj,
                                    unsigned short* dst, int64_t Kp) {
  const int64_t total = rows * Kp;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / Kp, k = idx - r * Kp;
    unsigned short h0 = 0, l0 = 0, h1 = 0, l1 = 0;
    if (k < K) {
      const double2 v = src[r * srow + k * sk];
      split_bf16((float)v.x, h0, l0);
      split_bf16(conj ? -(float)v.y : (float)v.y, h1, l1);
    }
    dst[idx] = h0;
    dst[total + idx] = l0;
    dst[2 * total + idx] = h1;
    dst[3 * total + idx] = l1;
  }
}
void launch_split_planes(const double2* src, int64_t rows, int64_t K, int64_t srow, int64_t sk, int conj,
                         unsigned short* dst, int64_t Kp, hipStream_t s) {
  if (rows * Kp == 0) return;
  hipLaunchKernelGGL(split_planes_kernel, dim3(nblocks(rows * Kp, 256)), dim3(256), 0, s, src, rows, K, srow, sk, conj,
                     dst, Kp);
}

__device__ __forceinline__ int64_t digits_off(uint32_t x, int n, const int64_t* d, const int64_t* st) {
  int64_t off = 0;
  for (int q = n - 1; q > 0; --q) {
    const uint32_t dq = (uint32_t)d[q];
    const uint32_t v = x / dq;
    off += (int64_t)(x - v * dq) * st[q];
    x = v;
  }
  return off + (int64_t)x * st[0];
}

__device__ __forceinline__ void put_planes(unsigned short* dst, int64_t plane, int64_t at, double2 v, int conj) {
  unsigned short h0, l0, h1, l1;
  split_bf16((float)v.x, h0, l0);
  split_bf16(conj ? -(float)v.y : (float)v.y, h1, l1);
  dst[at] = h0;
  dst[plane + at] = l0;
  dst[2 * plane + at] = h1;
  dst[3 * plane + at] = l1;
}

__global__ __launch_bounds__(256) void split_nd_kernel(SplitNd p) {
  const int64_t total = p.rows * p.Kp, plane = total;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / p.Kp, k = idx - r * p.Kp;
    double2 v = make_double2(0.0, 0.0);
    if (k < p.K) v = p.src[digits_off((uint32_t)r, p.nm, p.md, p.ms) + digits_off((uint32_t)k, p.nk, p.kd, p.ks)];
    put_planes(p.dst, plane, idx, v, p.conj);
  }
}

__global__ __launch_bounds__(256) void split_nd_tiled_kernel(SplitNd p) {
  __shared__ double2 tile[32][65];
  const int64_t plane = p.rows * p.Kp;
  const int64_t r0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * 32;
  const int t = threadIdx.x;
  {
    const int rr = t & 63;
    const int64_t r = r0 + rr;
    const int64_t ro = r < p.rows ? digits_off((uint32_t)r, p.nm, p.md, p.ms) : 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = (t >> 6) + 4 * e;
      const int64_t k = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (r < p.rows && k < p.K) v = p.src[ro + digits_off((uint32_t)k, p.nk, p.kd, p.ks)];
      tile[kk][rr] = v;
    }
  }
  __syncthreads();
  {
    const int kk = t & 31;
    const int64_t k = k0 + kk;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int rr = (t >> 5) + 8 * e;
      const int64_t r = r0 + rr;
      if (r < p.rows && k < p.Kp) put_planes(p.dst, plane, r * p.Kp + k, tile[kk][rr], p.conj);
    }
  }
}

void launch_split_nd(const SplitNd& p, int tiled, hipStream_t s) {
  if (p.rows * p.Kp == 0) return;
  if (tiled) {
    dim3 grid((unsigned)((p.rows + 63) / 64), (unsigned)((p.Kp + 31) / 32));
    hipLaunchKernelGGL(split_nd_tiled_kernel, grid, dim3(256), 0, s, p);
  } else {
    hipLaunchKernelGGL(split_nd_kernel, dim3(nblocks(p.rows * p.Kp, 256)), dim3(256), 0, s, p);
  }
}

// WR x WC waves, each computing (16 WM) x (16 WN) of the block tile
template <int WM, int WN, int TAG, int WR = 2, int WC = 2>
__global__ __launch_bounds__(64 * WR * WC) void zgemm_bf16p_kernel(BfGemm p) {
  constexpr int NT = 64 * WR * WC;
  constexpr int BM = 16 * WM * WR, BN = 16 * WN * WC;
  constexpr int UA = 16 * BM / NT, UB = 16 * BN / NT;   // uint4 per thread per slice
  __shared__ __attribute__((aligned(16))) unsigned short sA[4][BM][TKB + PADB];
  __shared__ __attribute__((aligned(16))) unsigned short sB[4][BN][TKB + PADB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN, ntile = tilesM * tilesN;
  const int64_t L = blockIdx.x;
  int64_t tile;
  {
    const int64_t q = ntile / 8, r = ntile % 8, x = L % 8, slot = L / 8;
    tile = x * q + (x < r ? x : r) + slot;
  }
  // column-major walk when B is the larger operand: consecutive tiles of
  // an XCD share a column block of B, which is then fetched once
  const int64_t m0 = (p.colmajor ? tile % tilesM : tile / tilesN) * BM,
                n0 = (p.colmajor ? tile / tilesM : tile % tilesN) * BN;
  const int64_t sidx = blockIdx.y;
  const int64_t kbeg = sidx * p.kchunk;
  const int64_t kend = (kbeg + p.kchunk < p.Kp) ? kbeg + p.kchunk : p.Kp;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t planeA = p.lda * p.Kp, planeB = p.ldb * p.Kp;
  uint4 ra[UA], rb[UB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < UA; ++r) {
      const int e = tid + NT * r;            // (plane, row, quarter)
      const int q = e & 3, rp = e >> 2, pl = rp / BM, row = rp % BM;
      const int64_t gm = m0 + row, gr = p.amd ? (gm / p.amd) * p.ams + gm % p.amd : gm;
      ra[r] = gm < p.M ? *(const uint4*)(p.A + pl * planeA + gr * p.Kp + k0 + 8 * q) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < UB; ++r) {
      const int e = tid + NT * r;
      const int q = e & 3, rp = e >> 2, pl = rp / BN, row = rp % BN;
      const int64_t gn = n0 + row, gr = p.bmd ? (gn / p.bmd) * p.bms + gn % p.bmd : gn;
      rb[r] = gn < p.N ? *(const uint4*)(p.B + pl * planeB + gr * p.Kp + k0 + 8 * q) : make_uint4(0, 0, 0, 0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int r = 0; r < UA; ++r) {
      const int e = tid + NT * r;
      const int q = e & 3, rp = e >> 2, pl = rp / BM, row = rp % BM;
      *(uint4*)&sA[pl][row][8 * q] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < UB; ++r) {
      const int e = tid + NT * r;
      const int q = e & 3, rp = e >> 2, pl = rp / BN, row = rp % BN;
      *(uint4*)&sB[pl][row][8 * q] = rb[r];
    }
  };
  flt4 accR[WM][WN], accI[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      accR[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  if (kbeg < kend) {
    gload(kbeg);
    sstore();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);
  for (int64_t k0 = kbeg; k0 < kend; k0 += TKB) {
    const bool more = k0 + TKB < kend;
    if (more) gload(k0 + TKB);
    us8 b[WN][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = *(const us8*)&sB[q][16 * WN * wc + 16 * j + (lane & 15)][kq];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      us8 a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = *(const us8*)&sA[q][16 * WM * wr + 16 * i + (lane & 15)][kq];
      // negated imaginary planes: flip the sign bit of each bf16 (two per dword)
      us8 nih, nil;
      {
        uint4 u2 = __builtin_bit_cast(uint4, a[2]), u3 = __builtin_bit_cast(uint4, a[3]);
        u2.x ^= 0x80008000u; u2.y ^= 0x80008000u; u2.z ^= 0x80008000u; u2.w ^= 0x80008000u;
        u3.x ^= 0x80008000u; u3.y ^= 0x80008000u; u3.z ^= 0x80008000u; u3.w ^= 0x80008000u;
        nih = __builtin_bit_cast(us8, u2);
        nil = __builtin_bit_cast(us8, u3);
      }
      // the six split products of Re and of Im, issued term by term across the
      // 2*WN independent accumulators of this row block so that consecutive
      // MFMAs never depend on each other
      const us8* ra[6] = {&a[0], &a[0], &a[1], &nih, &nih, &nil};
      const int rbq[6] = {0, 1, 0, 2, 3, 2};
      const us8* ia[6] = {&a[0], &a[0], &a[1], &a[2], &a[2], &a[3]};
      const int ibq[6] = {2, 3, 2, 0, 1, 0};
#pragma unroll
      for (int tm = 0; tm < 6; ++tm) {
#pragma unroll
        for (int j = 0; j < WN; ++j) accR[i][j] = mfma_bf16(*ra[tm], b[j][rbq[tm]], accR[i][j]);
#pragma unroll
        for (int j = 0; j < WN; ++j) accI[i][j] = mfma_bf16(*ia[tm], b[j][ibq[tm]], accI[i][j]);
      }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }
  {
    int64_t rows[WM][4], cols[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[i][r] = m0 + 16 * WM * wr + 16 * i + 4 * (lane >> 4) + r;
#pragma unroll
    for (int j = 0; j < WN; ++j) cols[j] = n0 + 16 * WN * wc + 16 * j + (lane & 15);
    double2* P = p.nsplit > 1 ? p.P + sidx * p.M * p.N : nullptr;
    store_tile<WM, WN>(p.M, p.N, p.C, P, p.om, p.scm, p.scn, p.alpha, p.beta, rows, cols, accR, accI, p.c32);
  }
}

// ---------------------------------------------------------------------------
// The same product with the operand tiles streamed straight from global memory
// into LDS (global_load_lds_dwordx4: each lane's 16 bytes land at the wave's
// LDS base + 16 * lane, no VGPR staging, no ds_write) and two LDS stages, so
// that the loads of slice s+1 fly while slice s is multiplied and one barrier
// per slice suffices.  A plane of a tile is [rows][32 bf16] (64 bytes per
// row, no padding); the four 16-byte quarters of row R are stored XOR-
// permuted by swz(R), which keeps the fragment reads (16 rows x one quarter
// per instruction) free of bank conflicts for both 32 and 64 banks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// GRP: a grouped GEMM (BfGemm.probs); each workgroup takes the problem whose
// tile range holds its tile and runs it with that problem's shape, operand
// rows and output (a separate instantiation, so that the plain kernels keep
// their code)
template <int WM, int WN, int TAG, int WR, int WC, bool GRP = false>
__global__ __launch_bounds__(64 * WR * WC) void zgemm_bf16d_kernel(BfGemm p) {
  constexpr int NW = WR * WC;
  constexpr int BM = 16 * WM * WR, BN = 16 * WN * WC;
  constexpr int CA = 4 * BM / 16, CB = 4 * BN / 16;   // 1 KB chunks (16 rows of one plane) per stage
  constexpr int NCH = CA + CB, PER = NCH / NW;
  static_assert(NCH % NW == 0, "chunks must divide among the waves");
  constexpr int STAGE = NCH * 1024;                    // bytes
  __shared__ __attribute__((aligned(1024))) unsigned char smem[2 * STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int64_t tilesM = (p.M + BM - 1) / BM, tilesN = (p.N + BN - 1) / BN;
  const int64_t ntile = GRP ? p.gtiles : tilesM * tilesN;
  const int64_t L = blockIdx.x;
  int64_t tile;
  {
    const int64_t q = ntile / 8, r = ntile % 8, x = L % 8, slot = L / 8;
    tile = x * q + (x < r ? x : r) + slot;
  }
  int64_t M = p.M, N = p.N, amd = p.amd, bmd = p.bmd, scm = p.scm;
  const unsigned short* Ap = p.A;
  const unsigned short* Bp = p.B;
  double2* Cp = p.C;
  int colmajor = p.colmajor;
  if constexpr (GRP) {
    int lo = 0, hi = p.nprob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (p.probs[mid].tile0 <= tile) lo = mid;
      else hi = mid - 1;
    }
    const GroupProb& g = p.probs[lo];
    tile -= g.tile0;
    M = g.M;
    N = g.N;
    Ap += g.arow * p.Kp;
    Bp += g.brow * p.Kp;
    amd = g.amd;
    bmd = g.bmd;
    Cp = p.c32 ? (double2*)((float2*)p.C + g.coff) : p.C + g.coff;
    scm = g.ldc;
    colmajor = N > M ? 1 : 0;
    tilesM = (M + BM - 1) / BM;
    tilesN = (N + BN - 1) / BN;
  }
  // column-major walk when B is the larger operand: consecutive tiles of
  // an XCD share a column block of B, which is then fetched once
  const int64_t m0 = (colmajor ? tile % tilesM : tile / tilesN) * BM,
                n0 = (colmajor ? tile / tilesM : tile % tilesN) * BN;
  const int64_t sidx = blockIdx.y;
  const int64_t kbeg = sidx * p.kchunk;
  const int64_t kend = (kbeg + p.kchunk < p.Kp) ? kbeg + p.kchunk : p.Kp;
  const int wr = wave / WC, wc = wave % WC;
  // source of this lane's 16 bytes in each of the wave's chunks (k offset 0);
  // rows past the matrix edge re-read the last row: they only feed output
  // rows/columns that are never stored
  const unsigned short* src[PER];
  int ldsoff[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int c = wave + NW * j;
    const int rin = lane >> 2, slot = lane & 3;
    if (c < CA) {
      const int pl = c / (BM / 16), R = 16 * (c % (BM / 16)) + rin;
      int64_t gm = (m0 + R < M) ? m0 + R : M - 1;
      if (amd) gm = (gm / amd) * p.ams + gm % amd;
      src[j] = Ap + pl * p.lda * p.Kp + gm * p.Kp + 8 * (slot ^ swz(R));
    } else {
      const int cb = c - CA;
      const int pl = cb / (BN / 16), R = 16 * (cb % (BN / 16)) + rin;
      int64_t gn = (n0 + R < N) ? n0 + R : N - 1;
      if (bmd) gn = (gn / bmd) * p.bms + gn % bmd;
      src[j] = Bp + pl * p.ldb * p.Kp + gn * p.Kp + 8 * (slot ^ swz(R));
    }
    ldsoff[j] = c * 1024;
  }
  auto issue = [&](int64_t k0, int stage) {
#pragma unroll
    for (int j = 0; j < PER; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(src[j] + k0),
                                       (__attribute__((address_space(3))) void*)(smem + stage * STAGE + ldsoff[j]),
                                       16, 0, 0);
  };
  flt4 accR[WM][WN], accI[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      accR[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  const int kq = lane >> 4, r16 = lane & 15;
  // byte offsets of this lane's fragment rows inside a plane of the A / B tile
  int offA[WM], offB[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int R = 16 * WM * wr + 16 * i + r16;
    offA[i] = R * 64 + 16 * (kq ^ swz(R));
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int R = 16 * WN * wc + 16 * j + r16;
    offB[j] = CA * 1024 + R * 64 + 16 * (kq ^ swz(R));
  }
  if (kbeg < kend) issue(kbeg, 0);
  int stage = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += TKB) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (k0 + TKB < kend) issue(k0 + TKB, stage ^ 1);
    const unsigned char* sb = smem + stage * STAGE;
    us8 b[WN][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = *(const us8*)(sb + offB[j] + q * (BN / 16) * 1024);
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      us8 a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = *(const us8*)(sb + offA[i] + q * (BM / 16) * 1024);
      us8 nih, nil;
      {
        uint4 u2 = __builtin_bit_cast(uint4, a[2]), u3 = __builtin_bit_cast(uint4, a[3]);
        u2.x ^= 0x80008000u; u2.y ^= 0x80008000u; u2.z ^= 0x80008000u; u2.w ^= 0x80008000u;
        u3.x ^= 0x80008000u; u3.y ^= 0x80008000u; u3.z ^= 0x80008000u; u3.w ^= 0x80008000u;
        nih = __builtin_bit_cast(us8, u2);
        nil = __builtin_bit_cast(us8, u3);
      }
      const us8* ra[6] = {&a[0], &a[0], &a[1], &nih, &nih, &nil};
      const int rbq[6] = {0, 1, 0, 2, 3, 2};
      const us8* ia[6] = {&a[0], &a[0], &a[1], &a[2], &a[2], &a[3]};
      const int ibq[6] = {2, 3, 2, 0, 1, 0};
#pragma unroll
      for (int tm = 0; tm < 6; ++tm) {
#pragma unroll
        for (int j = 0; j < WN; ++j) accR[i][j] = mfma_bf16(*ra[tm], b[j][rbq[tm]], accR[i][j]);
#pragma unroll
        for (int j = 0; j < WN; ++j) accI[i][j] = mfma_bf16(*ia[tm], b[j][ibq[tm]], accI[i][j]);
      }
    }
    stage ^= 1;
  }
  {
    int64_t rows[WM][4], cols[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[i][r] = m0 + 16 * WM * wr + 16 * i + 4 * (lane >> 4) + r;
#pragma unroll
    for (int j = 0; j < WN; ++j) cols[j] = n0 + 16 * WN * wc + 16 * j + (lane & 15);
    double2* P = p.nsplit > 1 ? p.P + sidx * M * N : nullptr;
    store_tile<WM, WN>(M, N, Cp, P, p.om, scm, GRP ? 1 : p.scn, p.alpha, p.beta, rows, cols, accR, accI, p.c32);
  }
}

template <int WM, int WN, int WR, int WC>
static void launch_bf16d_tile(const BfGemm& h, hipStream_t s) {
  constexpr int BM = 16 * WM * WR, BN = 16 * WN * WC, NT = 64 * WR * WC;
  const int64_t tiles = h.nprob > 0 ? h.gtiles : ((h.M + BM - 1) / BM) * ((h.N + BN - 1) / BN);
  dim3 grid((unsigned)tiles, (unsigned)h.nsplit);
  if (h.nprob > 0)
    hipLaunchKernelGGL((zgemm_bf16d_kernel<WM, WN, 1, WR, WC, true>), dim3((unsigned)tiles), dim3(NT), 0, s, h);
  else if (h.tag == 1) hipLaunchKernelGGL((zgemm_bf16d_kernel<WM, WN, 1, WR, WC>), grid, dim3(NT), 0, s, h);
  else if (h.tag == 2) hipLaunchKernelGGL((zgemm_bf16d_kernel<WM, WN, 2, WR, WC>), grid, dim3(NT), 0, s, h);
  else hipLaunchKernelGGL((zgemm_bf16d_kernel<WM, WN, 0, WR, WC>), grid, dim3(NT), 0, s, h);
}

template <int WM, int WN, int WR = 2, int WC = 2>
static void launch_bf16p_tile(const BfGemm& h, hipStream_t s) {
  constexpr int BM = 16 * WM * WR, BN = 16 * WN * WC, NT = 64 * WR * WC;
  const int64_t tiles = ((h.M + BM - 1) / BM) * ((h.N + BN - 1) / BN);
  dim3 grid((unsigned)tiles, (unsigned)h.nsplit);
  if (h.tag == 1) hipLaunchKernelGGL((zgemm_bf16p_kernel<WM, WN, 1, WR, WC>), grid, dim3(NT), 0, s, h);
  else if (h.tag == 2) hipLaunchKernelGGL((zgemm_bf16p_kernel<WM, WN, 2, WR, WC>), grid, dim3(NT), 0, s, h);
  else hipLaunchKernelGGL((zgemm_bf16p_kernel<WM, WN, 0, WR, WC>), grid, dim3(NT), 0, s, h);
}

int bf16p_pick_tile(const BfGemm& h) {
  // the candidate with the least padded work divided by the fraction of
  // peak it sustains on large random operands, times the wave quantisation
  // of its grid over the workgroups the chip holds at once; a tile is only
  // taken when its grid keeps at least half of those slots busy
  struct Cand { int tile, bm, bn; double rate; int64_t slots; };
  const Cand cand[4] = {{9, 128, 128, 0.41, 256}, {13, 64, 256, 0.35, 256}, {2, 128, 64, 0.35, 512},
                        {0, 64, 64, 0.31, 1024}};
  const int64_t nsplit = h.nsplit < 1 ? 1 : h.nsplit;
  int tile = 0;
  double best = -1.0;
  for (const Cand& c : cand) {
    const int64_t tm = (h.M + c.bm - 1) / c.bm, tn = (h.N + c.bn - 1) / c.bn, nwg = tm * tn * nsplit;
    if (c.tile != 0 && 2 * nwg < c.slots) continue;
    const double waves = (double)((nwg + c.slots - 1) / c.slots) * (double)c.slots / (double)nwg;
    const double cost = (double)(tm * c.bm) * (double)(tn * c.bn) / c.rate * waves;
    if (best < 0.0 || cost < best) { tile = c.tile; best = cost; }
  }
  return tile;
}

// tile: 0 = 64x64, 1 = 128x128, 2 = 128x64, 3 = 64x128 (rows x cols of C,
// four waves), 4 = 128x128 and 5 = 128x64 with eight waves, 6-13 the direct-
// load kernels (zgemm_bf16d_kernel); negative = bf16p_pick_tile
void launch_bf16p(const BfGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.Kp <= 0) return;
  BfGemm h = g;
  if (h.nsplit < 1 || h.kchunk <= 0) { h.nsplit = 1; h.kchunk = h.Kp; }
  h.colmajor = h.N > h.M ? 1 : 0;
  const int tile = h.tile < 0 ? bf16p_pick_tile(h) : h.tile;
  switch (tile) {
    case 1: launch_bf16p_tile<4, 4>(h, s); break;
    case 2: launch_bf16p_tile<4, 2>(h, s); break;
    case 3: launch_bf16p_tile<2, 4>(h, s); break;
    case 4: launch_bf16p_tile<4, 2, 2, 4>(h, s); break;  // 128 x 128, 8 waves
    case 5: launch_bf16p_tile<2, 2, 4, 2>(h, s); break;  // 128 x 64, 8 waves
    case 6: launch_bf16d_tile<4, 2, 2, 4>(h, s); break;  // 128 x 128, 8 waves, direct LDS loads
    case 7: launch_bf16d_tile<4, 2, 2, 2>(h, s); break;  // 128 x 64, 4 waves, direct LDS loads
    case 8: launch_bf16d_tile<4, 4, 2, 2>(h, s); break;  // 128 x 128, 4 waves, direct LDS loads
    case 9: launch_bf16d_tile<2, 2, 4, 4>(h, s); break;  // 128 x 128, 16 waves, direct LDS loads
    case 10: launch_bf16d_tile<2, 2, 2, 2>(h, s); break;  // 64 x 64, 4 waves, direct LDS loads
    case 11: launch_bf16d_tile<2, 2, 4, 2>(h, s); break;  // 128 x 64, 8 waves, direct LDS loads
    case 12: launch_bf16d_tile<2, 2, 2, 4>(h, s); break;  // 64 x 128, 8 waves, direct LDS loads
    case 13: launch_bf16d_tile<2, 2, 2, 8>(h, s); break;  // 64 x 256, 16 waves, direct LDS loads
    default: launch_bf16p_tile<2, 2>(h, s); break;
  }
}

void launch_splitk_reduce_bf(const BfGemm& g, hipStream_t s) {
  ReduceArgs a{g.P, g.M * g.N, g.M * g.N, g.N, g.nsplit, g.C, 0, g.scm, g.scn, g.om, g.alpha, g.beta, g.c32};
  launch_reduce(a, s);
}

// packed <ab||cd> rows written directly as split planes [4][ldv][Kp], at rows
// r0 .. r0 + npairs of each plane
__global__ __launch_bounds__(256) void ladder_pack_planes_kernel(const double2* W, int64_t ldw, int a0, int b0, int nv,
                                                                 unsigned short* V, int64_t ldv, int64_t r0,
                                                                 int64_t pbase, const int2* pv, int64_t Pv,
                                                                 int64_t Kp) {
  const int64_t pr = blockIdx.y;
  const int2 ab = pv[pbase + pr];
  const int64_t ra = (int64_t)(ab.x - a0) * nv, cb = (int64_t)(ab.y - b0) * nv;
  const int64_t plane = ldv * Kp;
  for (int64_t pc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < Kp; pc += (int64_t)gridDim.x * blockDim.x) {
    unsigned short h0 = 0, l0 = 0, h1 = 0, l1 = 0;
    if (pc < Pv) {
      const int2 cd = pv[pc];
      const double2 w1 = W[(ra + cd.x) * ldw + cb + cd.y];
      const double2 w2 = W[(ra + cd.y) * ldw + cb + cd.x];
      split_bf16((float)(w1.x - w2.x), h0, l0);
      split_bf16((float)(w1.y - w2.y), h1, l1);
    }
    const int64_t o = (r0 + pr) * Kp + pc;
    V[o] = h0;
    V[plane + o] = l0;
    V[2 * plane + o] = h1;
    V[3 * plane + o] = l1;
  }
}
void launch_ladder_pack_planes(const double2* W, int64_t ldw, int a0, int b0, int nv, unsigned short* V, int64_t ldv,
                               int64_t r0, int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp, hipStream_t s) {
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  if (npairs <= 0 || Pv <= 0) return;
  unsigned gx = (unsigned)((Kp + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(ladder_pack_planes_kernel, dim3(gx, (unsigned)npairs), dim3(256), 0, s, W, ldw, a0, b0, nv, V,
                     ldv, r0, pbase, pv, Pv, Kp);
}

template <typename WT>
__global__ __launch_bounds__(256) void ladder_pack_planes_upper_kernel(const WT* W, int64_t ldw, int a0, int b0,
                                                                       int nv, unsigned short* V, int64_t ldv,
                                                                       int64_t pbase, const int2* pv, int64_t Pv,
                                                                       int64_t Kp, int64_t vrow0) {
  const int64_t pr = blockIdx.y, prow = pbase + pr;
  const int2 ab = pv[prow];
  const int64_t m = nv - a0;
  const int64_t ra = (int64_t)(ab.x - a0) * m, cb = (int64_t)(ab.y - b0) * m;
  const int64_t plane = ldv * Kp;
  // columns pc < prow are the lower part, which the mirror writes
  for (int64_t pc = prow + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < Kp;
       pc += (int64_t)gridDim.x * blockDim.x) {
    unsigned short h0 = 0, l0 = 0, h1 = 0, l1 = 0;
    if (pc < Pv) {
      const int2 cd = pv[pc];  // c >= a >= a0 and d > c
      const WT w1 = W[(ra + cd.x - a0) * ldw + cb + cd.y - a0];
      const WT w2 = W[(ra + cd.y - a0) * ldw + cb + cd.x - a0];
      split_bf16((float)(w1.x - w2.x), h0, l0);
      split_bf16((float)(w1.y - w2.y), h1, l1);
    }
    const int64_t o = (prow - vrow0) * Kp + pc;
    V[o] = h0;
    V[plane + o] = l0;
    V[2 * plane + o] = h1;
    V[3 * plane + o] = l1;
  }
}
// one block row per pair (a, b) of pbase + blockIdx.y, its block found from a
__global__ __launch_bounds__(256) void ladder_pack_planes_grouped_kernel(const float2* Wall, const LadBlk* blk, int nv,
                                                                         unsigned short* V, int64_t ldv,
                                                                         int64_t pbase, const int2* pv, int64_t Pv,
                                                                         int64_t Kp) {
  const int64_t prow = pbase + blockIdx.y;
  const int2 ab = pv[prow];
  const LadBlk B = blk[ab.x];
  const float2* W = Wall + B.woff;
  const int64_t a0 = B.a0, ldw = B.ldw;
  const int64_t m = nv - a0;
  const int64_t ra = (int64_t)(ab.x - a0) * m, cb = (int64_t)(ab.y - a0 - 1) * m;
  const int64_t plane = ldv * Kp;
  for (int64_t pc = prow + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < Kp;
       pc += (int64_t)gridDim.x * blockDim.x) {
    unsigned short h0 = 0, l0 = 0, h1 = 0, l1 = 0;
    if (pc < Pv) {
      const int2 cd = pv[pc];  // c >= a >= a0 and d > c
      const float2 w1 = W[(ra + cd.x - a0) * ldw + cb + cd.y - a0];
      const float2 w2 = W[(ra + cd.y - a0) * ldw + cb + cd.x - a0];
      split_bf16(w1.x - w2.x, h0, l0);
      split_bf16(w1.y - w2.y, h1, l1);
    }
    const int64_t o = prow * Kp + pc;
    V[o] = h0;
    V[plane + o] = l0;
    V[2 * plane + o] = h1;
    V[3 * plane + o] = l1;
  }
}
void launch_ladder_pack_planes_grouped(const void* Wall, const LadBlk* blk, int nv, unsigned short* V, int64_t ldv,
                                       int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp, hipStream_t s) {
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  if (npairs <= 0 || Pv <= 0) return;
  unsigned gx = (unsigned)((Kp + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(ladder_pack_planes_grouped_kernel, dim3(gx, (unsigned)npairs), dim3(256), 0, s,
                     (const float2*)Wall, blk, nv, V, ldv, pbase, pv, Pv, Kp);
}

void launch_ladder_pack_planes_upper(const void* W, int w32, int64_t ldw, int a0, int b0, int nv, unsigned short* V,
                                     int64_t ldv, int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp,
                                     hipStream_t s, int64_t vrow0) {
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  if (npairs <= 0 || Pv <= 0) return;
  unsigned gx = (unsigned)((Kp + 255) / 256);
  if (gx > 64) gx = 64;
  if (w32)
    hipLaunchKernelGGL(ladder_pack_planes_upper_kernel<float2>, dim3(gx, (unsigned)npairs), dim3(256), 0, s,
                       (const float2*)W, ldw, a0, b0, nv, V, ldv, pbase, pv, Pv, Kp, vrow0);
  else
    hipLaunchKernelGGL(ladder_pack_planes_upper_kernel<double2>, dim3(gx, (unsigned)npairs), dim3(256), 0, s,
                       (const double2*)W, ldw, a0, b0, nv, V, ldv, pbase, pv, Pv, Kp, vrow0);
}
// V[pl][r][0:c1] = 0 for r < rows (planes [4][ldv][Kp])
__global__ __launch_bounds__(256) void planes_zero_cols_kernel(unsigned short* V, int64_t ldv, int64_t rows,
                                                               int64_t c1, int64_t Kp) {
  const int64_t total = 4 * rows * c1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pl = e / (rows * c1), rem = e - pl * rows * c1, r = rem / c1, c = rem - r * c1;
    V[pl * ldv * Kp + r * Kp + c] = 0;
  }
}
void launch_planes_zero_cols(unsigned short* V, int64_t ldv, int64_t rows, int64_t c1, int64_t Kp, hipStream_t s) {
  const int64_t total = 4 * rows * c1;
  if (total <= 0) return;
  hipLaunchKernelGGL(planes_zero_cols_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65535 * 16)),
                     dim3(256), 0, s, V, ldv, rows, c1, Kp);
}

// Lower part of the diagonal block of a row group: local row r holds pair
// col0 + r, so V[pl][r][col0 + c] = conj V[pl][c][col0 + r] for c < r < n
// (the imaginary planes change sign).  64 x 64 tiles of the lower triangle
// through LDS, one bf16 per access.
__global__ __launch_bounds__(256) void ladder_mirror_block_kernel(unsigned short* V, int64_t ldv, int64_t n,
                                                                  int64_t Kp, int64_t col0) {
  __shared__ unsigned short t[64][65];
  const int64_t L = blockIdx.x;
  int64_t tp = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
  while ((tp + 1) * (tp + 2) / 2 <= L) ++tp;
  while (tp * (tp + 1) / 2 > L) --tp;
  const int64_t tq = L - tp * (tp + 1) / 2;
  const int64_t p0 = tp * 64, q0 = tq * 64;  // rows p0 .. take columns col0 + q0 ..
  const int64_t plane = ldv * Kp;
  const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int pl = 0; pl < 4; ++pl) {
    const unsigned short flip = pl >= 2 ? 0x8000 : 0;
    unsigned short* Vp = V + pl * plane;
    // the upper part: rows q0 + r, columns col0 + p0 + c
    for (int r = ty; r < 64; r += 4) {
      const int64_t q = q0 + r, p = p0 + c;
      t[r][c] = (q < n && p < n && q < p) ? Vp[q * Kp + col0 + p] : (unsigned short)0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
      const int64_t p = p0 + r, q = q0 + c;
      if (p < n && q < p) {
        const unsigned short w = t[c][r];
        Vp[p * Kp + col0 + q] = (w & 0x7fff) ? (unsigned short)(w ^ flip) : w;
      }
    }
    __syncthreads();
  }
}
void launch_ladder_mirror_block(unsigned short* V, int64_t ldv, int64_t n, int64_t Kp, int64_t col0, hipStream_t s) {
  if (n <= 1) return;
  const int64_t nt = (n + 63) / 64;
  hipLaunchKernelGGL(ladder_mirror_block_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, V, ldv, n, Kp,
                     col0);
}

// T[pl][q][koff + r] = conj V[pl][r][c0 + q] for r < rows, q < ncols (planes
// of V: [4][ldv][Kp]; of T: [4][ncols][Kt]), zero in T's other columns;
// 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void ladder_transpose_planes_kernel(const unsigned short* V, int64_t ldv,
                                                                      int64_t rows, int64_t c0, int64_t ncols,
                                                                      int64_t Kp, unsigned short* T, int64_t Kt,
                                                                      int64_t koff) {
  __shared__ unsigned short t[64][65];
  const int64_t q0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * 64;  // rows, columns of T
  const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int pl = 0; pl < 4; ++pl) {
    const unsigned short flip = pl >= 2 ? 0x8000 : 0;
    for (int e = ty; e < 64; e += 4) {
      const int64_t r = k0 + e - koff, q = q0 + c;
      unsigned short w = 0;
      if (r >= 0 && r < rows && q < ncols) {
        w = V[pl * ldv * Kp + r * Kp + c0 + q];
        if (w & 0x7fff) w ^= flip;
      }
      t[e][c] = w;
    }
    __syncthreads();
    for (int e = ty; e < 64; e += 4) {
      const int64_t q = q0 + e, kk = k0 + c;
      if (q < ncols && kk < Kt) T[pl * ncols * Kt + q * Kt + kk] = t[c][e];
    }
    __syncthreads();
  }
}
void launch_ladder_transpose_planes(const unsigned short* V, int64_t ldv, int64_t rows, int64_t c0, int64_t ncols,
                                    int64_t Kp, unsigned short* T, int64_t Kt, int64_t koff, hipStream_t s) {
  if (ncols <= 0 || Kt <= 0) return;
  hipLaunchKernelGGL(ladder_transpose_planes_kernel, dim3((unsigned)((ncols + 63) / 64), (unsigned)((Kt + 63) / 64)),
                     dim3(256), 0, s, V, ldv, rows, c0, ncols, Kp, T, Kt, koff);
}

// dst[pl][r][kk] = src[pl][r][c0 + kk] for kk < Kt (planes [4][rows][Kp] and
// [4][rows][Kt])
__global__ __launch_bounds__(256) void planes_copy_cols_kernel(const unsigned short* src, int64_t rows, int64_t Kp,
                                                               int64_t c0, unsigned short* dst, int64_t Kt) {
  const int64_t total = 4 * rows * Kt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pr = e / Kt, kk = e - pr * Kt;  // pr = plane * rows + r
    dst[e] = src[pr * Kp + c0 + kk];
  }
}
void launch_planes_copy_cols(const unsigned short* src, int64_t rows, int64_t Kp, int64_t c0, unsigned short* dst,
                             int64_t Kt, hipStream_t s) {
  const int64_t total = 4 * rows * Kt;
  if (total <= 0) return;
  hipLaunchKernelGGL(planes_copy_cols_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65535 * 16)),
                     dim3(256), 0, s, src, rows, Kp, c0, dst, Kt);
}


// 64 x 64 tiles (tp >= tq) of the strictly lower triangle: read block (q, p)
// of the upper part through LDS, write its conjugate transpose at (p, q);
// global accesses are pairs of bf16 (4 bytes), except where a pair straddles
// the diagonal
__global__ __launch_bounds__(256) void ladder_mirror_planes_kernel(unsigned short* V, int64_t ldv, int64_t n,
                                                                   int64_t Kp) {
  __shared__ unsigned short t[64][66];
  // blockIdx.x enumerates the lower-triangle tiles (tp, tq), tq <= tp
  const int64_t L = blockIdx.x;
  int64_t tp = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
  while ((tp + 1) * (tp + 2) / 2 <= L) ++tp;
  while (tp * (tp + 1) / 2 > L) --tp;
  const int64_t tq = L - tp * (tp + 1) / 2;
  const int64_t p0 = tp * 64, q0 = tq * 64;
  const int64_t plane = ldv * Kp;
  const int c = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int pl = 0; pl < 4; ++pl) {
    const unsigned flip = pl >= 2 ? 0x80008000u : 0u;
    unsigned short* Vp = V + pl * plane;
    // rows q0 + r of the upper part, columns p0 + 2c, p0 + 2c + 1
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = ty + 8 * e;
      const int64_t q = q0 + r, p = p0 + 2 * c;
      unsigned w = 0;
      if (q < n && p < n) {
        // Kp and p are even: the pair is 4-byte aligned and inside the row
        w = *(const unsigned*)(Vp + q * Kp + p);
        if (!(q < p)) w &= 0xffff0000u;
        if (!(q < p + 1) || p + 1 >= n) w &= 0x0000ffffu;
      }
      t[r][2 * c] = (unsigned short)(w & 0xffffu);
      t[r][2 * c + 1] = (unsigned short)(w >> 16);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = ty + 8 * e;
      const int64_t p = p0 + r, q = q0 + 2 * c;
      if (p >= n) continue;
      const unsigned w = ((unsigned)t[2 * c][r] | ((unsigned)t[2 * c + 1][r] << 16)) ^ flip;
      if (q + 1 < p) {
        *(unsigned*)(Vp + p * Kp + q) = w;
      } else if (q < p) {
        Vp[p * Kp + q] = (unsigned short)(w & 0xffffu);
      }
    }
    __syncthreads();
  }
}
void launch_ladder_mirror_planes(unsigned short* V, int64_t ldv, int64_t n, int64_t Kp, hipStream_t s) {
  if (n <= 1) return;
  const int64_t nt = (n + 63) / 64;
  hipLaunchKernelGGL(ladder_mirror_planes_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, V, ldv, n, Kp);
}

template <typename T, int WM, int WN>
static void launch_tile(const GemmDesc& g, hipStream_t s) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid((unsigned)tiles, (unsigned)(g.batch * g.nsplit));
  if (g.tag == 1) hipLaunchKernelGGL((zgemm_kernel<T, WM, WN, 1>), grid, dim3(256), 0, s, g);
  else if (g.tag == 2) hipLaunchKernelGGL((zgemm_kernel<T, WM, WN, 2>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((zgemm_kernel<T, WM, WN, 0>), grid, dim3(256), 0, s, g);
}

// Tile choice: 64x64 by default.  With the accumulators in VGPRs it runs two
// (FP64) or three (FP32) waves per SIMD and measures faster than the larger
// tiles (FP64 128x64, FP32 128x128 / 128x64), which stay selectable (tile 1, 2).
// FP64 tiles 3 (128x32) and 4 (64x32) are for outputs only a few columns
// wide (Gram blocks of a subspace against a few new vectors).
void launch_zgemm(const GemmDesc& g0, int prec, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0 || g0.K <= 0) return;
  GemmDesc g = g0;
  if (g.nsplit < 1) g.nsplit = 1;
  if (g.nsplit == 1 || g.kchunk <= 0) { g.nsplit = 1; g.kchunk = g.K; }
  const bool use_big = g.tile == 1;
  if (prec == 2) {
    launch_bf16x3(g, s);
  } else if (prec == 0) {
    if (use_big) launch_tile<double, 4, 2>(g, s);
    else if (g.tile == 3) launch_tile<double, 4, 1>(g, s);
    else if (g.tile == 4) launch_tile<double, 2, 1>(g, s);
    else launch_tile<double, 2, 2>(g, s);
  } else {
    if (g.tile == 2) launch_tile<float, 4, 2>(g, s);
    else if (use_big) launch_tile<float, 4, 4>(g, s);
    else launch_tile<float, 2, 2>(g, s);
  }
}

// ---------------------------------------------------------------------------
// generic permute / axpby into a contiguous output
// ---------------------------------------------------------------------------
struct PermArgs {
  int nd;
  int64_t od[8];
  int64_t is[8];
  int64_t os[8];
  const double2* in;
  double2* out;
  int64_t total;
  cplx alpha, beta;
  int conj;
};

template <bool SMALL>
__global__ __launch_bounds__(256) void permute_kernel(PermArgs p) {
  const bool has_beta = (p.beta.re != 0.0 || p.beta.im != 0.0);
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < p.total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t off = 0, ooff = 0;
    if (SMALL) {  // 32-bit index arithmetic (total < 2^32)
      uint32_t rem = (uint32_t)idx;
      for (int d = p.nd - 1; d >= 0; --d) {
        const uint32_t dd = (uint32_t)p.od[d], q = rem / dd, r = rem - q * dd;
        off += (int64_t)r * p.is[d];
        ooff += (int64_t)r * p.os[d];
        rem = q;
      }
    } else {
      int64_t rem = idx;
      for (int d = p.nd - 1; d >= 0; --d) {
        const int64_t q = rem / p.od[d];
        const int64_t r = rem - q * p.od[d];
        off += r * p.is[d];
        ooff += r * p.os[d];
        rem = q;
      }
    }
    double2 v = p.in[off];
    if (p.conj) v.y = -v.y;
    double2 o;
    o.x = p.alpha.re * v.x - p.alpha.im * v.y;
    o.y = p.alpha.re * v.y + p.alpha.im * v.x;
    if (has_beta) {
      const double2 old = p.out[ooff];
      o.x += p.beta.re * old.x - p.beta.im * old.y;
      o.y += p.beta.re * old.y + p.beta.im * old.x;
    }
    p.out[ooff] = o;
  }
}

// Transposing permute: dims di (unit input stride) and dO (unit output stride)
// differ; 32 x 32 tiles of (di, dO) go through LDS so that both the reads and
// the writes are coalesced.  The other dims (mixed radix, 32-bit) index the
// tiles together with the tile position: blockIdx.x = rest * tiles + tile.
struct PermTiled {
  PermArgs a;
  int di, dO;
  int64_t tdi, tdo, ntile, nrest;
};
__global__ __launch_bounds__(256) void permute_tiled_kernel(PermTiled q) {
  __shared__ double2 tile[32][33];
  const PermArgs& p = q.a;
  const bool has_beta = (p.beta.re != 0.0 || p.beta.im != 0.0);
  for (int64_t blk = blockIdx.x; blk < q.ntile * q.nrest; blk += gridDim.x) {
    const int64_t rest = blk / q.ntile, tl = blk - rest * q.ntile;
    const int64_t i0 = (tl / q.tdo) * 32, o0 = (tl % q.tdo) * 32;
    int64_t ioff = 0, ooff = 0;
    {
      uint32_t rem = (uint32_t)rest;
      for (int d = p.nd - 1; d >= 0; --d) {
        if (d == q.di || d == q.dO) continue;
        const uint32_t dd = (uint32_t)p.od[d], qq = rem / dd, r = rem - qq * dd;
        ioff += (int64_t)r * p.is[d];
        ooff += (int64_t)r * p.os[d];
        rem = qq;
      }
    }
    const int64_t ni = p.od[q.di], no = p.od[q.dO];
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = t & 31, b = (t >> 5) + 8 * e;  // a along di, b along dO
      const int64_t ia = i0 + a, ob = o0 + b;
      double2 v = make_double2(0.0, 0.0);
      if (ia < ni && ob < no) v = p.in[ioff + ia + ob * p.is[q.dO]];
      tile[b][a] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int b = t & 31, a = (t >> 5) + 8 * e;
      const int64_t ia = i0 + a, ob = o0 + b;
      if (ia < ni && ob < no) {
        double2 v = tile[b][a];
        if (p.conj) v.y = -v.y;
        double2 o;
        o.x = p.alpha.re * v.x - p.alpha.im * v.y;
        o.y = p.alpha.re * v.y + p.alpha.im * v.x;
        double2* dst = p.out + ooff + ia * p.os[q.di] + ob;
        if (has_beta) {
          const double2 old = *dst;
          o.x += p.beta.re * old.x - p.beta.im * old.y;
          o.y += p.beta.re * old.y + p.beta.im * old.x;
        }
        *dst = o;
      }
    }
    __syncthreads();
  }
}

void launch_permute(int nd, const int64_t* od, const int64_t* istr, const int64_t* ostr, const double2* in,
                    double2* out, cplx alpha, cplx beta, int conj, hipStream_t s) {
  PermArgs a;
  a.nd = nd;
  a.total = 1;
  for (int d = 0; d < nd; ++d) {
    a.od[d] = od[d];
    a.is[d] = istr[d];
    a.os[d] = ostr[d];
    a.total *= od[d];
  }
  if (a.total == 0) return;
  a.in = in;
  a.out = out;
  a.alpha = alpha;
  a.beta = beta;
  a.conj = conj;
  int di = -1, dO = -1;
  for (int d = 0; d < nd; ++d) {
    if (istr[d] == 1 && di < 0) di = d;
    if (ostr[d] == 1 && dO < 0) dO = d;
  }
  if (di >= 0 && dO >= 0 && di != dO && od[di] >= 8 && od[dO] >= 8 && a.total < ((int64_t)1 << 32)) {
    PermTiled q;
    q.a = a;
    q.di = di;
    q.dO = dO;
    q.tdi = (od[di] + 31) / 32;
    q.tdo = (od[dO] + 31) / 32;
    q.ntile = q.tdi * q.tdo;
    q.nrest = a.total / (od[di] * od[dO]);
    const int64_t blocks = std::min<int64_t>(q.ntile * q.nrest, (int64_t)1 << 20);
    hipLaunchKernelGGL(permute_tiled_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q);
    return;
  }
  if (a.total < ((int64_t)1 << 32))
    hipLaunchKernelGGL(permute_kernel<true>, dim3(nblocks(a.total, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(permute_kernel<false>, dim3(nblocks(a.total, 256)), dim3(256), 0, s, a);
}

__global__ void add_diag_kernel(double2* M, const double* d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    M[i * n + i].x += d[i];
}
void launch_add_diag(double2* M, const double* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(add_diag_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, M, d, n);
}

__global__ void resid_kernel(const double2* AX, const double2* X, const double* w, double2* R, int rows, int64_t n) {
  const int64_t total = (int64_t)rows * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double wr = w[idx / n];
    R[idx] = make_double2(AX[idx].x - wr * X[idx].x, AX[idx].y - wr * X[idx].y);
  }
}
void launch_resid(const double2* AX, const double2* X, const double* w, double2* R, int rows, int64_t n,
                  hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(resid_kernel, dim3(nblocks((int64_t)rows * n, 256)), dim3(256), 0, s, AX, X, w, R, rows, n);
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
__global__ void fill_kernel(double2* p, int64_t n, cplx v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(v.re, v.im);
}
void launch_fill(double2* p, int64_t n, cplx v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n, v);
}

__global__ void scale_real_kernel(double2* p, const double* w, int64_t n, int64_t period, int invert) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double f = w[i % period];
    const double m = invert ? 1.0 / f : f;
    p[i].x *= m;
    p[i].y *= m;
  }
}
void launch_scale_real(double2* p, const double* w, int64_t n, int64_t period, int invert, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_real_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, w, n, period, invert);
}

__global__ void herm_add_kernel(const double2* X, double2* out, int64_t n) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / n, c = idx - r * n;
    const double2 a = X[idx], b = X[c * n + r];
    out[idx] = make_double2(a.x + b.x, a.y - b.y);
  }
}
void launch_herm_add(const double2* X, double2* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(herm_add_kernel, dim3(nblocks(n * n, 256)), dim3(256), 0, s, X, out, n);
}

__global__ void m11_add_delta_kernel(double2* M, const double2* f, int no, int nv, int which) {
  const int64_t n1 = (int64_t)no * nv;
  const int64_t total = which == 0 ? (int64_t)no * nv * nv : (int64_t)no * no * nv;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (which == 0) {  // delta_iI f[a][A]
      const int64_t i = idx / (nv * nv), r = idx - i * nv * nv, a = r / nv, A = r - a * nv;
      double2* d = M + (i * nv + a) * n1 + i * nv + A;
      d->x += f[a * nv + A].x;
      d->y += f[a * nv + A].y;
    } else {  // delta_aA h[i][I]
      const int64_t i = idx / ((int64_t)no * nv), r = idx - i * no * nv, I = r / nv, a = r - I * nv;
      double2* d = M + (i * nv + a) * n1 + I * nv + a;
      d->x += f[i * no + I].x;
      d->y += f[i * no + I].y;
    }
  }
}
void launch_m11_add_delta(double2* M, const double2* f, int no, int nv, int which, hipStream_t s) {
  const int64_t total = which == 0 ? (int64_t)no * nv * nv : (int64_t)no * no * nv;
  hipLaunchKernelGGL(m11_add_delta_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, M, f, no, nv, which);
}

__global__ void div_d2_kernel(double2* t, const double* eps, int no, int nv) {
  const int64_t total = (int64_t)no * no * nv * nv;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx;
    const int b = r % nv; r /= nv;
    const int a = r % nv; r /= nv;
    const int j = r % no; r /= no;
    const int i = (int)r;
    const double D = eps[i] + eps[j] - eps[no + a] - eps[no + b];
    t[idx].x /= D;
    t[idx].y /= D;
  }
}
void launch_div_d2(double2* t, const double* eps, int no, int nv, hipStream_t s) {
  const int64_t total = (int64_t)no * no * nv * nv;
  hipLaunchKernelGGL(div_d2_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, t, eps, no, nv);
}
__global__ void div_d1_kernel(double2* t, const double* eps, int no, int nv) {
  const int64_t total = (int64_t)no * nv;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / nv), a = (int)(idx % nv);
    const double D = eps[i] - eps[no + a];
    t[idx].x /= D;
    t[idx].y /= D;
  }
}
void launch_div_d1(double2* t, const double* eps, int no, int nv, hipStream_t s) {
  hipLaunchKernelGGL(div_d1_kernel, dim3(nblocks((int64_t)no * nv, 256)), dim3(256), 0, s, t, eps, no, nv);
}

// pair index of p<q among n: p*(2n-p-1)/2 + (q-p-1)
__device__ __forceinline__ int64_t pidx(int64_t p, int64_t q, int64_t n) { return p * (2 * n - p - 1) / 2 + (q - p - 1); }

// unpack: one thread per unpacked element
// one grid row (blockIdx.y) per vector z; the index arithmetic inside a
// vector is 32-bit
__global__ void unpack_doubles_kernel(int kind, const double2* Y, int64_t ldY, int64_t off, int k, int no, int nv,
                                      double2* Ya, double2* Yp, unsigned short* planes, int64_t pK, int64_t pKp) {
  const uint32_t uo = (uint32_t)no, uv = (uint32_t)nv;
  const uint32_t Po = uo * (uo - 1) / 2;
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  uint32_t per;
  if (kind == 0) per = uo * uo * uv * uv;
  else if (kind == 1) per = uo * uo * uv;
  else if (kind == 2) per = uo * uv * uv;
  else per = uv * Po * uv;
  const int64_t total = (int64_t)per * k;
  const int64_t z = blockIdx.y;
  // planes: row-major [rows][pK] elements into [4][rows][pKp] (pK divides
  // the per-vector size, or pK = total: one row)
  const bool flat = pK >= total;
  const uint32_t pK32 = flat ? 1u : (uint32_t)pK, rows_z = flat ? 0u : per / pK32;
  const int64_t plane = flat ? pKp : (total / pK) * pKp;
  for (uint32_t r0 = blockIdx.x * blockDim.x + threadIdx.x; r0 < per; r0 += gridDim.x * blockDim.x) {
    uint32_t r = r0;
    double sgn = 1.0;
    bool zero = false, canon = true;
    int64_t pos = 0;
    if (kind == 0) {
      const uint32_t b = r % uv; r /= uv;
      const uint32_t a = r % uv; r /= uv;
      const uint32_t j = r % uo, i = r / uo;
      if (i == j || a == b) zero = true;
      else {
        const int64_t i0 = i < j ? i : j, j0 = i < j ? j : i, a0 = a < b ? a : b, b0 = a < b ? b : a;
        if (i > j) sgn = -sgn;
        if (a > b) sgn = -sgn;
        canon = (i < j) && (a < b);
        pos = pidx(i0, j0, no) * Pv + pidx(a0, b0, nv);
      }
    } else if (kind == 1) {
      const uint32_t a = r % uv; r /= uv;
      const uint32_t j = r % uo, i = r / uo;
      if (i == j) zero = true;
      else {
        const int64_t i0 = i < j ? i : j, j0 = i < j ? j : i;
        if (i > j) sgn = -1.0;
        canon = i < j;
        pos = pidx(i0, j0, no) * nv + a;
      }
    } else if (kind == 3) {
      // EE doubles with the occupied pair packed, stored [z][a][pair ij][b]
      const uint32_t b = r % uv; r /= uv;
      const uint32_t p = r % Po, a = r / Po;
      if (a == b) zero = true;
      else {
        const int64_t a0 = a < b ? a : b, b0 = a < b ? b : a;
        if (a > b) sgn = -1.0;
        canon = a < b;
        pos = (int64_t)p * Pv + pidx(a0, b0, nv);
      }
    } else {
      const uint32_t b = r % uv; r /= uv;
      const uint32_t a = r % uv, i = r / uv;
      if (a == b) zero = true;
      else {
        const int64_t a0 = a < b ? a : b, b0 = a < b ? b : a;
        if (a > b) sgn = -1.0;
        canon = a < b;
        pos = (int64_t)i * Pv + pidx(a0, b0, nv);
      }
    }
    double2 v = make_double2(0.0, 0.0);
    if (!zero) {
      const double2 y = Y[z * ldY + off + pos];
      v = make_double2(sgn * y.x, sgn * y.y);
    }
    const int64_t idx = z * per + r0;
    if (Ya) Ya[idx] = v;
    if (Yp) Yp[idx] = (!zero && canon) ? v : make_double2(0.0, 0.0);
    if (planes) {
      if (flat) {
        put_planes(planes, plane, idx, v, 0);
      } else {
        const uint32_t rr = r0 / pK32, col = r0 - rr * pK32;
        const int64_t row = z * rows_z + rr;
        put_planes(planes, plane, row * pKp + col, v, 0);
        if ((int64_t)col < pKp - pK) put_planes(planes, plane, row * pKp + pK + col, make_double2(0.0, 0.0), 0);
      }
    }
  }
}
void launch_unpack_doubles(int kind, const double2* Y, int64_t ldY, int64_t off, int k, int no, int nv, double2* Ya,
                           double2* Yp, hipStream_t s, unsigned short* planes, int64_t pK, int64_t pKp) {
  const int64_t Po = (int64_t)no * (no - 1) / 2;
  const int64_t per = kind == 0 ? (int64_t)no * no * nv * nv
                                : (kind == 1 ? (int64_t)no * no * nv : (kind == 2 ? (int64_t)no * nv * nv : nv * Po * nv));
  if (per * k == 0) return;
  if (per >= ((int64_t)1 << 32)) throw std::invalid_argument("unpack_doubles: more than 2^32 elements per vector");
  if (planes && pK <= 0) pK = pKp = per * k;
  if (planes && pK < per * k && per % pK != 0) throw std::invalid_argument("unpack_doubles: plane rows across vectors");
  unsigned gx = nblocks(per, 256);
  if (gx > 65535) gx = 65535;
  hipLaunchKernelGGL(unpack_doubles_kernel, dim3(gx, (unsigned)k), dim3(256), 0, s, kind, Y, ldY, off, k, no, nv, Ya,
                     Yp, planes, pK, pKp);
}

// Split-bf16 planes [4][rows][Kp] of the EE doubles unpacked in the ring
// layout: row (z,i,a), column (k,c) holds Y_ikac (zero for i = k, and for
// columns o*v <= q < Kp)
// Yij [k][v][P_o][v] holds Y with the occupied pair packed: Y_ikac =
// sign(i,k) * Yij[z][a][pair(i,k)][c], read along c
__global__ __launch_bounds__(256) void ee_ring_planes_kernel(const double2* Yij, int k, int no, int nv,
                                                             unsigned short* dst, int64_t Kp) {
  // one block row per output row (z,i,a); 32-bit column arithmetic
  const uint32_t uo = (uint32_t)no, uv = (uint32_t)nv;
  const int64_t Po = (int64_t)no * (no - 1) / 2;
  const int64_t rows = (int64_t)k * no * nv, plane = rows * Kp;
  const uint32_t ov = uo * uv;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const int64_t a = r % nv, zi = r / nv, i = zi % no, z = zi / no;
    const double2* src = Yij + (z * nv + a) * Po * nv;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < (uint32_t)Kp; q += gridDim.x * blockDim.x) {
      double2 val = make_double2(0.0, 0.0);
      if (q < ov) {
        const uint32_t kk = q / uv, c = q - kk * uv;
        if ((int64_t)kk != i) {
          const int64_t i0 = i < kk ? i : kk, k0 = i < kk ? kk : i;
          const double2 y = src[pidx(i0, k0, no) * nv + c];
          val = i > kk ? make_double2(-y.x, -y.y) : y;
        }
      }
      put_planes(dst, plane, r * Kp + q, val, 0);
    }
  }
}
void launch_ee_ring_planes(const double2* Yij, int k, int no, int nv, unsigned short* dst, int64_t Kp,
                           hipStream_t s) {
  const int64_t rows = (int64_t)k * no * nv;
  if (rows * Kp == 0) return;
  unsigned gx = (unsigned)((Kp + 255) / 256);
  if (gx > 64) gx = 64;
  const unsigned gy = (unsigned)(rows < 65535 ? rows : 65535);
  hipLaunchKernelGGL(ee_ring_planes_kernel, dim3(gx, gy), dim3(256), 0, s, Yij, k, no, nv, dst, Kp);
}

__device__ __forceinline__ void put_planes_f(unsigned short* dst, int64_t plane, int64_t at, float2 v) {
  unsigned short h0, l0, h1, l1;
  split_bf16(v.x, h0, l0);
  split_bf16(v.y, h1, l1);
  dst[at] = h0;
  dst[plane + at] = l0;
  dst[2 * plane + at] = h1;
  dst[3 * plane + at] = l1;
}

// Split-bf16 planes of the EE doubles straight from the packed vectors
// (Y[z][pair ij][pair ab], i<j, a<b):
//  * yq [4][k*v][Kpy]: row (z,a), column (pair ij, b) = Y_ijab, zero for a = b
//    and for the padding columns P_o*v <= q < Kpy;
//  * rq [4][k*o*v][Kpr] (optional): row (z,i,a), column (k,c) = Y_ikac, zero
//    for i = k and for the padding columns o*v <= q < Kpr.
// Block (t, z): for t < P_o * npair one occupied pair and one pair A <= B of
// 64-wide tiles of the virtual index; the upper triangle of the tile is read
// once into LDS (as float2: every plane is split from the float value) and
// both (A,B) and its mirror (B,A) are written along their rows.  The last o
// blocks of a row z write the zero (i,i) blocks of rq and the padding.
constexpr int EPT = 64;
__global__ __launch_bounds__(256) void ee_pair_planes_kernel(const double2* Y, int64_t ldY, int64_t off, int no,
                                                             int nv, unsigned short* yq, int64_t Kpy, int64_t plane_y,
                                                             unsigned short* rq, int64_t Kpr, int64_t plane_r) {
  __shared__ float2 s[EPT][EPT + 1];
  const int z = blockIdx.y;
  const int nt = (nv + EPT - 1) / EPT, npair = nt * (nt + 1) / 2;
  const int Po = no * (no - 1) / 2;
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  const int tc = threadIdx.x % EPT, tr = threadIdx.x / EPT;  // 4 rows per pass
  constexpr int RP = 256 / EPT;
  const float2 zero = make_float2(0.f, 0.f);
  const int bid = blockIdx.x;
  if (bid >= Po * npair) {
    const int i = bid - Po * npair;
    if (rq) {
      for (int a = tr; a < nv; a += RP) {
        const int64_t row = ((int64_t)z * no + i) * nv + a;
        for (int c = tc; c < nv; c += EPT) put_planes_f(rq, plane_r, row * Kpr + (int64_t)i * nv + c, zero);
        for (int64_t q = (int64_t)no * nv + tc; q < Kpr; q += EPT) put_planes_f(rq, plane_r, row * Kpr + q, zero);
      }
    }
    if (i == 0) {
      for (int a = tr; a < nv; a += RP) {
        const int64_t row = (int64_t)z * nv + a;
        for (int64_t q = (int64_t)Po * nv + tc; q < Kpy; q += EPT) put_planes_f(yq, plane_y, row * Kpy + q, zero);
      }
    }
    return;
  }
  const int p = bid / npair;
  int t = bid - p * npair, A = 0;
  while (t >= nt - A) {
    t -= nt - A;
    ++A;
  }
  const int B = A + t;
  int i = 0, rem = p;
  while (rem >= no - 1 - i) {
    rem -= no - 1 - i;
    ++i;
  }
  const int kk = i + 1 + rem;
  const double2* src = Y + (int64_t)z * ldY + off + (int64_t)p * Pv;
  for (int r = tr; r < EPT; r += RP) {
    const int a = A * EPT + r, b = B * EPT + tc;
    float2 v = zero;
    if (a < b && b < nv) {
      const double2 y = src[pidx(a, b, nv)];
      v = make_float2((float)y.x, (float)y.y);
    }
    s[r][tc] = v;
  }
  __syncthreads();
  for (int g = 0; g < (A < B ? 2 : 1); ++g) {
    const int R = g == 0 ? A : B, Cb = g == 0 ? B : A;
    const int c = Cb * EPT + tc;
    if (c >= nv) continue;
    for (int r = tr; r < EPT; r += RP) {
      const int a = R * EPT + r;
      if (a >= nv) break;
      float2 v;
      if (g == 0 && (A < B || r < tc)) v = s[r][tc];
      else if (g == 0 && r == tc) v = zero;
      else v = make_float2(-s[tc][r].x, -s[tc][r].y);
      put_planes_f(yq, plane_y, ((int64_t)z * nv + a) * Kpy + (int64_t)p * nv + c, v);
      if (rq) {
        put_planes_f(rq, plane_r, (((int64_t)z * no + i) * nv + a) * Kpr + (int64_t)kk * nv + c, v);
        put_planes_f(rq, plane_r, (((int64_t)z * no + kk) * nv + a) * Kpr + (int64_t)i * nv + c,
                     make_float2(-v.x, -v.y));
      }
    }
  }
}
void launch_ee_pair_planes(const double2* Y, int64_t ldY, int64_t off, int k, int no, int nv, unsigned short* yq,
                           int64_t Kpy, unsigned short* rq, int64_t Kpr, hipStream_t s) {
  const int64_t Po = (int64_t)no * (no - 1) / 2, nt = (nv + EPT - 1) / EPT;
  if (k <= 0 || nv <= 0 || no <= 0) return;
  if (Kpy < Po * nv || (rq && Kpr < (int64_t)no * nv)) throw std::invalid_argument("ee_pair_planes: K padding");
  if (!yq) throw std::invalid_argument("ee_pair_planes: no destination");
  const int64_t gx = Po * (nt * (nt + 1) / 2) + no;
  if (gx > 0x7fffffff || k > 65535) throw std::invalid_argument("ee_pair_planes: grid");
  hipLaunchKernelGGL(ee_pair_planes_kernel, dim3((unsigned)gx, (unsigned)k), dim3(256), 0, s, Y, ldY, off, no, nv,
                     yq, Kpy, (int64_t)k * nv * Kpy, rq, Kpr, (int64_t)k * no * nv * Kpr);
}

// pack: one thread per packed element; po/pv are the pair tables of o and v
__global__ void pack_doubles_kernel(int kind, const double2* U, double2* S, const double2* Y, int64_t ld, int64_t off,
                                    int k, int no, int nv, const double* eps, cplx alpha, int accumulate,
                                    const int2* po, const int2* pv) {
  const int64_t Po = (int64_t)no * (no - 1) / 2, Pv = (int64_t)nv * (nv - 1) / 2;
  int64_t n2;
  if (kind == 0) n2 = Po * Pv;
  else if (kind == 1) n2 = Po * nv;
  else n2 = (int64_t)no * Pv;
  const int64_t per = kind == 0 ? (int64_t)no * no * nv * nv : (kind == 1 ? (int64_t)no * no * nv : (int64_t)no * nv * nv);
  const int64_t total = n2 * k;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = idx / n2, q = idx - z * n2;
    int64_t uoff;
    double D;
    if (kind == 0) {
      const int64_t pij = q / Pv, pab = q - pij * Pv;
      const int2 ij = po[pij], ab = pv[pab];
      uoff = (((int64_t)ij.x * no + ij.y) * nv + ab.x) * nv + ab.y;
      D = eps[no + ab.x] + eps[no + ab.y] - eps[ij.x] - eps[ij.y];
    } else if (kind == 1) {
      const int64_t pij = q / nv, a = q - pij * nv;
      const int2 ij = po[pij];
      uoff = ((int64_t)ij.x * no + ij.y) * nv + a;
      D = eps[no + a] - eps[ij.x] - eps[ij.y];
    } else {
      const int64_t i = q / Pv, pab = q - i * Pv;
      const int2 ab = pv[pab];
      uoff = (i * nv + ab.x) * nv + ab.y;
      D = eps[no + ab.x] + eps[no + ab.y] - eps[i];
    }
    double2 o = make_double2(0.0, 0.0);
    if (U) {
      const double2 u = U[z * per + uoff];
      o.x = alpha.re * u.x - alpha.im * u.y;
      o.y = alpha.re * u.y + alpha.im * u.x;
    }
    if (Y) {
      const double2 y = Y[z * ld + off + q];
      o.x += D * y.x;
      o.y += D * y.y;
    }
    double2* dst = S + z * ld + off + q;
    if (accumulate) {
      o.x += dst->x;
      o.y += dst->y;
    }
    *dst = o;
  }
}
void launch_pack_doubles(int kind, const double2* U, double2* S, const double2* Y, int64_t ld, int64_t off, int k,
                         int no, int nv, const double* eps, cplx alpha, int accumulate, const int2* po,
                         const int2* pv, hipStream_t s) {
  const int64_t Po = (int64_t)no * (no - 1) / 2, Pv = (int64_t)nv * (nv - 1) / 2;
  int64_t n2 = kind == 0 ? Po * Pv : (kind == 1 ? Po * nv : (int64_t)no * Pv);
  if (n2 * k == 0) return;
  hipLaunchKernelGGL(pack_doubles_kernel, dim3(nblocks(n2 * k, 256)), dim3(256), 0, s, kind, U, S, Y, ld, off, k,
                     no, nv, eps, alpha, accumulate, po, pv);
}

__global__ void antisym_add_kernel(const double2* X, double2* out, int64_t k, int64_t d1, int64_t d2, int64_t d3,
                                   int64_t d4, int which, cplx alpha) {
  const int64_t total = k * d1 * d2 * d3 * d4;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx;
    const int64_t e4 = r % d4; r /= d4;
    const int64_t e3 = r % d3; r /= d3;
    const int64_t e2 = r % d2; r /= d2;
    const int64_t e1 = r % d1; const int64_t z = r / d1;
    auto at = [&](int64_t a, int64_t b, int64_t c, int64_t d) { return X[(((z * d1 + a) * d2 + b) * d3 + c) * d4 + d]; };
    double2 v = at(e1, e2, e3, e4);
    if (which == 0) {
      const double2 w = at(e2, e1, e3, e4);
      v.x -= w.x; v.y -= w.y;
    } else if (which == 1) {
      const double2 w = at(e1, e2, e4, e3);
      v.x -= w.x; v.y -= w.y;
    } else {
      const double2 w1 = at(e2, e1, e3, e4), w2 = at(e1, e2, e4, e3), w3 = at(e2, e1, e4, e3);
      v.x += -w1.x - w2.x + w3.x;
      v.y += -w1.y - w2.y + w3.y;
    }
    double2 o = out[idx];
    o.x += alpha.re * v.x - alpha.im * v.y;
    o.y += alpha.re * v.y + alpha.im * v.x;
    out[idx] = o;
  }
}
void launch_antisym_add(const double2* X, double2* out, int64_t k, int64_t d1, int64_t d2, int64_t d3, int64_t d4,
                        int which, cplx alpha, hipStream_t s) {
  const int64_t total = k * d1 * d2 * d3 * d4;
  if (total == 0) return;
  hipLaunchKernelGGL(antisym_add_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, X, out, k, d1, d2, d3, d4, which,
                     alpha);
}

// ---------------------------------------------------------------------------
// ladder: pack antisymmetrised <ab||cd> rows from the assembled (ac|bd) block
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ladder_pack_kernel(const double2* W, int64_t ldw, int a0, int b0, int nv,
                                                          double2* V, int64_t pbase, const int2* pv, int64_t Pv) {
  const int64_t pr = blockIdx.y;              // row pair, relative to pbase
  const int2 ab = pv[pbase + pr];
  const int64_t ra = (int64_t)(ab.x - a0) * nv, cb = (int64_t)(ab.y - b0) * nv;
  for (int64_t pc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < Pv; pc += (int64_t)gridDim.x * blockDim.x) {
    const int2 cd = pv[pc];
    const double2 w1 = W[(ra + cd.x) * ldw + cb + cd.y];
    const double2 w2 = W[(ra + cd.y) * ldw + cb + cd.x];
    V[pr * Pv + pc] = make_double2(w1.x - w2.x, w1.y - w2.y);
  }
}
void launch_ladder_pack(const double2* W, int64_t ldw, int a0, int b0, int nv, double2* V, int64_t pbase,
                        int64_t npairs, const int2* pv, hipStream_t s) {
  const int64_t Pv = (int64_t)nv * (nv - 1) / 2;
  if (npairs <= 0 || Pv <= 0) return;
  unsigned gx = (unsigned)((Pv + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(ladder_pack_kernel, dim3(gx, (unsigned)npairs), dim3(256), 0, s, W, ldw, a0, b0, nv, V, pbase, pv,
                     Pv);
}

// ---------------------------------------------------------------------------
// Davidson helpers
// ---------------------------------------------------------------------------
int row_dot_blocks(int64_t n) {
  int64_t b = (n + 4095) / 4096;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

__global__ __launch_bounds__(256) void row_dots_kernel(const double2* X, int64_t ldx, const double2* Y, int64_t ldy,
                                                       int64_t n, double2* partial, int nb) {
  const int r = blockIdx.y, blk = blockIdx.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blk * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
  double sr = 0.0, si = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double2 x = X[(int64_t)r * ldx + i], y = Y[(int64_t)r * ldy + i];
    sr += x.x * y.x + x.y * y.y;
    si += x.x * y.y - x.y * y.x;
  }
  __shared__ double shr[256], shi[256];
  shr[threadIdx.x] = sr;
  shi[threadIdx.x] = si;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      shr[threadIdx.x] += shr[threadIdx.x + w];
      shi[threadIdx.x] += shi[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)r * nb + blk] = make_double2(shr[0], shi[0]);
}
void launch_row_dots(const double2* X, int64_t ldx, const double2* Y, int64_t ldy, int rows, int64_t n,
                     double2* partial, int nb, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(row_dots_kernel, dim3(nb, rows), dim3(256), 0, s, X, ldx, Y, ldy, n, partial, nb);
}

// Input check of a device-resident L [nq][n][n]: per Cholesky vector Q, the
// largest |Re L_pr - Re L_rp| + |Im L_pr + Im L_rp| (zero for Hermitian L^Q),
// the largest |component| and the number of non-finite components, written
// to out[3 Q .. 3 Q + 2]; one block per Q, rows of L read along r.
__global__ __launch_bounds__(256) void check_L_kernel(const double2* L, int64_t n, double* out) {
  const int64_t q = blockIdx.x;
  const double2* Lq = L + q * n * n;
  double dev = 0.0, mx = 0.0, bad = 0.0;
  for (int64_t e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int64_t p = e / n, r = e - p * n;
    const double2 a = Lq[e], b = Lq[r * n + p];
    if (!isfinite(a.x) || !isfinite(a.y)) {
      bad += 1.0;
      continue;
    }
    mx = fmax(mx, fmax(fabs(a.x), fabs(a.y)));
    if (isfinite(b.x) && isfinite(b.y)) dev = fmax(dev, fabs(a.x - b.x) + fabs(a.y + b.y));
  }
  __shared__ double sd[256], sm[256], sb[256];
  sd[threadIdx.x] = dev;
  sm[threadIdx.x] = mx;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + w]);
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * q] = sd[0];
    out[3 * q + 1] = sm[0];
    out[3 * q + 2] = sb[0];
  }
}
void launch_check_L(const double2* L, int64_t nq, int64_t n, double* out, hipStream_t s) {
  if (nq <= 0 || n <= 0) return;
  hipLaunchKernelGGL(check_L_kernel, dim3((unsigned)nq), dim3(256), 0, s, L, n, out);
}

// Workspace of the allocation-free sigma entry point: one array per device,
// held from module load until the process ends.  Host code never passes the
// name itself to a kernel (on the host it is only a stand-in); it takes the
// device address once per device with hipGetSymbolAddress and uses that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* scratch_address() {
  static std::mutex mu;
  static void* addr[64] = {};
  static bool done[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!done[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      ptr = nullptr;
    }
    addr[dev] = ptr;
    done[dev] = true;
  }
  return addr[dev];
}

__global__ void precondition_kernel(const double2* R, double2* N, const double* D, const double* w, int rows,
                                    int64_t n) {
  const int64_t total = (int64_t)rows * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / n, i = idx - r * n;
    double den = w[r] - D[i];
    if (fabs(den) < 1e-4) den = den < 0.0 ? -1e-4 : 1e-4;
    N[idx] = make_double2(R[idx].x / den, R[idx].y / den);
  }
}
void launch_precondition(const double2* R, double2* N, const double* D, const double* w, int rows, int64_t n,
                         hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(precondition_kernel, dim3(nblocks((int64_t)rows * n, 256)), dim3(256), 0, s, R, N, D, w, rows, n);
}

// EE doubles output, antisymmetrised and packed in one pass:
//   S[z][off + pair(i,j)*Pv + pair(a,b)] = A0[ij ab] - A0[ji ab]            (P(ij))
//        + A1[ij ab] - A1[ij ba]                                            (P(ab))
//        + A2[ij ab] - A2[ji ab] - A2[ij ba] + A2[ji ba]                    (P(ij)P(ab))
//        + D_ijab Y[z][off + ...]
// for i<j, a<b; A0..A2 are [k][o][o][v][v] (A2 may be null)
template <class AT>
__global__ __launch_bounds__(256) void pack_ee_kernel(const AT* A0, const AT* A1, const AT* A2, double2* S,
                                                      const double2* Y, int64_t ld, int64_t off, int k, int no, int nv,
                                                      const double* eps, const int2* po, const int2* pv) {
  const int64_t Po = (int64_t)no * (no - 1) / 2, Pv = (int64_t)nv * (nv - 1) / 2;
  const int64_t n2 = Po * Pv, per = (int64_t)no * no * nv * nv;
  const int64_t total = n2 * k;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = idx / n2, q = idx - z * n2;
    const int64_t pij = q / Pv, pab = q - pij * Pv;
    const int2 ij = po[pij], ab = pv[pab];
    const int64_t b0 = z * per;
    const int64_t o_ijab = (((int64_t)ij.x * no + ij.y) * nv + ab.x) * nv + ab.y;
    const int64_t o_jiab = (((int64_t)ij.y * no + ij.x) * nv + ab.x) * nv + ab.y;
    const int64_t o_ijba = (((int64_t)ij.x * no + ij.y) * nv + ab.y) * nv + ab.x;
    const int64_t o_jiba = (((int64_t)ij.y * no + ij.x) * nv + ab.y) * nv + ab.x;
    AT a = A0[b0 + o_ijab], c = A0[b0 + o_jiab];
    double rx = (double)a.x - (double)c.x, ry = (double)a.y - (double)c.y;
    a = A1[b0 + o_ijab];
    c = A1[b0 + o_ijba];
    rx += (double)a.x - (double)c.x;
    ry += (double)a.y - (double)c.y;
    if (A2) {
      const AT w1 = A2[b0 + o_ijab], w2 = A2[b0 + o_jiab], w3 = A2[b0 + o_ijba], w4 = A2[b0 + o_jiba];
      rx += (double)w1.x - (double)w2.x - (double)w3.x + (double)w4.x;
      ry += (double)w1.y - (double)w2.y - (double)w3.y + (double)w4.y;
    }
    const double D = eps[no + ab.x] + eps[no + ab.y] - eps[ij.x] - eps[ij.y];
    const double2 y = Y[z * ld + off + q];
    S[z * ld + off + q] = make_double2(rx + D * y.x, ry + D * y.y);
  }
}
void launch_pack_ee(const double2* A0, const double2* A1, const double2* A2, double2* S, const double2* Y, int64_t ld,
                    int64_t off, int k, int no, int nv, const double* eps, const int2* po, const int2* pv,
                    hipStream_t s, int a32) {
  const int64_t n2 = (int64_t)no * (no - 1) / 2 * ((int64_t)nv * (nv - 1) / 2);
  if (n2 * k == 0) return;
  if (a32)
    hipLaunchKernelGGL(pack_ee_kernel<float2>, dim3(nblocks(n2 * k, 256)), dim3(256), 0, s, (const float2*)A0,
                       (const float2*)A1, (const float2*)A2, S, Y, ld, off, k, no, nv, eps, po, pv);
  else
    hipLaunchKernelGGL(pack_ee_kernel<double2>, dim3(nblocks(n2 * k, 256)), dim3(256), 0, s, A0, A1, A2, S, Y, ld,
                       off, k, no, nv, eps, po, pv);
}

// EE doubles output from accumulators that store only the half they need:
// A0 is antisymmetric in (a,b) and kept as [k][o][o][P_v], A1 antisymmetric in
// (i,j) and kept as [k][P_o][v][v]; A2 stays [k][o][o][v][v] (or null).
//   S = A0[ij,ab] - A0[ji,ab] + A1[ij,ab] - A1[ij,ba] + P(ij)P(ab) A2 + D Y
template <class AT>
__global__ __launch_bounds__(256) void pack_ee_half_kernel(const AT* A0, const AT* A1, const AT* A2, double2* S,
                                                           const double2* Y, int64_t ld, int64_t off, int k, int no,
                                                           int nv, const double* eps, const int2* po) {
  // one block per (z, pair ij, 16x16 tile (ta <= tb) of (a, b)); the
  // transposed reads A1[..][b][a], A2[..][b][a] go through LDS
  __shared__ AT t1[16][17], t2[16][17], t3[16][17];
  const int64_t Po = (int64_t)no * (no - 1) / 2, Pv = (int64_t)nv * (nv - 1) / 2;
  const int nt = (nv + 15) / 16;
  const int64_t ntile = (int64_t)nt * (nt + 1) / 2;
  const int64_t blk = blockIdx.x;
  const int64_t tile = blk % ntile, zp = blk / ntile, pij = zp % Po, z = zp / Po;
  int ta = 0;
  {
    int64_t rem = tile;
    while (rem >= nt - ta) { rem -= nt - ta; ++ta; }
    const int tb = ta + (int)rem;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int2 ij = po[pij];
    const int64_t per0 = (int64_t)no * no * Pv, per1 = Po * nv * nv, per2 = (int64_t)no * no * nv * nv;
    const int64_t b1 = z * per1 + pij * nv * nv;
    const int64_t b2ij = z * per2 + ((int64_t)ij.x * no + ij.y) * nv * nv;
    const int64_t b2ji = z * per2 + ((int64_t)ij.y * no + ij.x) * nv * nv;
    // transposed blocks: rows b of tile tb, columns a of tile ta
    {
      const int bb = 16 * tb + ty, aa = 16 * ta + tx;
      AT zero;
      zero.x = 0; zero.y = 0;
      const bool in = bb < nv && aa < nv;
      t1[ty][tx] = in ? A1[b1 + (int64_t)bb * nv + aa] : zero;
      if (A2) {
        t2[ty][tx] = in ? A2[b2ij + (int64_t)bb * nv + aa] : zero;
        t3[ty][tx] = in ? A2[b2ji + (int64_t)bb * nv + aa] : zero;
      }
    }
    __syncthreads();
    const int a = 16 * ta + ty, b = 16 * tb + tx;
    if (a < nv && b < nv && a < b) {
      const int64_t pab = (int64_t)a * (2 * nv - a - 1) / 2 + (b - a - 1);
      const AT x0 = A0[z * per0 + ((int64_t)ij.x * no + ij.y) * Pv + pab];
      const AT x1 = A0[z * per0 + ((int64_t)ij.y * no + ij.x) * Pv + pab];
      const AT y0 = A1[b1 + (int64_t)a * nv + b];
      const AT y1 = t1[tx][ty];
      double rx = (double)x0.x - (double)x1.x + (double)y0.x - (double)y1.x;
      double ry = (double)x0.y - (double)x1.y + (double)y0.y - (double)y1.y;
      if (A2) {
        const AT w1 = A2[b2ij + (int64_t)a * nv + b], w2 = A2[b2ji + (int64_t)a * nv + b];
        const AT w3 = t2[tx][ty], w4 = t3[tx][ty];
        rx += (double)w1.x - (double)w2.x - (double)w3.x + (double)w4.x;
        ry += (double)w1.y - (double)w2.y - (double)w3.y + (double)w4.y;
      }
      const double D = eps[no + a] + eps[no + b] - eps[ij.x] - eps[ij.y];
      const int64_t q = pij * Pv + pab;
      const double2 y = Y[z * ld + off + q];
      S[z * ld + off + q] = make_double2(rx + D * y.x, ry + D * y.y);
    }
  }
}
void launch_pack_ee_half(const double2* A0, const double2* A1, const double2* A2, double2* S, const double2* Y,
                         int64_t ld, int64_t off, int k, int no, int nv, const double* eps, const int2* po,
                         const int2* pv, hipStream_t s, int a32) {
  const int64_t Po = (int64_t)no * (no - 1) / 2, Pv = (int64_t)nv * (nv - 1) / 2;
  if (Po * Pv * k == 0) return;
  (void)pv;
  const int64_t nt = (nv + 15) / 16, blocks = (int64_t)k * Po * (nt * (nt + 1) / 2);
  if (a32)
    hipLaunchKernelGGL(pack_ee_half_kernel<float2>, dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)A0,
                       (const float2*)A1, (const float2*)A2, S, Y, ld, off, k, no, nv, eps, po);
  else
    hipLaunchKernelGGL(pack_ee_half_kernel<double2>, dim3((unsigned)blocks), dim3(256), 0, s, A0, A1, A2, S, Y, ld,
                       off, k, no, nv, eps, po);
}

// dst[o][p(a<b)][i] = src[o][a][b][i] for src [outer][n][n][inner]
__global__ void pack_pairs_kernel(const double2* src, double2* dst, int64_t outer, int n, int64_t inner,
                                  const int2* pairs, int anti) {
  const int64_t P = (int64_t)n * (n - 1) / 2, total = outer * P * inner;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % inner, r = idx / inner, p = r % P, o = r / P;
    const int2 ab = pairs[p];
    double2 v = src[((o * n + ab.x) * n + ab.y) * inner + i];
    if (anti) {
      const double2 w = src[((o * n + ab.y) * n + ab.x) * inner + i];
      v.x -= w.x;
      v.y -= w.y;
    }
    dst[idx] = v;
  }
}
void launch_pack_pairs(const double2* src, double2* dst, int64_t outer, int n, int64_t inner, const int2* pairs,
                       hipStream_t s, int anti) {
  const int64_t total = outer * ((int64_t)n * (n - 1) / 2) * inner;
  if (total == 0) return;
  hipLaunchKernelGGL(pack_pairs_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, src, dst, outer, n, inner, pairs,
                     anti);
}

// ---------------------------------------------------------------------------
// adjoint helpers
// ---------------------------------------------------------------------------
// which 0: gf[a][A] += sum_i gX[(i,a),(i,A)] ; which 1: gf[i][I] += sum_a gX[(i,a),(I,a)]
__global__ void m11_delta_adjoint_kernel(const double2* gX, double2* gf, int no, int nv, int which) {
  const int64_t n1 = (int64_t)no * nv;
  const int64_t total = which == 0 ? (int64_t)nv * nv : (int64_t)no * no;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    if (which == 0) {
      const int64_t a = idx / nv, A = idx - a * nv;
      for (int64_t i = 0; i < no; ++i) {
        const double2 g = gX[(i * nv + a) * n1 + i * nv + A];
        acc.x += g.x;
        acc.y += g.y;
      }
    } else {
      const int64_t i = idx / no, I = idx - i * no;
      for (int64_t a = 0; a < nv; ++a) {
        const double2 g = gX[(i * nv + a) * n1 + I * nv + a];
        acc.x += g.x;
        acc.y += g.y;
      }
    }
    gf[idx].x += acc.x;
    gf[idx].y += acc.y;
  }
}
void launch_m11_delta_adjoint(const double2* gX, double2* gf, int no, int nv, int which, hipStream_t s) {
  const int64_t total = which == 0 ? (int64_t)nv * nv : (int64_t)no * no;
  if (total == 0) return;
  hipLaunchKernelGGL(m11_delta_adjoint_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, gX, gf, no, nv, which);
}

// G[(x - x0) nv + y][b nv + d] = s * Gam[pair(x,b)][pair(y,d)],
// s = sign(b - x) sign(d - y), zero when x == b or y == d
__global__ __launch_bounds__(256) void expand_gamma_kernel(const double2* Gam, int64_t Pv, int x0, int x1, int nv,
                                                           double2* G) {
  const int64_t v = nv;
  const int64_t total = (int64_t)(x1 - x0) * v * v * v;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx;
    const int64_t d = r % v; r /= v;
    const int64_t b = r % v; r /= v;
    const int64_t y = r % v;
    const int64_t x = x0 + r / v;
    double2 out = make_double2(0.0, 0.0);
    if (x != b && y != d) {
      const int64_t p = x < b ? pidx(x, b, v) : pidx(b, x, v);
      const int64_t q = y < d ? pidx(y, d, v) : pidx(d, y, v);
      const double2 g = Gam[p * Pv + q];
      const double s = ((b > x) == (d > y)) ? 1.0 : -1.0;
      out = make_double2(s * g.x, s * g.y);
    }
    G[idx] = out;
  }
}
void launch_expand_gamma(const double2* Gam, int64_t Pv, int x0, int x1, int nv, double2* G, hipStream_t s) {
  const int64_t total = (int64_t)(x1 - x0) * nv * nv * nv;
  if (total <= 0) return;
  hipLaunchKernelGGL(expand_gamma_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, Gam, Pv, x0, x1, nv, G);
}

// dL[Q][p][q] = (G[Q][p][q] + conj(G[Q][q][p])) / 2
__global__ void herm_project_kernel(const double2* G, double2* dL, int64_t nq, int64_t n) {
  const int64_t total = nq * n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t Q = idx / (n * n), r = idx - Q * n * n, p = r / n, q = r - p * n;
    const double2 a = G[idx], b = G[Q * n * n + q * n + p];
    dL[idx] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
}
void launch_herm_project(const double2* G, double2* dL, int64_t nq, int64_t n, hipStream_t s) {
  if (nq * n * n == 0) return;
  hipLaunchKernelGGL(herm_project_kernel, dim3(nblocks(nq * n * n, 256)), dim3(256), 0, s, G, dL, nq, n);
}

}  // namespace adc
