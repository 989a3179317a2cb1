// Device kernels for gfx950 (CDNA4, wave64).  See kernels.h for the
// descriptor of each launch.
#include <map>
#include <tuple>
#include "kernels.h"
#include "prof.h"

#include <climits>
#include <limits>
#include <mutex>

namespace mfh {

namespace {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T noise_rel();
template <>
__device__ __forceinline__ double noise_rel<double>() { return 64.0 * 1.1102230246251565e-16; }
template <>
__device__ __forceinline__ float noise_rel<float>() { return 64.0f * 5.9604644775390625e-08f; }

__device__ __forceinline__ double wave_max(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// block-wide reductions; every thread receives the result
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < (int)(blockDim.x / kWave); ++i) r = fmax(r, sh[i]);
  return r;
}
__device__ int block_min(int v, int* sh) {
  v = wave_min(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  int r = sh[0];
  for (int i = 1; i < (int)(blockDim.x / kWave); ++i) r = min(r, sh[i]);
  return r;
}
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < (int)(blockDim.x / kWave); ++i) r += sh[i];
  return r;
}

template <typename D>
__device__ __forceinline__ int find_desc(const D* d, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile0 <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// The same search by a whole workgroup (every thread calls it): each thread
// probes one descriptor, so a round is one parallel load instead of a chain
// of dependent ones; the probes at or below key form a prefix, counted by
// one barrier.  More than blockDim.x descriptors take a coarse round first.
template <typename D>
__device__ __forceinline__ int find_desc_wg(const D* d, int n, int key) {
  const int t = threadIdx.x, nt = blockDim.x;
  int lo = 0, hi = n;                       // d[lo].tile0 <= key; the answer is in [lo, hi)
  while (hi - lo > nt) {
    const int step = (hi - lo + nt - 1) / nt;
    const int i = lo + t * step;
    const int c = __syncthreads_count(i < hi && d[i].tile0 <= key);
    lo += (c - 1) * step;
    hi = min(hi, lo + step);
  }
  const int c = __syncthreads_count(lo + t < hi && d[lo + t].tile0 <= key);
  return lo + c - 1;
}

// 16x16x4 MFMA: lane l supplies A(l%16, l/16) and B(l/16, l%16); its four
// accumulator values hold D(row(l/16, v), l%16), v = 0..3.  The row map
// differs between the float64 and float32 instructions.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// bfloat16: the high 16 bits of a float32; conversion rounds to nearest,
// ties to even (NaN stays NaN)
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ unsigned short float_to_bf16(float v) {
  const unsigned b = __float_as_uint(v);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (unsigned short)((b >> 16) | 0x0040u);
  return (unsigned short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
template <typename T>
__device__ __forceinline__ T load_op(const T* p, size_t idx, bool bf16) {
  if constexpr (sizeof(T) == 4) {
    if (bf16) return bf16_to_float(reinterpret_cast<const unsigned short*>(p)[idx]);
  }
  return p[idx];
}
// The GEMM's operand loads keep a bfloat16 element's raw bits (zero-extended)
// in the register and widen it when the register is written to LDS: a
// conversion right after the load would wait for that load before the next
// one is issued.
template <typename T>
__device__ __forceinline__ T load_raw(const T* p, size_t idx, bool bf16) {
  if constexpr (sizeof(T) == 4) {
    if (bf16) return __uint_as_float((unsigned)reinterpret_cast<const unsigned short*>(p)[idx]);
  }
  return p[idx];
}
template <typename T>
__device__ __forceinline__ T widen_raw(T v, bool bf16) {
  if constexpr (sizeof(T) == 4) {
    if (bf16) return __uint_as_float(__float_as_uint(v) << 16);
  }
  return v;
}

// ---------------------------------------------------------------- GEMM ----
// 64x64 output tile per workgroup, 4 waves each owning a 32x32 quadrant as
// 2x2 MFMA 16x16x4 tiles.  K advances in steps of kGemmBK<T> staged through
// LDS; the next step's operands are loaded into registers while the MFMAs
// work on the current one.
// BN = 64: 64 x 64 output tiles, the four waves in a 2 x 2 grid of 32 x 32
// (2 x 2 MFMA tiles each).  BN = 16 (right-hand-side blocks of at most 16
// columns): 64 x 16 tiles, each wave one 16 x 16 MFMA tile, so no MFMA work
// is spent on empty columns.
template <typename T, int BN>
struct GemmLds {
  T As[kGemmBK<T>][kTile + 1];
  T Bs[kGemmBK<T>][BN + 1];
};
// ROWS: 0 no row maps; 1 a row map on B only, op N (the apply's reads of
// x(I_p^f)); 2 row maps on A and/or B in either op; 3 B formed from the
// partial slices of a split product whose reduction launch was folded into
// this one (op N, no row maps; gemm_narrow_fold_kernel only).  Each case is its own body: the general one
// costs the others about a tenth of a launch.
template <typename T, int BN, int ROWS>
__device__ __forceinline__ void gemm_tile_body(const GemmDesc<T>& d, int lt, GemmLds<T, BN>& L,
                                               const FoldDesc<T>* __restrict__ fd = nullptr) {
  constexpr int BM = kTile, BK = kGemmBK<T>, NQ = BK * 64 / 256, NQB = BK * BN / 256;
  constexpr bool NARROW = BN == 16;
  auto& As = L.As;
  auto& Bs = L.Bs;
  typedef typename Mfma<T>::v4 v4;
  const int tid = threadIdx.x;
  const int tm = lt % d.tiles_m, rest = lt / d.tiles_m;
  const int tn = rest % d.tiles_n, ks = rest / d.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int m = d.m, n = d.n, flags = d.flags;
  const int k = d.kdev ? *d.kdev : d.k;
  const bool split = d.ksplit > 1;
  if ((flags & GF_LOWER_C) && n0 >= m0 + BM) return;   // above the diagonal (never read back)
  int kb0 = 0, kend = k;
  if (flags & GF_A_LOWER) kend = min(kend, m0 + BM);
  if (flags & GF_B_UPPER) kend = min(kend, n0 + BN);
  if (flags & GF_A_UPPER) kb0 = max(kb0, m0);
  if (flags & GF_B_LOWER) kb0 = max(kb0, n0);
  kb0 = (kb0 / BK) * BK;
  if (split) {                       // this workgroup's share of k (kchunk is a multiple of kGemmSplitAlign)
    kb0 = max(kb0, ks * d.kchunk);
    kend = min(kend, (ks + 1) * d.kchunk);
  }
  const T* __restrict__ A = d.A;
  const T* __restrict__ B = d.B;
  const int* __restrict__ arow = d.arow;
  const int* __restrict__ brow = d.brow;
  const int lda = d.lda, ldb = d.ldb, opA = d.opA, opB = d.opB;
  const int bsplit = ROWS == 3 ? fd->split : 0;
  // the fold descriptor's fields, read once (uniform) and selected per thread
  int fS0 = 0, fS1 = 0, fld0 = 0, fld1 = 0;
  const T* __restrict__ fp0 = nullptr;
  const T* __restrict__ fp1 = nullptr;
  if constexpr (ROWS == 3) {
    fS0 = fd->slices[0]; fS1 = fd->slices[1];
    fld0 = fd->ld[0]; fld1 = fd->ld[1];
    fp0 = fd->part[0]; fp1 = fd->part[1];
  }
  const bool abf = (flags & GF_A_BF16) != 0, bbf = (flags & GF_B_BF16) != 0;
  v4 acc00 = {0, 0, 0, 0}, acc01 = {0, 0, 0, 0}, acc10 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = NARROW ? wave * 16 : (wave >> 1) * 32, wn = NARROW ? 0 : (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // per-thread load coordinates: (row of the tile, k offset) for each of NQ loads
  // op N: row = tid & 63, k = (tid >> 6) + 4q;   op T: k = tid % BK, row = tid / BK + (256 / BK) q
  T ra[NQ], rb[NQB];
  T fw[ROWS == 3 ? NQB : 1][ROWS == 3 ? kFoldSlices : 1];   // folded partial slices
  int fs[ROWS == 3 ? NQB : 1];                               // 0: B as read; 1 + source
  auto load = [&](int kb) {
    // A thread's loads of one operand all fall in one stored row (op N of A:
    // row tid & 63; op T of A and op N of B: k = tid % BK; op T of B: column
    // tid % BN), so a row map costs one index load per operand and k block,
    // issued ahead of the data loads; clamped indices keep it in the map.
    int amap = 0, bmap = 0;
    if constexpr (ROWS == 2) {
      if (arow) amap = arow[opA == 0 ? min(m0 + (tid & 63), m - 1) : min(kb + tid % BK, kend - 1)];
      if (brow) bmap = brow[opB == 0 ? min(kb + tid % BK, kend - 1) : min(n0 + tid % BN, n - 1)];
    }
    if constexpr (ROWS == 1) bmap = brow[min(kb + tid % BK, kend - 1)];   // op N: row kb + tid % BK
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int i, kk;
      if (opA == 0) { i = tid & 63; kk = (tid >> 6) + 4 * q; }
      else { kk = tid % BK; i = tid / BK + (256 / BK) * q; }
      const int gi = m0 + i, gk = kb + kk;
      if constexpr (ROWS == 2) {
        const bool ok = gi < m && gk < kend;
        int sr = opA == 0 ? gi : gk;   // stored row
        sr = arow ? amap : sr;
        ra[q] = ok ? load_raw(A, opA == 0 ? sr + (size_t)gk * lda : sr + (size_t)gi * lda, abf) : (T)0;
      } else {
        ra[q] = (gi < m && gk < kend)
                    ? load_raw(A, opA == 0 ? gi + (size_t)gk * lda : gk + (size_t)gi * lda, abf)
                    : (T)0;
      }
    }
#pragma unroll
    for (int q = 0; q < NQB; ++q) {
      int j, kk;
      if (opB == 0) { kk = tid % BK; j = tid / BK + (256 / BK) * q; }
      else { j = tid % BN; kk = tid / BN + (256 / BN) * q; }
      const int gj = n0 + j, gk = kb + kk;
      const bool ok = gj < n && gk < kend;
      if constexpr (ROWS == 3) {
        // op N: the element's partial slices (at most kFoldSlices) stay in
        // registers until stash() sums them.  Each lane of a column inside
        // the tile issues kFoldSlices loads (slice indices clamped), so
        // that none waits for another; columns outside load nothing.
        int S = 0, src = 0;
        if (gj < n) {   // a column is shared by a whole wave (FP32) or half a wave (FP64)
          // rows past kend (last k step) read row kend - 1 and are zeroed in stash()
          const int gkc = min(gk, kend - 1);
          src = gkc >= bsplit ? 1 : 0;
          S = src ? fS1 : fS0;
          const int ld = src ? fld1 : fld0;
          const size_t bi = gkc + (size_t)gj * ldb;
          const T* __restrict__ p = B + bi;
          size_t str = 0;
          if (S) {
            p = (src ? fp1 : fp0) + (gkc - (src ? bsplit : 0)) + (size_t)gj * ld;
            str = (size_t)ld * n;
          }
          const int last = S > 0 ? S - 1 : 0;
#pragma unroll
          for (int u = 0; u < kFoldSlices; ++u) fw[q][u] = p[(size_t)min(u, last) * str];
          rb[q] = B[bi];
        }
        fs[q] = ok ? (S << 2) | (src << 1) | 1 : 0;
      } else if constexpr (ROWS == 2) {
        int sr = opB == 0 ? gk : gj;   // stored row
        sr = brow ? bmap : sr;
        rb[q] = ok ? load_raw(B, opB == 0 ? sr + (size_t)gj * ldb : sr + (size_t)gk * ldb, bbf) : (T)0;
      } else {
        int bk = gk;
        if constexpr (ROWS == 1) bk = bmap;   // op N when only B's rows are mapped (kk = tid % BK)
        rb[q] = ok ? load_raw(B, opB == 0 ? bk + (size_t)gj * ldb : gj + (size_t)gk * ldb, bbf) : (T)0;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int i, kk;
      if (opA == 0) { i = tid & 63; kk = (tid >> 6) + 4 * q; }
      else { kk = tid % BK; i = tid / BK + (256 / BK) * q; }
      As[kk][i] = widen_raw(ra[q], abf);
    }
#pragma unroll
    for (int q = 0; q < NQB; ++q) {
      int j, kk;
      if (opB == 0) { kk = tid % BK; j = tid / BK + (256 / BK) * q; }
      else { j = tid % BN; kk = tid / BN + (256 / BN) * q; }
      if constexpr (ROWS == 3) {
        const int S = fs[q] >> 2, src = (fs[q] >> 1) & 1;
        if (!(fs[q] & 1)) rb[q] = (T)0;   // outside the tile; inside with no slices: B as read
        if (S) {   // the reduction's arithmetic, slices in order
          T s = (T)0;
#pragma unroll
          for (int u = 0; u < kFoldSlices; ++u) s += u < S ? fw[q][u] : (T)0;
          const T bb = (T)(src ? fd->beta[1] : fd->beta[0]);
          T v = (T)(src ? fd->alpha[1] : fd->alpha[0]) * s;
          if (bb != (T)0) v += bb * rb[q];
          rb[q] = v;
        }
      }
      Bs[kk][j] = ROWS == 3 ? rb[q] : widen_raw(rb[q], bbf);
    }
  };
  if (kb0 < kend) load(kb0);
  for (int kb = kb0; kb < kend; kb += BK) {
    stash();
    __syncthreads();
    if (kb + BK < kend) load(kb + BK);      // in flight while the MFMAs run
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kq = k4 * 4 + lk;
      if constexpr (NARROW) {
        acc00 = Mfma<T>::run(As[kq][wm + li], Bs[kq][li], acc00);
      } else {
        const T a0 = As[kq][wm + li], a1 = As[kq][wm + 16 + li];
        const T b0 = Bs[kq][wn + li], b1 = Bs[kq][wn + 16 + li];
        acc00 = Mfma<T>::run(a0, b0, acc00);
        acc01 = Mfma<T>::run(a0, b1, acc01);
        acc10 = Mfma<T>::run(a1, b0, acc10);
        acc11 = Mfma<T>::run(a1, b1, acc11);
      }
    }
    __syncthreads();
  }
  const T alpha = (T)d.alpha, beta = (T)d.beta;
  T* __restrict__ C = split ? d.part + (size_t)ks * m * n : d.C;
  const int ldc = split ? m : d.ldc;
  const v4* accs[4] = {&acc00, &acc01, &acc10, &acc11};
#pragma unroll
  for (int ab = 0; ab < (NARROW ? 1 : 4); ++ab) {
    const int a = ab >> 1, b = ab & 1;
    const v4 acc = *accs[ab];
    const int col = n0 + wn + b * 16 + li;
    // the four C values (beta != 0) are loaded before any is used, so that
    // their loads are in flight together
    T cv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wm + a * 16 + Mfma<T>::row(lk, v);
      const bool rd = !split && beta != (T)0 && row < m && col < n && (!(flags & GF_LOWER_C) || row >= col);
      cv[v] = rd ? C[row + (size_t)col * ldc] : (T)0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wm + a * 16 + Mfma<T>::row(lk, v);
      if (row < m && col < n) {
        T* c = C + row + (size_t)col * ldc;
        if (split) {
          *c = acc[v];
        } else if (!(flags & GF_LOWER_C) || row >= col) {
          T val = alpha * acc[v];
          if (beta != (T)0) val += beta * cv[v];
          *c = val;
        }
      }
    }
  }
}

template <typename T, int BN>
__device__ __forceinline__ void gemm_tile(const GemmDesc<T>* __restrict__ descs, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const GemmDesc<T>& d = descs[di];
  const int lt = (int)blockIdx.x - d.tile0;
  __shared__ GemmLds<T, BN> L;   // one LDS block for every body
  if (d.arow || (d.brow && d.opB != 0)) gemm_tile_body<T, BN, 2>(d, lt, L);
  else if (d.brow) gemm_tile_body<T, BN, 1>(d, lt, L);
  else gemm_tile_body<T, BN, 0>(d, lt, L);
}

template <typename T>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc<T>* __restrict__ descs, int ndesc) {
  gemm_tile<T, kTile>(descs, ndesc);
}
template <typename T>
__global__ __launch_bounds__(256) void gemm_narrow_kernel(const GemmDesc<T>* __restrict__ descs, int ndesc) {
  gemm_tile<T, kTileNarrow>(descs, ndesc);
}

// A batch of which some products read B from folded split-K partials; a
// kernel of its own, so that the other launches keep their registers.
template <typename T>
__global__ __launch_bounds__(256) void gemm_narrow_fold_kernel(const GemmDesc<T>* __restrict__ descs,
                                                               const FoldDesc<T>* __restrict__ folds, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const GemmDesc<T>& d = descs[di];
  const FoldDesc<T>* f = folds + di;
  const int lt = (int)blockIdx.x - d.tile0;
  __shared__ GemmLds<T, kTileNarrow> L;
  if (f->slices[0] > 0 || f->slices[1] > 0) gemm_tile_body<T, kTileNarrow, 3>(d, lt, L, f);
  else if (d.arow || (d.brow && d.opB != 0)) gemm_tile_body<T, kTileNarrow, 2>(d, lt, L);
  else if (d.brow) gemm_tile_body<T, kTileNarrow, 1>(d, lt, L);
  else gemm_tile_body<T, kTileNarrow, 0>(d, lt, L);
}

template <typename T>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const GemmDesc<T>* __restrict__ descs, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const GemmDesc<T>& d = descs[di];
  const int lt = (int)blockIdx.x - d.tile0;
  const int m0 = (lt % d.tiles_m) * kTile, n0 = (lt / d.tiles_m) * kTile;
  const int m = d.m, n = d.n, S = d.ksplit;
  const bool lower = (d.flags & GF_LOWER_C) != 0;
  const T alpha = (T)d.alpha, beta = (T)d.beta;
  const size_t mn = (size_t)m * n;
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int row = m0 + (e & 63), col = n0 + (e >> 6);
    if (row >= m || col >= n || (lower && row < col)) continue;
    const T* p = d.part + row + (size_t)col * m;
    T s = 0;
    for (int q0 = 0; q0 < S; q0 += 8) {   // eight slices' loads in flight at once, summed in slice order
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = q0 + u < S ? p[(size_t)(q0 + u) * mn] : (T)0;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    T* c = d.C + row + (size_t)col * d.ldc;
    T val = alpha * s;
    if (beta != (T)0) val += beta * *c;
    *c = val;
  }
}

// One wave: D = A B with A(i,0) = i, B(0,j) = 1 (so D(i,j) = i), and with
// A(i,0) = 1, B(0,j) = j (so D(i,j) = j); reports where each lane's four
// accumulator values sit, next to the row map the GEMM epilogue assumes.
template <typename T>
__global__ void mfma_probe_kernel(int* rows, int* cols, int* assumed) {
  typedef typename Mfma<T>::v4 v4;
  const int l = threadIdx.x, li = l & 15, lk = l >> 4;
  v4 d1 = {0, 0, 0, 0}, d2 = {0, 0, 0, 0};
  d1 = Mfma<T>::run(lk == 0 ? (T)li : (T)0, lk == 0 ? (T)1 : (T)0, d1);
  d2 = Mfma<T>::run(lk == 0 ? (T)1 : (T)0, lk == 0 ? (T)li : (T)0, d2);
  for (int v = 0; v < 4; ++v) {
    rows[l * 4 + v] = (int)d1[v];
    cols[l * 4 + v] = (int)d2[v];
    assumed[l * 4 + v] = Mfma<T>::row(lk, v);
  }
}

// ------------------------------------------ register-resident skeleton ----
// Pivot key: |v| truncated in the high word (FP64: 20 mantissa bits; FP32:
// 16, which leaves room for a position inside one 32-bit word in the
// register kernel below), the complement of the element's position in the
// low word, ordered by column, then row, so the largest key is the largest
// truncated magnitude with the lowest column, then the lowest row.  A zero
// magnitude never wins (key 0 = no candidate).
typedef unsigned long long u64;

__device__ __forceinline__ unsigned qmag(double v) {
  return (unsigned)(__double_as_longlong(fabs(v)) >> 32);
}
__device__ __forceinline__ unsigned qmag(float v) { return (unsigned)__float_as_uint(fabsf(v)) >> 7; }

__device__ __forceinline__ u64 make_key(unsigned q, unsigned idx) {
  return q == 0u ? 0ull : (((u64)q) << 32) | (u64)(0xFFFFFFFFu - idx);
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(v & 0xFFFFFFFFull), o, kWave);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), o, kWave);
    const u64 w = (((u64)hi) << 32) | lo;
    v = w > v ? w : v;
  }
  return v;
}

__device__ u64 block_max_u64(u64 v, u64* sh) {
  v = wave_max_u64(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  u64 r = sh[0];
  for (int i = 1; i < (int)(blockDim.x / kWave); ++i) r = sh[i] > r ? sh[i] : r;
  return r;
}

// store through the global address space: generic (flat) stores would also
// hold up the wave's next wait for LDS results
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Wave-wide max / min with all 64 lanes active, returned in a scalar
// register: DPP exchanges inside each row of 16 lanes (swap neighbours, swap
// pairs, mirror in 8, mirror in 16), then the four row results are read out.
template <bool MAX>
__device__ __forceinline__ unsigned wave_ext_u32(unsigned v) {
  auto pick = [](unsigned x, unsigned y) { return MAX ? (x > y ? x : y) : (x < y ? x : y); };
  v = pick(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));
  v = pick(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));
  v = pick(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));
  v = pick(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return pick(pick(r0, r1), pick(r2, r3));
}

__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xFFFFFFFFll));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)b >> 32));
  return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}
__device__ __forceinline__ unsigned uniform(unsigned v) { return (unsigned)__builtin_amdgcn_readfirstlane((int)v); }
// value of v in lane l (l wave-uniform), in a scalar register
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xFFFFFFFFll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), l);
  return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}
__device__ __forceinline__ u64 uniform(u64 v) {
  return ((u64)uniform((unsigned)(v >> 32)) << 32) | uniform((unsigned)(v & 0xFFFFFFFFull));
}

// One row of a register block as a vector: a wave-uniform index selects an
// element with one indexed register move (no branch over the columns).
template <typename T, int N>
struct RegRow {
  typedef T type __attribute__((ext_vector_type(N)));
};

// ------------------------------------------------------- small Cholesky ----
// Leaf Cholesky A = L L^T with X = L^{-1} built in the same sweep (forward
// substitution of L X = I, one rank-1 step per column of L), the
// whole n x n block (n <= NMAX) in registers.  Thread t owns rows
// a = (t & 63) + 64 i and columns b = (t >> 6) + CG j, like the skeleton
// kernel below.  Step j: column j of A and row j of X go to LDS (double
// buffered, so one barrier per step); every thread scales them by
// 1 / sqrt(A(j, j)), subtracts l l^T from its trailing entries and
// l X(j, :) from its rows of X, and the owners store column j of L and
// row j of X.  A non-positive pivot sets status bit 1 and continues with 1.
template <typename T, int NMAX, int NT>
__global__ __launch_bounds__(NT) void potrf_kernel(const PotrfDesc<T>* __restrict__ descs, int* status) {
  constexpr int RI = NMAX / 64, CG = NT / 64, CJ = NMAX / CG;
  static_assert(RI * 64 == NMAX && CJ * CG == NMAX, "square register block");
  typedef typename RegRow<T, CJ>::type row_t;
  __shared__ T s_col[2][NMAX];
  __shared__ __align__(16) T s_xr[2][CG][CJ];
  __shared__ T s_rinv[NMAX];
  const PotrfDesc<T> d = descs[blockIdx.x];
  const int n = d.n, t = threadIdx.x, lane = t & 63;
  const int g = (int)uniform((unsigned)(t >> 6));
  const bool inv = d.Inv != nullptr;
  row_t e[RI], x[RI];
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int jj = 0; jj < CJ; ++jj) {
      const int a = lane + 64 * i, b = g + CG * jj;
      e[i][jj] = (a < n && b < n && a >= b) ? d.A[a + (size_t)b * d.lda] : (T)0;
      x[i][jj] = (a == b) ? (T)1 : (T)0;
    }
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    const int p = j & 1, gj = j % CG, jc = j / CG, lj = j & 63, ir = j >> 6;
    if (g == gj) {
#pragma unroll
      for (int i = 0; i < RI; ++i) s_col[p][lane + 64 * i] = e[i][jc];
    }
    if (inv) {
#pragma unroll
      for (int i = 0; i < RI; ++i)
        if (i == ir) {
          if (lane == lj) {
#pragma unroll
            for (int jj = 0; jj < CJ; ++jj) s_xr[p][g][jj] = x[i][jj];
          }
        }
    }
    __syncthreads();
    T djj = uniform(s_col[p][j]);
    if (!(djj > (T)0)) {
      bad = true;
      djj = (T)1;
    }
    const T ljj = sqrt(djj);
    const T rinv = (T)1 / ljj;
    // loads first, then selects (a conditional load per column would
    // serialise the LDS round trips)
    T la[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int a = lane + 64 * i;
      const T v = s_col[p][a];
      la[i] = a > j ? v * rinv : (T)0;
    }
    row_t lb;
#pragma unroll
    for (int jj = 0; jj < CJ; ++jj) lb[jj] = s_col[p][g + CG * jj];
#pragma unroll
    for (int jj = 0; jj < CJ; ++jj) lb[jj] = (g + CG * jj) > j ? lb[jj] * rinv : (T)0;
#pragma unroll
    for (int i = 0; i < RI; ++i) e[i] -= la[i] * lb;
    if (g == gj) {
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        const int a = lane + 64 * i;
        const T v = e[i][jc];
        e[i][jc] = a == j ? ljj : (a > j ? la[i] : v);
      }
    }
    if (inv) {
      // row j of X is final once scaled by rinv; it stays unscaled in
      // registers (no later step changes it) and is scaled at the end
      row_t xj;
#pragma unroll
      for (int jj = 0; jj < CJ; ++jj) xj[jj] = s_xr[p][g][jj] * rinv;
#pragma unroll
      for (int i = 0; i < RI; ++i) x[i] -= la[i] * xj;
      if (t == 0) s_rinv[j] = rinv;
    }
  }
  __syncthreads();
  if (bad && t == 0) atomicOr(status, 1);
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int jj = 0; jj < CJ; ++jj) {
      const int a = lane + 64 * i, b = g + CG * jj;
      if (a >= n || b >= n) continue;
      if (a >= b) d.A[a + (size_t)b * d.lda] = e[i][jj];
      if (inv) d.Inv[a + (size_t)b * d.ldi] = a >= b ? x[i][jj] * s_rinv[a] : (T)0;
    }
}

// Blocked leaf Cholesky: the same A = L L^T and X = L^{-1} by 16-column
// blocks, one 256-thread workgroup per matrix, A and X in LDS
// (column-major, one element of padding per column).  For block k:
//  - wave 0 factors the 16 x 16 diagonal block D in registers (lane r holds
//    row r; the entries of the column being eliminated reach the other lanes
//    by lane reads, so no barrier) and forms D^{-1} in the same sweep;
//  - all waves, on 16 x 16 x 4 MFMA tiles: the panel below becomes
//    L_ik = A_ik D^{-T}, row block k of X becomes D^{-1} X_k;
//  - then the trailing lower blocks take A_ij -= L_ik L_jk^T and the later
//    row blocks of X take X_i -= L_ik X_k (block forward substitution of
//    L X = I).
// The next diagonal block is updated and factored by wave 0 while the other
// waves finish the trailing update (look-ahead), so each block of 16 columns
// costs two barriers instead of sixteen.  Rows and columns beyond n are the
// identity.  A non-positive pivot sets status bit 1 and continues with 1.
constexpr int kPotrfNB = 16;
// 1 / sqrt(v) for v > 0: the hardware estimate, then Newton steps
// y <- y (3 - v y^2) / 2 (one for float32, three for float64, each about
// doubling the correct bits of the estimate)
__device__ __forceinline__ float rsqrt_nr(float v) {
  const float y = __builtin_amdgcn_rsqf(v);
  return y * (1.5f - 0.5f * v * y * y);
}
__device__ __forceinline__ double rsqrt_nr(double v) {
  double y = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int i = 0; i < 3; ++i) y = y * (1.5 - 0.5 * v * y * y);
  return y;
}
template <typename T, int NMAX>
constexpr size_t potrf_blk_lds() {
  return sizeof(T) * (2 * (size_t)NMAX * (NMAX + 1) + kPotrfNB * (kPotrfNB + 1));
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void potrf_blk_kernel(const PotrfDesc<T>* __restrict__ descs, int* status) {
  constexpr int NB = kPotrfNB, LD = NMAX + 1, DL = NB + 1;
  typedef typename Mfma<T>::v4 v4;
  extern __shared__ __align__(16) char smem[];
  T* S = reinterpret_cast<T*>(smem);            // A, then L (lower part)
  T* X = S + (size_t)NMAX * LD;                  // X = L^{-1}
  T* Di = X + (size_t)NMAX * LD;                 // D^{-1} of the current block, ld DL
  const PotrfDesc<T> d = descs[blockIdx.x];
  const int n = d.n, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nbk = (n + NB - 1) / NB, np = nbk * NB;
  const bool inv = d.Inv != nullptr;
  // thread t takes rows t & 63 (+ 64) of columns t >> 6, + 4, ...: a batch
  // of independent loads in flight before the LDS stores
  {
    constexpr int RB = NMAX / 64, CB = 8;
    const int r0 = t & 63, cg = t >> 6;
    for (int cb = 0; cb < np; cb += 4 * CB) {
      T v[RB][CB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int r = r0 + 64 * i, c = cb + cg + 4 * j;
          v[i][j] = r == c ? (T)1 : (T)0;
          if (r < n && c < n && r >= c) v[i][j] = d.A[r + (size_t)c * d.lda];
          else if (r < n && c < n) v[i][j] = 0;
        }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int r = r0 + 64 * i, c = cb + cg + 4 * j;
          if (r < np && c < np) {
            S[r + c * LD] = v[i][j];
            X[r + c * LD] = r == c ? (T)1 : (T)0;
          }
        }
    }
  }
  __syncthreads();
  bool bad = false;
  // C(16 x 16) = P(16 x 16) Q(16 x 16) on one wave: P(i, q) = p(i, q),
  // Q(q, j) = qf(q, j) read from LDS; lane (li, lk) gets C(row(lk, v), li)
  auto tile = [&](auto p, auto qf) {
    v4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
      const int q = 4 * k4 + lk;
      acc = Mfma<T>::run(p(li, q), qf(q, li), acc);
    }
    return acc;
  };
  // wave 0: factor diagonal block k in registers, D^{-1} to Di.  Lane
  // r + 16 g holds row r, columns g, g + 4, g + 8, g + 12 of D and of D^{-1};
  // a step reads the entries it needs from other lanes by shuffles
  auto diag = [&](int k) {
    const int k0 = k * NB, r = lane & 15, g = lane >> 4;
    T a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = g + 4 * q;
      a[q] = c <= r ? S[(k0 + r) + (k0 + c) * LD] : (T)0;
      x[q] = r == c ? (T)1 : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int gj = j & 3, qj = j >> 2;   // column j sits in lanes (., gj), register qj
      T piv = lane_value(a[qj], j + 16 * gj);
      if (!(piv > (T)0)) {
        bad = true;
        piv = (T)1;
      }
      const T colv = __shfl(a[qj], r + 16 * gj);        // D(r, j), unscaled
      T lc[4], xj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        lc[q] = __shfl(a[qj], (g + 4 * q) + 16 * gj);    // D(c, j) for this lane's columns c
        xj[q] = __shfl(x[q], j + 16 * g);                // row j of D^{-1}, unscaled
      }
      const T rinv = rsqrt_nr(piv), ljj = piv * rinv;
      const T l = r > j ? colv * rinv : (T)0;           // L(r, j)
      if (g == gj) a[qj] = r == j ? ljj : l;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = g + 4 * q;
        if (c > j && r >= c) a[q] -= l * (lc[q] * rinv);
        const T xs = xj[q] * rinv;                       // row j of D^{-1} is final once scaled
        x[q] = r == j ? xs : x[q] - l * xs;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = g + 4 * q;
      if (c <= r) S[(k0 + r) + (k0 + c) * LD] = a[q];
      Di[r + c * DL] = x[q];
    }
  };
  if (wave == 0) diag(0);
  __syncthreads();
  // look-ahead: in the trailing update of block k, wave 0 takes the next
  // diagonal tile first and factors it while the other waves finish the
  // remaining tiles, so the serial diagonal work overlaps the update
  for (int k = 0; k < nbk; ++k) {
    const int k0 = k * NB;
    // panel L_ik = A_ik D^{-T} (i > k) and row block k of X: D^{-1} X_k
    {
      const int npan = nbk - 1 - k, ntile = npan + (inv ? k + 1 : 0);
      for (int q = wave; q < ntile; q += 4) {
        if (q < npan) {
          const int r0 = (k + 1 + q) * NB;
          const v4 c = tile([&](int i, int kk) { return S[(r0 + i) + (k0 + kk) * LD]; },
                            [&](int kk, int j) { return Di[j + kk * DL]; });
#pragma unroll
          for (int v = 0; v < 4; ++v) S[(r0 + Mfma<T>::row(lk, v)) + (k0 + li) * LD] = c[v];
        } else {
          const int c0 = (q - npan) * NB;
          const v4 c = tile([&](int i, int kk) { return Di[i + kk * DL]; },
                            [&](int kk, int j) { return X[(k0 + kk) + (c0 + j) * LD]; });
#pragma unroll
          for (int v = 0; v < 4; ++v) X[(k0 + Mfma<T>::row(lk, v)) + (c0 + li) * LD] = c[v];
        }
      }
    }
    __syncthreads();
    // trailing: A_ij -= L_ik L_jk^T (k < j <= i), X_i -= L_ik X_k (i > k);
    // tile 0 is the next diagonal block (wave 0), the others go to waves 1-3
    {
      const int m = nbk - 1 - k, ntri = m * (m + 1) / 2, ntile = ntri + (inv ? m * (k + 1) : 0);
      auto trail = [&](int q) {
        if (q < ntri) {
          int ib = 0;
          while ((ib + 1) * (ib + 2) / 2 <= q) ++ib;
          const int jb = q - ib * (ib + 1) / 2;
          const int r0 = (k + 1 + ib) * NB, c0 = (k + 1 + jb) * NB;
          const v4 c = tile([&](int i, int kk) { return S[(r0 + i) + (k0 + kk) * LD]; },
                            [&](int kk, int j) { return S[(c0 + j) + (k0 + kk) * LD]; });
#pragma unroll
          for (int v = 0; v < 4; ++v) S[(r0 + Mfma<T>::row(lk, v)) + (c0 + li) * LD] -= c[v];
        } else {
          const int qq = q - ntri, ib = qq / (k + 1), cb = qq % (k + 1);
          const int r0 = (k + 1 + ib) * NB, c0 = cb * NB;
          const v4 c = tile([&](int i, int kk) { return S[(r0 + i) + (k0 + kk) * LD]; },
                            [&](int kk, int j) { return X[(k0 + kk) + (c0 + j) * LD]; });
#pragma unroll
          for (int v = 0; v < 4; ++v) X[(r0 + Mfma<T>::row(lk, v)) + (c0 + li) * LD] -= c[v];
        }
      };
      if (wave == 0) {
        if (m > 0) {
          trail(0);
          diag(k + 1);   // LDS operations of one wave complete in order
        }
      } else {
        for (int q = wave; q < ntile; q += 3) trail(q);
      }
    }
    __syncthreads();
  }
  if (bad && t == 0) atomicOr(status, 1);
  {
    const int r0 = t & 63, cg = t >> 6;
    for (int c = cg; c < n; c += 4)
#pragma unroll
      for (int i = 0; i < NMAX / 64; ++i) {
        const int r = r0 + 64 * i;
        if (r >= n) continue;
        if (r >= c) d.A[r + (size_t)c * d.lda] = S[r + c * LD];
        if (inv) d.Inv[r + (size_t)c * d.ldi] = r >= c ? X[r + c * LD] : (T)0;
      }
  }
}

// Thread t owns rows a = (t & 63) + 64 i (i < RI) and columns
// b = (t >> 6) + CG j (j < CJ) of the block, CG = NT / 64 column groups, so
// a column belongs to one wave and its liveness is wave-uniform.
// Positions are (column << 16) | row.
template <typename T, int RI, int CJ, bool FULL, int NT>
__global__ __launch_bounds__(NT) void skreg_kernel(const SkRegDesc<T>* __restrict__ descs, double eps,
                                                     int adaptive, int* status) {
  constexpr int CG = NT / 64, MR = RI * 64, MC = CJ * CG;
  static_assert(RI * CJ <= 128 && MR < 65536 && MC < 65536, "register block too large");
  typedef typename RegRow<T, CJ>::type row_t;
  constexpr unsigned kMag = sizeof(T) == 4 ? 0x7FFFFF80u : 0x7FFFFFFFu;
  __shared__ T s_cc[2][CG][MR];                 // candidate column of each wave
  __shared__ __align__(16) T s_wrow[FULL ? CG : 1][CJ];   // pivot row, per wave
  __shared__ u64 s_key[3];                      // block-wide max key of a step (three in turn)
  __shared__ char s_inI[FULL ? MR : 1];
  __shared__ char s_inJ[FULL ? MC : 1];
  __shared__ short s_rstep[FULL ? 1 : MR];
  __shared__ short s_cstep[FULL ? 1 : MC];
  const SkRegDesc<T> d = descs[blockIdx.x];
  const int t = threadIdx.x, lane = t & 63;
  const int g = (int)uniform((unsigned)(t >> 6));
  const int M = FULL ? d.nr : d.nI, N = FULL ? d.nc : d.nJ;
  // B_hat mode: a pivot column is zeroed in e once its step is done (so the
  // update leaves it alone) and kept in m: the multipliers in rows that were
  // live, the U entries in the others.  The search still masks finished
  // columns: a multiplier that is not finite turns a zeroed entry into NaN
  // (NaN times 0), and such a column must not be chosen twice.
  row_t e[RI], m[FULL ? 1 : RI];
  unsigned rl = 0, cl = 0, inI = 0, inJ = 0;
#pragma unroll
  for (int i = 0; i < RI; ++i)
    if (lane + 64 * i < M) rl |= 1u << i;
#pragma unroll
  for (int j = 0; j < CJ; ++j)
    if (g + CG * j < N) cl |= 1u << j;
  cl = uniform(cl);
  if (M > 0 && N > 0) {
    // front offsets first, then every element load at once: indices past
    // the block are clamped to its last row / column and the value dropped
    int ro[RI];
    size_t co[CJ];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int a = min(lane + 64 * i, M - 1);
      ro[i] = FULL ? d.r0 + a : gload(d.I + a);
    }
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int b = min(g + CG * j, N - 1);
      co[j] = (size_t)(FULL ? d.c0 + b : gload(d.J + b)) * (size_t)d.ld;
    }
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const T v = gload(d.F + ro[i] + co[j]);
        e[i][j] = (((rl >> i) & 1u) && ((cl >> j) & 1u)) ? v : (T)0;
      }
  } else {
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) e[i][j] = 0;
  }
  if (FULL) {
    for (int a = t; a < MR; a += NT) s_inI[a] = 0;
    for (int b = t; b < MC; b += NT) s_inJ[b] = 0;
    __syncthreads();
    for (int k = t; k < d.nI; k += NT) s_inI[d.I[k] - d.r0] = 1;
    for (int k = t; k < d.nJ; k += NT) s_inJ[d.J[k] - d.c0] = 1;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RI; ++i) if (s_inI[lane + 64 * i]) inI |= 1u << i;
#pragma unroll
    for (int j = 0; j < CJ; ++j) if (s_inJ[g + CG * j]) inJ |= 1u << j;
    inJ = uniform(inJ);
  } else {
    for (int a = t; a < MR; a += NT) s_rstep[a] = -1;
    for (int b = t; b < MC; b += NT) s_cstep[b] = -1;
  }
  if (t < 3) s_key[t] = 0ull;
  __syncthreads();
  int kb = 0;
  const T stop_rel = (T)fmax(eps, (double)noise_rel<T>());
  int r = 0, r1 = -1;
  T u11 = 0;
  int par = 0;
  // Phase 1 searches I x J (whole-block mode) or all of B_hat; phase 2 (the
  // adaptive phase) the whole residual block.  Empty BDLR sets start in
  // phase 2, or stop at rank 0 without it.  Each pivot step: search the
  // registers; every wave writes its best key and the column holding it to
  // LDS (two buffers, alternating by step); one barrier; every wave takes the
  // block-wide max key, reads the pivot column from the winner's buffer and
  // the pivot row of its own columns from the lane that holds it; then the
  // rank-1 update.  A buffer is written again two steps later, after a
  // barrier that every reader of it has passed, so one barrier per step
  // suffices.  The inner loop has a single latch, which keeps the register
  // block in place.
  const int last = FULL && adaptive ? 2 : 1;
  int phase = (FULL && !(d.nI > 0 && d.nJ > 0)) ? 2 : 1;
  bool capped = false;
  T spiv = 0;                     // the last pivot taken or refused
  for (; phase <= last && !capped; ++phase) {
    const bool restricted = FULL && phase == 1;
    // adaptive 2: phase 2 searches the sampled cross only, rows I in every
    // column and every row in the columns J
    const bool cross = FULL && phase == 2 && adaptive == 2;
    for (;;) {
      const unsigned rsel = restricted ? (rl & inI) : rl;
      const unsigned csel = restricted ? (cl & inJ) : cl;
      unsigned rm[RI], rmi[RI];
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        rm[i] = ((rsel >> i) & 1u) ? kMag : 0u;
        rmi[i] = cross ? (((rsel & inI) >> i) & 1u ? kMag : 0u) : rm[i];
      }
      // thread-local best in (j, i) order, which is the position order; wave
      // winner: largest magnitude, then earliest (j, i), then lowest lane
      unsigned q, l, wl;
      if constexpr (sizeof(T) == 4) {
        // one word per element: magnitude bits 7..30, then 127 - (j RI + i)
        // (finished columns are skipped: csel is uniform in the wave)
        unsigned bk = 0;
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
          if (!((csel >> j) & 1u)) continue;
          const bool cj = ((inJ >> j) & 1u) != 0;
#pragma unroll
          for (int i = 0; i < RI; ++i) {
            const unsigned w = (__float_as_uint(e[i][j]) & (cj ? rm[i] : rmi[i])) | (unsigned)(127 - (j * RI + i));
            bk = w > bk ? w : bk;
          }
        }
        const unsigned m = wave_ext_u32<true>(bk);
        wl = (unsigned)(__ffsll((unsigned long long)__ballot(bk == m)) - 1);
        q = m >> 7;
        l = 127u - (m & 127u);
      } else {
        unsigned bq = 0, bl = 0;
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
          if (!((csel >> j) & 1u)) continue;
          const bool cj = ((inJ >> j) & 1u) != 0;
#pragma unroll
          for (int i = 0; i < RI; ++i) {
            const unsigned x = (unsigned)((u64)__double_as_longlong(e[i][j]) >> 32) & (cj ? rm[i] : rmi[i]);
            if (x > bq) { bq = x; bl = (unsigned)(j * RI + i); }
          }
        }
        q = wave_ext_u32<true>(bq);
        const unsigned m = wave_ext_u32<false>(bq == q ? (bl << 6) | (unsigned)lane : 0xFFFFFFFFu);
        l = m >> 6;
        wl = m & 63u;
      }
      // the wave's candidate (its best element) goes to LDS with the column
      // that holds it, so the winner's column is there after the one barrier
      const unsigned jw = l / RI, iw = l - jw * RI;
      const int cur = par;
      par ^= 1;
      if (q) {
#pragma unroll
        for (int i = 0; i < RI; ++i) s_cc[cur][g][lane + 64 * i] = e[i][jw];
      }
      // the block-wide maximum forms in LDS (atomic max); the slot of the
      // next step was last read two barriers ago and is cleared now
      if (lane == 0 && q) {
        const unsigned pos = (((unsigned)g + CG * jw) << 16) | (wl + 64u * iw);
        atomicMax(&s_key[kb], (((u64)q) << 32) | (u64)(0xFFFFFFFFu - pos));
      }
      if (t == 0) s_key[kb == 2 ? 0 : kb + 1] = 0ull;
      __syncthreads();
      u64 K = uniform(s_key[kb]);
      kb = kb == 2 ? 0 : kb + 1;
      if (K == 0ull) break;
      const unsigned pos = 0xFFFFFFFFu - (unsigned)(K & 0xFFFFFFFFull);
      const int as = (int)(pos & 0xFFFFu), bs = (int)(pos >> 16);
      const int ia = as >> 6, la = as & 63, gb = bs % CG, jb = bs / CG;
      const T* cc = s_cc[cur][gb];
      const T piv = uniform(cc[as]);
      T c[RI];
#pragma unroll
      for (int i = 0; i < RI; ++i) c[i] = cc[lane + 64 * i];
      if (u11 == (T)0) u11 = fabs(piv);
      // below the stopping ratio, or not finite (Inf or NaN: the front broke
      // down, flagged after the loop; a separate exit here would push the
      // register block out to scratch)
      spiv = piv;
      if (!(fabs(piv) >= stop_rel * u11 && fabs(piv) <= std::numeric_limits<T>::max())) break;
      if (r >= d.cap) {
        if (t == 0) atomicOr(status, 2);
        capped = true;
        break;
      }
      const T rpiv = (T)1 / piv;
      if (FULL && t == 0) {
        gstore(d.piv_r + r, d.r0 + as);
        gstore(d.piv_c + r, d.c0 + bs);
      }
      if (FULL) {
        T* Uc = d.U + (size_t)r * d.ldu;
        for (int a = t; a < M; a += NT) gstore(Uc + a, phase == 1 ? cc[a] / piv : cc[a]);
      }
      // multipliers: whole-block mode updates every row (the pivot row and
      // column become zero up to rounding); the LU of B_hat updates live rows
      // other than the pivot row, then moves its pivot column to m (the
      // multipliers l = e / piv in the rows that were live) and zeroes it
      T li[RI];
      unsigned upd = 0;
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        const bool w = FULL || (((rl >> i) & 1u) && lane + 64 * i != as);
        li[i] = w ? c[i] * rpiv : (T)0;
        if (w) upd |= 1u << i;
      }
      if constexpr (FULL) {
        // whole-block mode is bound by the vector ALU, so the pivot row of
        // the wave's columns goes through a per-wave LDS row: written by the
        // lane that holds it and read back by the same wave (LDS operations
        // of a wave complete in order, so no barrier)
#pragma unroll
        for (int i0 = 0; i0 < RI; ++i0)
          if (i0 == ia) {
            if (lane == la) {
#pragma unroll
              for (int j = 0; j < CJ; ++j) s_wrow[g][j] = e[i0][j];
            }
          }
        __builtin_amdgcn_wave_barrier();
        // lane j stores the wave's column g + CG j (zero in dead columns,
        // which hold rounding residue)
        if (lane < CJ && g + CG * lane < N) {
          const T vv = ((cl >> lane) & 1u) ? s_wrow[g][lane] : (T)0;
          gstore(d.V + (size_t)r * d.ldv + g + CG * lane, phase == 1 ? vv : vv / piv);
        }
        // the update in two halves of the row, which keeps FP64 blocks
        // within the register budget of 1024 threads
        constexpr int CH = CJ / 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          T u[CH];
#pragma unroll
          for (int j = 0; j < CH; ++j) u[j] = s_wrow[g][h * CH + j];
#pragma unroll
          for (int i = 0; i < RI; ++i)
#pragma unroll
            for (int j = 0; j < CH; ++j) e[i][h * CH + j] -= li[i] * u[j];
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // B_hat mode is bound by the latency of a step: the pivot row of the
        // wave's columns is read from the lane that holds it into scalar
        // registers, the code repeated per register row so the row index is
        // static.  Dead columns are zero, so they take no update.
#pragma unroll
        for (int i0 = 0; i0 < RI; ++i0)
          if (i0 == ia) {
            row_t u;
#pragma unroll
            for (int j = 0; j < CJ; ++j) u[j] = lane_value(e[i0][j], la);
#pragma unroll
            for (int i = 0; i < RI; ++i) e[i] -= li[i] * u;
          }
      }
      if (!FULL) {
        if (g == gb) {
#pragma unroll
          for (int i = 0; i < RI; ++i) {
            const T v = e[i][jb];
            m[i][jb] = ((upd >> i) & 1u) ? li[i] : v;
            e[i][jb] = (T)0;
          }
        }
        if (t == 0) { s_rstep[as] = (short)r; s_cstep[bs] = (short)r; }
      }
      if (lane == la) rl &= ~(1u << ia);
      if (g == gb) cl &= ~(1u << jb);
      ++r;
    }
    if (!(fabs(spiv) <= std::numeric_limits<T>::max())) {   // stopped at a pivot that is not finite
      if (t == 0) atomicOr(status, 16);
      capped = true;
    }
    if (phase == 1 && !capped && last == 2) r1 = r;
  }
  if (r1 < 0) r1 = r;
  if (t == 0) {
    *d.rank1 = FULL ? r1 : r;
    if (d.rank) *d.rank = r;
    *d.u11 = (double)u11;
  }
  if (!FULL) {
    __syncthreads();
    // pivot positions in the front, by step
    for (int a = t; a < M; a += NT)
      if (s_rstep[a] >= 0) d.piv_r[s_rstep[a]] = d.I[a];
    for (int b = t; b < N; b += NT)
      if (s_cstep[b] >= 0) d.piv_c[s_cstep[b]] = d.J[b];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int a = lane + 64 * i;
      if (a >= M) continue;
      const int s = s_rstep[a];
      if (s < 0) continue;
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const int b = g + CG * j;
        if (b >= N) continue;
        const int c = s_cstep[b];
        if (c >= 0) d.M[s + (size_t)c * d.ldm] = m[i][j];
      }
    }
  }
}

// ------------------------------------- skeleton factors C~ and R~^T -------
// Each row position (lane) owns one row i of C~ (x U_r = B(i, J_r), U_r
// upper) or one column a of R~^T (L_r y = B(I_r, a), L_r unit lower).  The
// solve runs over column blocks of KB: the contributions of all earlier
// solved values (LDS) to the block's right-hand sides are split over the
// workgroup's waves by solved index (wave w takes t = w, w + NW, ...), each
// with KB independent FMAs per value; wave 0 adds the other waves' partial
// sums to the right-hand sides and solves the triangular block itself in
// order.
template <typename T>
__global__ __launch_bounds__(kSkelFacThreads) void skelfac_kernel(const SkelFacDesc<T>* __restrict__ descs,
                                                                  int ndesc, int rmax) {
  constexpr int KB = kSkelFacBlock, W = kSkelFacRows, NW = kSkelFacThreads / 64;
  extern __shared__ __align__(16) char smem[];
  T* X = reinterpret_cast<T*>(smem);              // rmax x W solved values
  T* S = X + (size_t)rmax * W;                    // rmax x KB factor block
  T* P = S + (size_t)rmax * KB;                   // (NW - 1) x KB x W partial sums
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (descs[mid].wg0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1; }
  const SkelFacDesc<T> d = descs[lo];
  const int r = *d.rank;
  const int local = (int)blockIdx.x - d.wg0, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool upart = local < d.wgU;
  const int row = (upart ? local : local - d.wgU) * W + lane;
  const bool valid = row < (upart ? d.nr : d.nc);
  for (int k0 = 0; k0 < r; k0 += KB) {
    const int nb = min(KB, r - k0), tn = k0 + nb;
    __syncthreads();                              // earlier readers of S and P are done
    for (int q = threadIdx.x; q < tn * KB; q += kSkelFacThreads) {
      const int t = q / KB, c = q - (q / KB) * KB;
      T v = 0;
      if (c < nb) v = upart ? d.M[t + (size_t)(k0 + c) * d.ldm] : d.M[(k0 + c) + (size_t)t * d.ldm];
      S[q] = v;
    }
    T acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      T v = 0;
      if (wave == 0 && valid && c < nb)
        v = upart ? d.F[(d.r0 + row) + (size_t)d.piv_c[k0 + c] * d.ld]
                  : d.FR[d.piv_r[k0 + c] + (size_t)(d.c0 + row) * d.ldr];
      acc[c] = v;
    }
    __syncthreads();
    for (int t = wave; t < k0; t += NW) {
      const T xt = X[(size_t)t * W + lane];
      const T* st = S + t * KB;
#pragma unroll
      for (int c = 0; c < KB; ++c) acc[c] -= xt * st[c];
    }
    if (wave > 0) {
#pragma unroll
      for (int c = 0; c < KB; ++c) P[((size_t)(wave - 1) * KB + c) * W + lane] = acc[c];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int w2 = 0; w2 < NW - 1; ++w2)
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[c] += P[((size_t)w2 * KB + c) * W + lane];
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        if (c < nb) {
#pragma unroll
          for (int cp = 0; cp < c; ++cp) acc[c] -= acc[cp] * S[(k0 + cp) * KB + c];
          if (upart) acc[c] = acc[c] / S[(k0 + c) * KB + c];
          X[(size_t)(k0 + c) * W + lane] = acc[c];
          if (valid) {
            if (upart) d.U[(size_t)(k0 + c) * d.ldu + row] = acc[c];
            else d.V[(size_t)(k0 + c) * d.ldv + row] = acc[c];
          }
        }
      }
    }
  }
}

// -------------------------------- skeleton, phase 2 (full block residual) --
template <typename T>
__global__ __launch_bounds__(1024) void phase2_kernel(const Phase2Desc<T>* __restrict__ descs, double eps,
                                                      int* status) {
  extern __shared__ __align__(16) char smem[];
  __shared__ u64 s_red[16];
  const Phase2Desc<T> d = descs[blockIdx.x];
  const int nr = d.nr, nc = d.nc, tid = threadIdx.x, nt = blockDim.x;
  char* lr = smem;
  char* lc = smem + nr;
  const int r1 = *d.rank1;
  double u11 = *d.u11;
  for (int a = tid; a < nr; a += nt) lr[a] = 1;
  for (int b = tid; b < nc; b += nt) lc[b] = 1;
  __syncthreads();
  for (int s = tid; s < r1; s += nt) { lr[d.piv_r[s] - d.r0] = 0; lc[d.piv_c[s] - d.c0] = 0; }
  __syncthreads();
  T* E = d.F + d.r0 + (size_t)d.c0 * d.ld;
  const int ld = d.ld;
  const double stop_rel = fmax(eps, (double)noise_rel<T>());
  int r = r1;
  const int w = tid >> 6, lane = tid & 63, nw = nt >> 6;
  bool pending = false;   // the last appended (U, V) column is still to be subtracted
  for (;;) {
    // one pass: apply the pending rank-1 update, then find the pivot key
    const T* Up = d.U + (size_t)(r - 1) * d.ldu;
    const T* Vp = d.V + (size_t)(r - 1) * d.ldv;
    u64 best = 0;
    for (int b = w; b < nc; b += nw) {
      const T vb = pending ? Vp[b] : (T)0;
      const bool cb = lc[b] != 0;
      T* Eb = E + (size_t)b * ld;
      for (int a = lane; a < nr; a += 64) {
        T x = Eb[a];
        if (pending) {
          x -= Up[a] * vb;
          Eb[a] = x;
        }
        if (cb && lr[a]) {
          const u64 k = make_key(qmag(x), (unsigned)(b * nr + a));
          best = k > best ? k : best;
        }
      }
    }
    const u64 K = block_max_u64(best, s_red);
    if (K == 0ull) break;
    const unsigned idx = 0xFFFFFFFFu - (unsigned)(K & 0xFFFFFFFFull);
    const int as = (int)(idx % (unsigned)nr), bs = (int)(idx / (unsigned)nr);
    const T piv = E[as + (size_t)bs * ld];
    if (!(fabs((double)piv) <= (double)std::numeric_limits<T>::max())) {
      if (tid == 0) atomicOr(status, 16);
      break;
    }
    if (u11 == 0.0) u11 = fabs((double)piv);
    if (fabs((double)piv) < stop_rel * u11) break;
    if (r >= d.cap) {
      if (tid == 0) atomicOr(status, 2);
      break;
    }
    T* Uc = d.U + (size_t)r * d.ldu;
    T* Vc = d.V + (size_t)r * d.ldv;
    for (int a = tid; a < nr; a += nt) Uc[a] = E[a + (size_t)bs * ld];
    for (int b = tid; b < nc; b += nt) Vc[b] = E[as + (size_t)b * ld] / piv;
    __syncthreads();
    if (tid == 0) { lr[as] = 0; lc[bs] = 0; }
    ++r;
    pending = true;
    __syncthreads();
  }
  if (tid == 0) *d.rank = r;
}

// --------------------------- skeleton, phase 2 over several workgroups ----
// Barrier of the workgroups of one block.  Only the published keys and
// candidate columns cross workgroups, and they are written and read with
// agent-scope atomic accesses, which are coherent across the chip by
// themselves; each thread waits for its stores to complete, then thread 0
// arrives on the counter and polls it (bounded).  No cache-wide writeback or
// invalidation is needed, so the slices stay in the caches.  Returns false
// when the poll limit was reached.
template <typename T>
__device__ __forceinline__ void publish(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T fetch(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide maximum of a 64-bit key (every thread active), uniform result,
// one barrier: the wave maxima meet in slot sh[slot] by LDS atomic max
// (slots 0..2 zero before the first call, used in turn by consecutive calls;
// the next slot, last read two calls ago, is cleared here).
__device__ __forceinline__ u64 block_max_key(u64 v, u64* sh, int slot) {
  const unsigned hi = wave_ext_u32<true>((unsigned)(v >> 32));
  const unsigned lo = wave_ext_u32<true>((unsigned)(v >> 32) == hi ? (unsigned)(v & 0xFFFFFFFFull) : 0u);
  const u64 w = ((u64)hi << 32) | lo;
  if ((threadIdx.x & 63) == 0 && w != 0ull) atomicMax(&sh[slot], w);
  if (threadIdx.x == 0) sh[slot == 2 ? 0 : slot + 1] = 0ull;
  __syncthreads();
  return uniform(sh[slot]);
}

// Multi-workgroup phase 2.  Workgroup j owns a slice of wcols columns.  Each
// step it applies the previous pivot's rank-1 update to its slice, finds its
// best key, publishes that key's column, then the key in its slot.  A slot
// holds the key with a tag in bit 63 that flips every second step (slots and
// columns alternate between two buffers by step parity), so a workgroup
// knows every other workgroup has published once all slots of the step's
// buffer carry the step's tag: the polling of the slots is the barrier, and
// it brings the keys along.  Then all pick the same pivot and read its column.
// SLICE_LDS: the workgroup's columns are copied to LDS once (the front keeps
// the phase-1 residual); otherwise they are updated in place in the front.
template <typename T, bool SLICE_LDS>
__global__ __launch_bounds__(kCoopThreads) void phase2_coop_kernel(const Phase2CoopDesc<T>* __restrict__ descs, int ndesc,
                                                          double eps, int* status, long long wait_ticks) {
  extern __shared__ __align__(16) char smem[];
  __shared__ u64 s_red[32];
  __shared__ u64 s_pk[2][1];
  __shared__ int s_pok[2][1];
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].wg0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const Phase2CoopDesc<T> d = descs[lo];
  const int j = (int)blockIdx.x - d.wg0;
  const int nr = d.nr, nwg = d.nwg, tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nwave = nt >> 6;
  const int cb0 = j * d.wcols, w = min(d.wcols, d.nc - cb0);
  T* const Eg = d.F + d.r0 + (size_t)(d.c0 + cb0) * d.ld;
  T* Es;                                           // own columns, leading dimension les
  T* u;                                            // pivot column
  size_t les;
  if (SLICE_LDS) {
    Es = reinterpret_cast<T*>(smem);
    les = nr;
    u = Es + (size_t)nr * d.wcols;
    for (int c = wave; c < w; c += nwave)
      for (int i = lane; i < nr; i += 64) Es[i + (size_t)c * nr] = Eg[i + (size_t)c * d.ld];
  } else {
    Es = Eg;
    les = d.ld;
    u = reinterpret_cast<T*>(smem);
  }
  T* vloc = u + nr;                                // own entries of the new V column
  char* lr = reinterpret_cast<char*>(vloc + d.wcols);
  char* lc = lr + nr;
  if (tid < 3) s_red[tid] = 0ull;
  for (int i = tid; i < nr; i += nt) lr[i] = 1;
  for (int c = tid; c < w; c += nt) lc[c] = 1;
  __syncthreads();
  const int r1 = *d.rank1;
  for (int q = tid; q < r1; q += nt) {
    lr[d.piv_r[q] - d.r0] = 0;
    const int cc = d.piv_c[q] - d.c0 - cb0;
    if (cc >= 0 && cc < w) lc[cc] = 0;
  }
  __syncthreads();
  // live rows of this lane (rows lane + 64 k; nr <= kPhase2CoopMaxRows) as
  // bits, k < 64 in lmask0 and the rest in lmask1
  u64 lmask0 = 0, lmask1 = 0;
  for (int k = 0; k < 128 && lane + 64 * k < nr; ++k)
    if (lr[lane + 64 * k]) {
      if (k < 64) lmask0 |= 1ull << k;
      else lmask1 |= 1ull << (k - 64);
    }
  double u11 = *d.u11;
  const double stop_rel = fmax(eps, (double)noise_rel<T>());
  constexpr u64 kTag = 1ull << 63;
  int r = r1;
  int step = 0, rpar = 0, ppar = 0;
  bool pending = false;
  for (;; ++step) {
    const int par = step & 1;
    const u64 tag = ((step >> 1) & 1) ? kTag : 0ull;
    // update with the pending pivot (if any) and search own columns, rows in
    // groups of four independent load / update / store chains; the thread's
    // best is (truncated magnitude, position), visited in ascending position
    unsigned bq = 0, bidx = 0;
    auto consider = [&](T x, int i, unsigned base) {
      const int k = i >> 6;
      const unsigned q = (((k < 64 ? lmask0 : lmask1) >> (k & 63)) & 1ull) ? qmag(x) : 0u;
      if (q > bq) { bq = q; bidx = base + (unsigned)i; }
    };
    for (int c = wave; c < w; c += nwave) {
      const T v = pending ? vloc[c] : (T)0;
      const bool cc = lc[c] != 0;
      T* col = Es + (size_t)c * les;
      const unsigned base = (unsigned)(cb0 + c) * (unsigned)nr;
      int i = lane;
      for (; i + 192 < nr; i += 256) {
        T x0 = col[i], x1 = col[i + 64], x2 = col[i + 128], x3 = col[i + 192];
        if (pending) {
          x0 -= u[i] * v;
          x1 -= u[i + 64] * v;
          x2 -= u[i + 128] * v;
          x3 -= u[i + 192] * v;
          col[i] = x0;
          col[i + 64] = x1;
          col[i + 128] = x2;
          col[i + 192] = x3;
        }
        if (cc) {
          consider(x0, i, base);
          consider(x1, i + 64, base);
          consider(x2, i + 128, base);
          consider(x3, i + 192, base);
        }
      }
      for (; i < nr; i += 64) {
        T x = col[i];
        if (pending) {
          x -= u[i] * v;
          col[i] = x;
        }
        if (cc) consider(x, i, base);
      }
    }
    u64 best = make_key(bq, bidx);
    best = block_max_key(best, s_red, rpar);
    rpar = rpar == 2 ? 0 : rpar + 1;
    // publish the best key's column, then (after every thread's stores are
    // done) the tagged key
    if (best != 0ull) {
      const unsigned idx = 0xFFFFFFFFu - (unsigned)(best & 0xFFFFFFFFull);
      const int bc = (int)(idx / (unsigned)nr) - cb0;
      T* cd = d.cand + ((size_t)par * nwg + j) * nr;
      for (int i = tid; i < nr; i += nt) publish(cd + i, Es[i + (size_t)bc * les]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) publish(d.keys + (size_t)par * nwg + j, (unsigned long long)(best | tag));
    // wait for every slot of this buffer to carry this step's tag: wave 0
    // polls (no barrier inside the loop; its exit is wave-uniform), then one
    // barrier hands the key to the other waves
    if (wave == 0) {
      u64 km = 0;
      int ok_all = 0;
      const long long t_wait = wall_clock64();
      for (;;) {
        if (wait_ticks < 0) break;   // host-forced give-up (test hook): no poll at all
        u64 kq = 0;
        bool ok = true;
        for (int q = lane; q < nwg; q += 64) {
          const u64 k = fetch(d.keys + (size_t)par * nwg + q);
          if ((k & kTag) != tag) ok = false;
          const u64 kv = k & ~kTag;
          kq = kv > kq ? kv : kq;
        }
        if (__ballot(!ok) == 0ull) {
          const unsigned khi = wave_ext_u32<true>((unsigned)(kq >> 32));
          const unsigned klo =
              wave_ext_u32<true>((unsigned)(kq >> 32) == khi ? (unsigned)(kq & 0xFFFFFFFFull) : 0u);
          km = ((u64)khi << 32) | klo;
          ok_all = 1;
          break;
        }
        if ((long long)wall_clock64() - t_wait > wait_ticks) break;
        __builtin_amdgcn_s_sleep(1);
      }
      if (lane == 0) {
        s_pk[ppar][0] = km;
        s_pok[ppar][0] = ok_all;
      }
    }
    __syncthreads();
    const bool met = s_pok[ppar][0] != 0;
    const u64 K = uniform(s_pk[ppar][0]);
    ppar ^= 1;
    if (!met) {
      if (tid == 0) atomicOr(status, 8);
      break;
    }
    if (K == 0ull) break;
    const unsigned idx = 0xFFFFFFFFu - (unsigned)(K & 0xFFFFFFFFull);
    const int a = (int)(idx % (unsigned)nr);
    const int b = (int)(idx / (unsigned)nr);
    const int y = b / d.wcols;
    const T* cy = d.cand + ((size_t)par * nwg + y) * nr;
    for (int i = tid; i < nr; i += nt) u[i] = fetch(cy + i);
    __syncthreads();
    const T piv = u[a];
    if (!(fabs((double)piv) <= (double)std::numeric_limits<T>::max())) {   // the same in every workgroup
      if (tid == 0 && j == 0) atomicOr(status, 16);
      break;
    }
    if (u11 == 0.0) u11 = fabs((double)piv);
    if (fabs((double)piv) < stop_rel * u11) break;
    if (r >= d.cap) {
      if (tid == 0 && j == 0) atomicOr(status, 2);
      break;
    }
    for (int c = tid; c < w; c += nt) vloc[c] = Es[a + (size_t)c * les] / piv;
    __syncthreads();
    {   // this workgroup's share of U(:, r), and V(own columns, r)
      const int ch = (nr + nwg - 1) / nwg, i0 = j * ch, i1 = min(nr, i0 + ch);
      for (int i = i0 + tid; i < i1; i += nt) d.U[i + (size_t)r * d.ldu] = u[i];
      for (int c = tid; c < w; c += nt) d.V[(cb0 + c) + (size_t)r * d.ldv] = vloc[c];
    }
    if (tid == 0) {
      lr[a] = 0;
      if (b >= cb0 && b < cb0 + w) lc[b - cb0] = 0;
    }
    if (lane == (a & 63)) {
      const int k = a >> 6;
      if (k < 64) lmask0 &= ~(1ull << k);
      else lmask1 &= ~(1ull << (k - 64));
    }
    ++r;
    pending = true;
    __syncthreads();
  }
  if (tid == 0 && j == 0) *d.rank = r;
}

// ----------------------------------------------------------- extend-add ----
template <typename T>
__global__ __launch_bounds__(256) void extadd_kernel(const ExtAddDesc<T>* __restrict__ descs, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const ExtAddDesc<T>& d = descs[di];
  const int lt = (int)blockIdx.x - d.tile0;
  const int tr = lt % d.tiles_r, tc = lt / d.tiles_r;
  if (tc > tr) return;
  const int nfc = d.nfc;
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int a = tr * kTile + (e & 63), b = tc * kTile + (e >> 6);
    if (a < nfc && b < nfc && a >= b) {
      const T v = d.child[(d.npc + a) + (size_t)(d.npc + b) * d.ldc];
      d.parent[d.relmap[a] + (size_t)d.relmap[b] * d.ldp] += v;
    }
  }
}

// ----------------------------------------------------------------- copy ----
// ----------------------------------------------- sampled extend-add -------
// Entry (a, b) of a child's update (symmetric, so any order of a and b).
template <typename T>
__device__ T child_update(const ChildUpd<T>& c, int a, int b) {
  if (c.dense) {
    const int i = max(a, b), j = min(a, b);
    return c.F[(c.npc + i) + (size_t)(c.npc + j) * c.ld];
  }
  T v = 0;
  int nd = 0;
  for (;;) {   // the cluster-tree node where a and b part, or their leaf
    const FfNode n = c.nodes[nd];
    if (n.left < 0) {
      v = static_cast<const T*>(n.U)[(a - n.off) + (size_t)(b - n.off) * n.size];
      break;
    }
    const FfNode l = c.nodes[n.left], r = c.nodes[n.right];
    const bool al = a < l.off + l.size, bl = b < l.off + l.size;
    if (al == bl) {
      nd = al ? n.left : n.right;
      continue;
    }
    const int ri = (al ? b : a) - r.off, ci = (al ? a : b) - l.off;   // row in the right child, column in the left
    const T* U = static_cast<const T*>(n.U);
    const T* V = static_cast<const T*>(n.V);
    for (int k = 0; k < n.rank; ++k) v += U[ri + (size_t)k * r.size] * V[ci + (size_t)k * l.size];
    break;
  }
  T s = 0;
  for (int k = 0; k < c.rtop; ++k) s += c.Wt[a + (size_t)k * c.nf] * load_op(c.W, b + (size_t)k * c.nf, c.wbf != 0);
  return v - s;
}

// Entry (i, j) of a front that is never assembled (front positions):
// F_bar_p's entry (A's, when i or j is a pivot position) plus every child's
// update at the mapped position.
template <typename T>
__device__ T front_value(const GatherFront<T>& f, int i, int j, const int* __restrict__ rowptr,
                         const int* __restrict__ colind, const double* __restrict__ vals,
                         const int* __restrict__ perm) {
  T v = 0;
  if (i < f.npiv || j < f.npiv) {   // F_bar_p: A's entries in the pivot rows and columns
    const int gi = i < f.npiv ? f.start + i : f.upd[i - f.npiv];
    const int gj = j < f.npiv ? f.start + j : f.upd[j - f.npiv];
    const int row = perm[gi], col = perm[gj];
    int lo = rowptr[row], hi = rowptr[row + 1];
    const int end = hi;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (colind[mid] < col) lo = mid + 1;
      else hi = mid;
    }
    if (lo < end && colind[lo] == col) v = (T)vals[lo];
  }
  for (int c = 0; c < f.nchild; ++c) {
    const ChildUpd<T>& u = f.ch[c];
    const int a = u.inv[i], b = u.inv[j];
    if (a >= 0 && b >= 0) v += child_update(u, a, b);
  }
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const GatherDesc<T>* __restrict__ descs, int ndesc,
                                                     const GatherFront<T>* __restrict__ fronts,
                                                     const int* __restrict__ rowptr, const int* __restrict__ colind,
                                                     const double* __restrict__ vals, const int* __restrict__ perm) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const GatherDesc<T>& d = descs[di];
  const int64_t e = (int64_t)((int)blockIdx.x - d.tile0) * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d.nr * d.nc) return;
  const int rr = (int)(e % d.nr), cc = (int)(e / d.nr);
  const int i = d.rows ? d.rows[rr] : d.r0 + rr;
  const int j = d.cols ? d.cols[cc] : d.c0 + cc;
  d.out[rr + (size_t)cc * d.ldo] = front_value(fronts[d.front], i, j, rowptr, colind, vals, perm);
}

// index of v in the ascending list a[0 .. n), or -1
__device__ __forceinline__ int find_sorted(const int* __restrict__ a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == v) ? lo : -1;
}

template <typename T>
__global__ __launch_bounds__(kCrossThreads) void cross_kernel(const CrossDesc<T>* __restrict__ descs, double eps,
                                                              const int* __restrict__ rowptr,
                                                              const int* __restrict__ colind,
                                                              const double* __restrict__ vals,
                                                              const int* __restrict__ perm, int* status) {
  extern __shared__ __align__(16) char smem[];
  __shared__ u64 s_red[16];
  __shared__ T s_piv;
  __shared__ int s_ci, s_ri;
  const CrossDesc<T> d = descs[blockIdx.x];
  const int nr = d.nr, nc = d.nc, nI = d.nI, nJ = d.nJ, tid = threadIdx.x, nt = blockDim.x;
  char* lr = smem;        // live rows / columns (not yet a pivot's)
  char* lc = smem + nr;
  const int r1 = *d.rank1;
  for (int a = tid; a < nr; a += nt) lr[a] = 1;
  for (int b = tid; b < nc; b += nt) lc[b] = 1;
  __syncthreads();
  for (int s = tid; s < r1; s += nt) {
    lr[d.Il[d.piv_r[s]]] = 0;
    lc[d.Jl[d.piv_c[s]]] = 0;
  }
  __syncthreads();
  T* __restrict__ EJ = d.EJ;
  T* __restrict__ EI = d.EI;
  const int64_t nej = (int64_t)nr * nJ, nei = (int64_t)nI * nc;
  const double stop_rel = fmax(eps, (double)noise_rel<T>());
  double u11 = *d.u11;
  int r = r1;
  // largest live residual entry of the cross (position order on ties); each
  // later search runs in the same pass as the previous pivot's update
  u64 best = 0;
  for (int64_t e = tid; e < nej; e += nt) {
    const int i = (int)(e % nr), j = d.Jl[e / nr];
    if (lr[i] && lc[j]) {
      const u64 k = make_key(qmag(EJ[e]), (unsigned)(j * nr + i));
      best = k > best ? k : best;
    }
  }
  for (int64_t e = tid; e < nei; e += nt) {
    const int i = d.Il[e % nI], j = (int)(e / nI);
    if (lr[i] && lc[j]) {
      const u64 k = make_key(qmag(EI[e]), (unsigned)(j * nr + i));
      best = k > best ? k : best;
    }
  }
  for (;;) {
    const u64 K = block_max_u64(best, s_red);
    if (K == 0ull) break;
    const unsigned idx = 0xFFFFFFFFu - (unsigned)(K & 0xFFFFFFFFull);
    const int is = (int)(idx % (unsigned)nr), js = (int)(idx / (unsigned)nr);
    if (tid == 0) {
      const int ci = find_sorted(d.Jl, nJ, js), ri = find_sorted(d.Il, nI, is);
      s_ci = ci;
      s_ri = ri;
      // every key came from E(:, J) or E(I, :), so one of the two is found
      s_piv = ci >= 0 ? EJ[is + (size_t)ci * nr] : (ri >= 0 ? EI[ri + (size_t)js * nI] : (T)0);
    }
    __syncthreads();
    const int ci = s_ci, ri = s_ri;
    if (ci < 0 && ri < 0) break;
    const T piv = s_piv;
    if (!(fabs((double)piv) <= (double)std::numeric_limits<T>::max())) {
      if (tid == 0) atomicOr(status, 16);
      break;
    }
    if (u11 == 0.0) u11 = fabs((double)piv);
    if (fabs((double)piv) < stop_rel * u11) break;
    if (r >= d.cap) {
      if (tid == 0) atomicOr(status, 2);
      break;
    }
    T* Uc = d.U + (size_t)r * nr;
    T* Vc = d.V + (size_t)r * nc;
    // residual column js into U(:, r), residual row is / piv into V(:, r)
    for (int i = tid; i < nr; i += nt) {
      T v;
      if (ci >= 0) {
        v = EJ[i + (size_t)ci * nr];
      } else {
        v = front_value(*d.front, d.r0 + i, d.c0 + js, rowptr, colind, vals, perm);
        for (int k = 0; k < r; ++k) v -= d.U[i + (size_t)k * nr] * d.V[js + (size_t)k * nc];
      }
      Uc[i] = v;
    }
    for (int j = tid; j < nc; j += nt) {
      T v;
      if (ri >= 0) {
        v = EI[ri + (size_t)j * nI];
      } else {
        v = front_value(*d.front, d.r0 + is, d.c0 + j, rowptr, colind, vals, perm);
        for (int k = 0; k < r; ++k) v -= d.U[is + (size_t)k * nr] * d.V[j + (size_t)k * nc];
      }
      Vc[j] = v / piv;
    }
    if (tid == 0) {
      lr[is] = 0;
      lc[js] = 0;
    }
    ++r;
    __syncthreads();
    // the cross takes the rank-1 update, and the next search reads the new values
    best = 0;
    for (int64_t e = tid; e < nej; e += nt) {
      const int i = (int)(e % nr), j = d.Jl[e / nr];
      const T v = EJ[e] - Uc[i] * Vc[j];
      EJ[e] = v;
      if (lr[i] && lc[j]) {
        const u64 k = make_key(qmag(v), (unsigned)(j * nr + i));
        best = k > best ? k : best;
      }
    }
    for (int64_t e = tid; e < nei; e += nt) {
      const int i = d.Il[e % nI], j = (int)(e / nI);
      const T v = EI[e] - Uc[i] * Vc[j];
      EI[e] = v;
      if (lr[i] && lc[j]) {
        const u64 k = make_key(qmag(v), (unsigned)(j * nr + i));
        best = k > best ? k : best;
      }
    }
  }
  if (tid == 0) *d.rank = r;
}

template <typename T>
__global__ __launch_bounds__(256) void extadd_c_kernel(const ExtAddCDesc<T>* __restrict__ descs, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const ExtAddCDesc<T>& d = descs[di];
  const int lt = (int)blockIdx.x - d.tile0;
  const int tr = lt % d.tiles_r, tc = lt / d.tiles_r;
  if (tc > tr) return;
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int a = tr * kTile + (e & 63), b = tc * kTile + (e >> 6);
    if (a < d.nfc && b < d.nfc && a >= b)   // relmap increases: (a, b) lands in the parent's lower triangle
      d.parent[d.relmap[a] + (size_t)d.relmap[b] * d.ldp] += child_update(d.c, a, b);
  }
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void copy_kernel(const CopyDesc<S, D>* __restrict__ descs, int ndesc) {
  const int di = find_desc_wg(descs, ndesc, (int)blockIdx.x);
  const CopyDesc<S, D>& d = descs[di];
  const int lt = (int)blockIdx.x - d.tile0;
  const int tr = lt % d.tiles_r, tc = lt / d.tiles_r;
  // 256 threads, PER entries each: every load of the tile is issued before
  // the first store (a load used right away would wait before the next)
  constexpr int PER = kTile * kTile / 256;
  S sv[PER];
  D dv[PER];
  const bool acc = d.accumulate != 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * 256;
    const int i = tr * kTile + (e & 63), j = tc * kTile + (e >> 6);
    const bool in = i < d.rows && j < d.cols;
    sv[u] = in ? d.src[i + (size_t)j * d.lds] : (S)0;
    dv[u] = in && acc ? d.dst[i + (size_t)j * d.ldd] : (D)0;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * 256;
    const int i = tr * kTile + (e & 63), j = tc * kTile + (e >> 6);
    if (i < d.rows && j < d.cols) {
      D v = (D)(d.alpha * (double)sv[u]);
      const size_t o = i + (size_t)j * d.ldd;
      if constexpr (sizeof(D) == 4) {
        if (d.bf16 == 2) {
          reinterpret_cast<unsigned short*>(d.dst)[o] = float_to_bf16(v);
          continue;
        }
        if (d.bf16 == 1) v = bf16_to_float(float_to_bf16(v));
      }
      if (acc) v += dv[u];
      d.dst[o] = v;
    }
  }
}

// ------------------------------------------------- SMW capacitance -------
template <typename T>
__global__ __launch_bounds__(256) void cap_kernel(const CapDesc<T>* __restrict__ descs) {
  const CapDesc<T> d = descs[blockIdx.x];
  const int r = d.r, n = 2 * r;
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    d.A[idx] = (double)d.P[i + (size_t)(d.c + j) * d.ldp];
    d.B[idx] = (double)d.P[(r + i) + (size_t)(d.c + j) * d.ldp];
    const double e = i == j ? 1.0 : 0.0;
    d.Kinv[(r + i) + (size_t)j * n] = e;
    d.Kinv[i + (size_t)(r + j) * n] = e;
  }
  for (int idx = threadIdx.x; idx < n * d.c; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    d.Pa[i + (size_t)j * n] = (double)d.P[i + (size_t)j * d.ldp];
  }
}

// In-place inverse of an n x n float64 matrix by Gauss-Jordan elimination
// with partial pivoting (largest |A(i,k)|, lowest i on ties).  Step k swaps
// rows k and p, turns column k into the k-th unit column while the inverse
// builds up in its place, and the recorded row interchanges are undone as
// column interchanges in reverse order at the end.  One workgroup per
// matrix; a zero pivot column sets status bit 4.  Used for n above the
// register kernel's limit.
__global__ __launch_bounds__(1024) void gj_wide_kernel(const InvDesc* __restrict__ descs, int* status) {
  __shared__ double f[kInvMax];
  __shared__ double rowk[kInvMax];
  __shared__ int perm[kInvMax];
  __shared__ double redd[16];
  __shared__ int redi[16];
  const InvDesc d = descs[blockIdx.x];
  const int n = d.n, ld = d.ld, tid = threadIdx.x, nt = blockDim.x;
  double* A = d.A;
  for (int k = 0; k < n; ++k) {
    double mx = 0.0;
    for (int i = k + tid; i < n; i += nt) mx = fmax(mx, fabs(A[i + (size_t)k * ld]));
    const double mxall = block_max(mx, redd);
    int best = INT_MAX;
    for (int i = k + tid; i < n; i += nt)
      if (fabs(A[i + (size_t)k * ld]) == mxall) { best = i; break; }
    int p = block_min(best, redi);
    if (!(mxall > 0.0)) {
      if (tid == 0) atomicOr(status, 4);
      p = k;
    }
    if (tid == 0) perm[k] = p;
    double pv = A[p + (size_t)k * ld];
    if (!(fabs(pv) > 0.0)) pv = 1.0;
    const double inv = 1.0 / pv;
    __syncthreads();   // every thread has read the pivot before rows move
    for (int c = tid; c < n; c += nt) {
      const double vk = A[k + (size_t)c * ld], vp = A[p + (size_t)c * ld];
      const double nk = (c == k ? 1.0 : vp) * inv;   // new row k; A(k,k) becomes 1/pivot
      rowk[c] = nk;
      A[k + (size_t)c * ld] = nk;
      if (p != k) A[p + (size_t)c * ld] = vk;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nt) f[i] = (i == k) ? 0.0 : A[i + (size_t)k * ld];
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += nt) {
      const int i = idx % n, c = idx / n;
      if (i == k) continue;
      double* a = A + i + (size_t)c * ld;
      *a = (c == k ? 0.0 : *a) - f[i] * rowk[c];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < n; i += nt) {
        const double t = A[i + (size_t)k * ld];
        A[i + (size_t)k * ld] = A[i + (size_t)p * ld];
        A[i + (size_t)p * ld] = t;
      }
    __syncthreads();
  }
}

// The same elimination with the whole matrix in registers (n <= RI * 64):
// thread t owns rows a = (t & 63) + 64 i and columns b = (t >> 6) + CG j.
// Rows are not moved.  Step k: the wave owning column k picks the pivot row
// p among the rows not yet used (largest |A(i,k)|, lowest i on ties) and
// puts column k in LDS (barrier); each wave puts its part of row p in LDS
// (barrier); then row p becomes (A(p,:) with 1 at k) / A(p,k) and every other
// row i becomes (A(i,:) with 0 at k) - A(i,k) row p.  With p_k the pivot row
// of step k, the result B gives the inverse as inv(k, p_j) = B(p_k, j), which
// is how it is written back.
template <int RI, int CJ, int NT>
__global__ __launch_bounds__(NT) void gj_kernel(const InvDesc* __restrict__ descs, int* status) {
  constexpr int NMAX = RI * 64, CG = NT / 64;
  static_assert(CJ * CG >= NMAX && RI * CJ <= 64, "register block");
  typedef typename RegRow<double, CJ>::type row_t;
  __shared__ double s_col[2][NMAX];
  __shared__ int s_piv[2];
  __shared__ __align__(16) double s_row[CG][CJ];
  __shared__ short s_rstep[NMAX], s_prow[CJ * CG];
  const InvDesc d = descs[blockIdx.x];
  const int n = d.n, t = threadIdx.x, lane = t & 63;
  const int g = (int)uniform((unsigned)(t >> 6));
  row_t e[RI];
  unsigned rl = 0;
#pragma unroll
  for (int i = 0; i < RI; ++i) {
    const int a = lane + 64 * i;
    if (a < n) rl |= 1u << i;
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int b = g + CG * j;
      e[i][j] = (a < n && b < n) ? d.A[a + (size_t)b * d.ld] : 0.0;
    }
  }
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    const int p = k & 1, gk = k % CG, jk = k / CG;
    if (g == gk) {
      double cv[RI];
#pragma unroll
      for (int i = 0; i < RI; ++i) cv[i] = e[i][jk];
      // thread best: largest magnitude among its live rows, lowest i first
      u64 bk = 0;
      unsigned bi = 0;
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        const u64 kv = ((rl >> i) & 1u) ? (u64)__double_as_longlong(fabs(cv[i])) + 1ull : 0ull;
        if (kv > bk) { bk = kv; bi = (unsigned)i; }
      }
      const unsigned hi = wave_ext_u32<true>((unsigned)(bk >> 32));
      const unsigned lo = wave_ext_u32<true>((unsigned)(bk >> 32) == hi ? (unsigned)(bk & 0xFFFFFFFFull) : 0u);
      const u64 m = ((u64)hi << 32) | lo;
      const unsigned w = wave_ext_u32<false>(bk == m ? (bi << 6) | (unsigned)lane : 0xFFFFFFFFu);
#pragma unroll
      for (int i = 0; i < RI; ++i) s_col[p][lane + 64 * i] = cv[i];
      if (lane == 0) s_piv[p] = (int)((w & 63u) + 64u * (w >> 6));
    }
    __syncthreads();
    const int pr = (int)uniform((unsigned)s_piv[p]);
    const int ip = pr >> 6;
    double piv = uniform(s_col[p][pr]);
    if (!(fabs(piv) > 0.0)) {
      singular = true;
      piv = 1.0;
    }
    const double inv = 1.0 / piv;
    const bool prow_lane = lane == (pr & 63);
#pragma unroll
    for (int i = 0; i < RI; ++i)
      if (i == ip) {
        if (prow_lane) {
#pragma unroll
          for (int j = 0; j < CJ; ++j) s_row[g][j] = e[i][j];
        }
      }
    if (t == 0) { s_rstep[pr] = (short)k; s_prow[k] = (short)pr; }
    __syncthreads();
    // R = (row p with 1 at k) / piv; f = column k with 0 at row p
    row_t R;
#pragma unroll
    for (int j = 0; j < CJ; ++j) R[j] = s_row[g][j];
    if (g == gk) R[jk] = 1.0;
    R *= inv;
    double f[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const double v = s_col[p][lane + 64 * i];
      f[i] = (lane + 64 * i) == pr ? 0.0 : v;
    }
#pragma unroll
    for (int i = 0; i < RI; ++i) e[i] -= f[i] * R;
    if (g == gk) {
      // column k: (0) - f R(k)
#pragma unroll
      for (int i = 0; i < RI; ++i) e[i][jk] = 0.0 - f[i] * R[jk];
    }
#pragma unroll
    for (int i = 0; i < RI; ++i)
      if (i == ip) {
        if (prow_lane) e[i] = R;
      }
    if (prow_lane) rl &= ~(1u << ip);
  }
  if (singular && t == 0) atomicOr(status, 4);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int a = lane + 64 * i, b = g + CG * j;
      if (a < n && b < n) d.A[s_rstep[a] + (size_t)s_prow[b] * d.ld] = e[i][j];
    }
}

// --------------------------------------------------------- misc vectors ----
template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The host's view of a level: a[0..na), b[0..nb) and *c, in that order, written
// straight into pinned host memory (one launch in place of three copies).
__global__ void readback_kernel(const int* __restrict__ a, int na, const int* __restrict__ b, int nb,
                                const int* __restrict__ c, int* out) {
  const int n = na + nb + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = i < na ? a[i] : (i < na + nb ? b[i - na] : *c);
  __threadfence_system();
}

// Where A's entries go (F_bar_p, Eq. fbar), once per factorisation: a thread
// walks one row r of A; each lower entry k (i = iperm[r] >= j =
// iperm[colind[k]]) goes to the buffer of j's front p, row i - start inside
// its pivot block, else npiv + (the position of i in p's sorted update set),
// column j - start: dest[k] is that element's offset in the workspace and
// lvl[k] the height of p; upper entries get lvl[k] = -1.
__global__ void asm_map_kernel(const int* __restrict__ rowptr, const int* __restrict__ colind,
                               const int* __restrict__ iperm, const int* __restrict__ owner,
                               const AsmFront* __restrict__ fr, const int* __restrict__ upd, int n,
                               int64_t* __restrict__ dest, signed char* __restrict__ lvl) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const int i = iperm[r];
    const int k1 = rowptr[r + 1];
    for (int k = rowptr[r]; k < k1; ++k) {
      const int j = iperm[colind[k]];
      if (i < j) {
        lvl[k] = -1;
        continue;
      }
      const AsmFront f = fr[owner[j]];
      int row;
      if (i < f.start + f.npiv) {
        row = i - f.start;
      } else {
        int lo = 0, hi = f.nupd;                  // first position with upd >= i
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (upd[f.upd0 + mid] < i) lo = mid + 1;
          else hi = mid;
        }
        row = f.npiv + lo;
      }
      dest[k] = f.off + row + (int64_t)(j - f.start) * f.ld;
      lvl[k] = (signed char)f.height;
    }
  }
}

// A's entries of the fronts of height h, placed where dest says
template <typename T>
__global__ void assemble_kernel(T* __restrict__ ws, const int64_t* __restrict__ dest,
                                const signed char* __restrict__ lvl, const double* __restrict__ vals, int64_t nnz,
                                int h) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    if (lvl[k] == h) ws[dest[k]] = (T)vals[k];
}

constexpr int kVecBatch = 8;   // entries per thread per round in the apply's vector gathers

template <typename T>
__global__ __launch_bounds__(256) void vec_asm_kernel(const VecAsmDesc<T>* __restrict__ descs, int nrhs) {
  const VecAsmDesc<T>& d = descs[blockIdx.x];   // read in place (a copy indexed by child would sit in scratch)
  const int tid = threadIdx.x, nt = blockDim.x, k = blockIdx.y;
  T* t = d.t + (size_t)k * d.ldt;
  const T* x = d.xs + (size_t)k * d.ldx;
  // kVecBatch entries per thread at a time: their loads are all issued
  // before the first store, so one workgroup keeps many reads in flight
  const int nhat = d.nhat, npiv = d.npiv;
  for (int i0 = tid; i0 < nhat; i0 += nt * kVecBatch) {
    T v[kVecBatch];
#pragma unroll
    for (int u = 0; u < kVecBatch; ++u) {
      const int i = i0 + u * nt;
      v[u] = i < npiv ? x[i] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kVecBatch; ++u)
      if (i0 + u * nt < nhat) t[i0 + u * nt] = v[u];
  }
  __syncthreads();
  for (int c = 0; c < d.nchild; ++c) {   // children in order: no two threads touch one entry
    const T* ct = d.ct[c] + d.cnp[c] + (size_t)k * d.cld[c];
    const int* rel = d.crel[c];
    const int cnf = d.cnf[c];
    for (int a0 = tid; a0 < cnf; a0 += nt * kVecBatch) {
      int r[kVecBatch];
      T v[kVecBatch];
#pragma unroll
      for (int u = 0; u < kVecBatch; ++u) {
        const int a = a0 + u * nt;
        r[u] = a < cnf ? rel[a] : -1;
        v[u] = a < cnf ? ct[a] : (T)0;
      }
      // a child's relative map is one-to-one, so these entries are distinct.
      // The parent entries are loaded unconditionally (entry 0 for the
      // unused slots) so that their loads are in flight together.
      T tv[kVecBatch];
#pragma unroll
      for (int u = 0; u < kVecBatch; ++u) tv[u] = t[r[u] >= 0 ? r[u] : 0];
#pragma unroll
      for (int u = 0; u < kVecBatch; ++u)
        if (r[u] >= 0) v[u] += tv[u];
#pragma unroll
      for (int u = 0; u < kVecBatch; ++u)
        if (r[u] >= 0) t[r[u]] = v[u];
    }
    __syncthreads();
  }
}


template <typename T>
__global__ void perm_in_kernel(const double* r, T* xn, const int* perm, int N, int nrhs) {
  const int64_t tot = (int64_t)N * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N);
    const int64_t k = idx / N;
    xn[idx] = (T)r[perm[i] + k * N];
  }
}

template <typename T>
__global__ void perm_out_kernel(const T* xn, double* z, const int* iperm, int N, int nrhs) {
  const int64_t tot = (int64_t)N * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N);
    const int64_t k = idx / N;
    z[idx] = (double)xn[iperm[i] + k * N];
  }
}

// ------------------------------------------------------- Krylov / SpMV ----
constexpr int kSpmvLanes = 8;   // lanes per matrix row (rows of 3D stencils hold 7 to 27 entries)
// kSpmvLanes lanes per row, all right-hand sides: lane g of a row takes its
// entries g, g + kSpmvLanes, ..., so neighbouring lanes read neighbouring
// entries, and the lanes of the row combine their partial sums with shuffles
// (with windows, a row takes the columns whose windows hold it: those of one
// system, which are contiguous)
__device__ __forceinline__ void col_window(const int* win, int k, int n, int& lo, int& hi) {
  if (win) {
    lo = win[2 * k];
    hi = win[2 * k + 1];
  } else {
    lo = 0;
    hi = n;
  }
}

__global__ __launch_bounds__(256) void spmv_kernel(const int* __restrict__ rowptr, const int* __restrict__ colind,
                                                   const double* __restrict__ vals, const double* __restrict__ x,
                                                   double* y, int n, int nrhs, double alpha, double beta,
                                                   const int* __restrict__ win) {
  constexpr int KB = 16, G = kSpmvLanes;
  static_assert(KB % G == 0, "each lane writes KB / G columns");
  const int row = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G);
  const int g = threadIdx.x % G;
  if (row >= n) return;                    // whole groups leave together (G divides the wave)
  int c0 = 0, c1 = nrhs;
  if (win) {
    c0 = nrhs;
    c1 = 0;
    for (int k = 0; k < nrhs; ++k)
      if (win[2 * k] <= row && row < win[2 * k + 1]) {
        c0 = min(c0, k);
        c1 = k + 1;
      }
  }
  const int j0 = rowptr[row], j1 = rowptr[row + 1];
  const int kmax = min(KB, nrhs);   // bound on kb shared by every lane: loads past it are not issued
  for (int k0 = c0; k0 < c1; k0 += KB) {
    const int kb = min(KB, c1 - k0);
    double acc[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) acc[q] = 0.0;
    for (int j = j0 + g; j < j1; j += G) {
      const double v = vals[j];
      const double* xc = x + colind[j] + (size_t)k0 * n;
      // all loads in flight at once: columns past kb (up to kmax) re-read
      // column kb - 1 and are dropped (a load used right away, under a
      // per-lane branch, would wait before the next one is issued)
      double xv[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q < kmax) xv[q] = xc[(size_t)min(q, kb - 1) * n];   // kmax is uniform: no per-lane branch
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (q < kmax) acc[q] += q < kb ? v * xv[q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KB; ++q)
      if (q < kb)
        for (int o = G / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, G);
    // lane g writes columns g, g + G, ...: its sums are selected without
    // branches and its y values (beta != 0) loaded before any is used
    constexpr int H = KB / G;
    double mine[H], yv[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int q = g + h * G;
      mine[h] = 0.0;
#pragma unroll
      for (int qq = 0; qq < KB; ++qq) mine[h] = qq == q ? acc[qq] : mine[h];
      yv[h] = beta == 0.0 ? 0.0 : y[(size_t)(k0 + min(q, kb - 1)) * n + row];
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int q = g + h * G;
      if (q < kb) y[(size_t)(k0 + q) * n + row] = beta == 0.0 ? alpha * mine[h] : alpha * mine[h] + beta * yv[h];
    }
  }
}

constexpr int kMdotMax = 64;
// partial[(chunk * nrhs + k) * nv + i] = sum over the chunk of X_i(:,k) .* w(:,k)
// partial dot products of vectors i0 .. i0 + 7 (blockIdx.z = group) with w,
// right-hand side k, over one chunk of rows; accumulators in registers
constexpr int kMdotGroup = 8;
__global__ __launch_bounds__(256) void mdot_partial_kernel(const double* X, int64_t xstride, int nv, const double* w,
                                                           int n, int nrhs, double* partial, const int* win) {
  __shared__ double red[16];
  const int chunk = blockIdx.x, k = blockIdx.y, i0 = blockIdx.z * kMdotGroup;
  const int m = min(kMdotGroup, nv - i0);
  int wlo, whi;
  col_window(win, k, n, wlo, whi);
  const int per = (whi - wlo + gridDim.x - 1) / gridDim.x;
  const int lo = wlo + chunk * per, hi = min(whi, lo + per);
  double acc[kMdotGroup];
#pragma unroll
  for (int i = 0; i < kMdotGroup; ++i) acc[i] = 0.0;
  const double* wk = w + (size_t)k * n;
  const double* Xk = X + (size_t)i0 * xstride + (size_t)k * n;
  for (int row = lo + threadIdx.x; row < hi; row += blockDim.x) {
    const double wv = wk[row];
    // all kMdotGroup loads in flight together: vectors past m re-read
    // vector m - 1 into sums that are never stored
    double xv[kMdotGroup];
#pragma unroll
    for (int i = 0; i < kMdotGroup; ++i) xv[i] = Xk[min(i, m - 1) * xstride + row];
#pragma unroll
    for (int i = 0; i < kMdotGroup; ++i) acc[i] += xv[i] * wv;
  }
#pragma unroll
  for (int i = 0; i < kMdotGroup; ++i)
    if (i < m) {                                      // m is uniform: every thread reaches the barriers
      const double s = block_sum(acc[i], red);
      if (threadIdx.x == 0) partial[((size_t)chunk * nrhs + k) * nv + i0 + i] = s;
    }
}

// one wave per output idx = i * nrhs + k: lanes load the chunk partials
// (one load each for up to 64 chunks), then a butterfly sum in a fixed order
__global__ __launch_bounds__(256) void mdot_reduce_kernel(const double* partial, int nchunk, int nv, int nrhs,
                                                          double* out, int accumulate) {
  const int idx = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (idx >= nv * nrhs) return;                             // whole waves
  const int i = idx / nrhs, k = idx % nrhs;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += partial[((size_t)c * nrhs + k) * nv + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[idx] = accumulate ? out[idx] + s : s;
}

// column k = blockIdx.y, its window's rows strided over blockIdx.x
__global__ void maxpy_kernel(const double* X, int64_t xstride, int nv, const double* coef, double* w, int n, int nrhs,
                             double sign, const int* win) {
  const int k = blockIdx.y;
  int lo, hi;
  col_window(win, k, n, lo, hi);
  for (int row = lo + blockIdx.x * blockDim.x + threadIdx.x; row < hi; row += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)k * n + row;
    double s = 0.0;
#pragma unroll 8
    for (int i = 0; i < nv; ++i) s += coef[i * nrhs + k] * X[i * xstride + idx];
    w[idx] += sign * s;
  }
}

__global__ void scale_cols_kernel(const double* w, double* v, const double* nrm2, int n, int nrhs, const int* win) {
  const int k = blockIdx.y;
  int lo, hi;
  col_window(win, k, n, lo, hi);
  const double nn = sqrt(nrm2[k]);
  for (int row = lo + blockIdx.x * blockDim.x + threadIdx.x; row < hi; row += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)k * n + row;
    v[idx] = nn > 0.0 ? w[idx] / nn : 0.0;
  }
}

__global__ void xupdate_kernel(const double* Z, int64_t zstride, int nv, const double* y, double* x, int n, int nrhs,
                               const int* win) {
  const int k = blockIdx.y;
  int lo, hi;
  col_window(win, k, n, lo, hi);
  for (int row = lo + blockIdx.x * blockDim.x + threadIdx.x; row < hi; row += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)k * n + row;
    double s = 0.0;
#pragma unroll 8
    for (int i = 0; i < nv; ++i) s += y[i * nrhs + k] * Z[i * zstride + idx];
    x[idx] += s;
  }
}

__global__ void axpby_kernel(const double* a, const double* b, double* c, double alpha, double beta, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = alpha * a[i] + beta * b[i];
}

// Conjugate-gradient vector updates, one coefficient per right-hand side k
// (column k of the n x nrhs blocks); an inactive column (act[k] == 0, or a
// zero p^T A p) gets a zero step.
// alpha_k = rz_k / pq_k:  x += alpha p,  rprev = r,  r -= alpha q
__global__ void cg_xr_kernel(double* x, double* r, double* rprev, const double* p, const double* q,
                             const double* rz, const double* pq, const int* act, int n, int nrhs) {
  const int64_t tot = (int64_t)n * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / n);
    const double alpha = (act[k] && pq[k] > 0.0) ? rz[k] / pq[k] : 0.0;
    const double rv = r[idx];
    x[idx] += alpha * p[idx];
    rprev[idx] = rv;
    r[idx] = rv - alpha * q[idx];
  }
}
// beta_k = (rzn_k - rzo_k) / rz_k (flexible form):  p = z + beta p
__global__ void cg_p_kernel(double* p, const double* z, const double* rzn, const double* rzo, const double* rz,
                            const int* act, int n, int nrhs) {
  const int64_t tot = (int64_t)n * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / n);
    const double beta = (act[k] && rz[k] != 0.0) ? (rzn[k] - rzo[k]) / rz[k] : 0.0;
    p[idx] = z[idx] + beta * p[idx];
  }
}

inline int grid_for(int64_t n, int block = 256, int cap = 8192) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

// ------------------------------------------------------------ launchers ----
template <typename T>
void launch_gemm(const GemmDesc<T>* d, int ndesc, int tiles, hipStream_t st, int tn) {
  if (ndesc <= 0 || tiles <= 0) return;
  if (tn == kTileNarrow) MFH_LAUNCH(gemm_narrow_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc);
  else MFH_LAUNCH(gemm_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc);
}
template <typename T>
void launch_gemm_fold(const GemmDesc<T>* d, const FoldDesc<T>* f, int ndesc, int tiles, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH(gemm_narrow_fold_kernel<T>, dim3(tiles), dim3(256), 0, st, d, f, ndesc);
}
template <typename T>
void launch_gemm_reduce(const GemmDesc<T>* d, int ndesc, int tiles, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH(gemm_reduce_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc);
}
template <typename T>
void launch_mfma_probe(int* rows, int* cols, int* assumed, hipStream_t st) {
  MFH_LAUNCH(mfma_probe_kernel<T>, dim3(1), dim3(64), 0, st, rows, cols, assumed);
}
template void launch_mfma_probe<float>(int*, int*, int*, hipStream_t);
template void launch_mfma_probe<double>(int*, int*, int*, hipStream_t);
template <typename T>
void launch_potrf(const PotrfDesc<T>* d, int ndesc, int nmax, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  // blocked MFMA form wherever A and X fit LDS together (all but float64
  // blocks above 64), the register form otherwise
  constexpr size_t lds64 = potrf_blk_lds<T, 64>(), lds128 = potrf_blk_lds<T, 128>();
  if (nmax <= 64)
    MFH_LAUNCH((potrf_blk_kernel<T, 64>), dim3(ndesc), dim3(256), lds64, st, d, status);
  else if constexpr (sizeof(T) == 4)
    MFH_LAUNCH((potrf_blk_kernel<T, 128>), dim3(ndesc), dim3(256), lds128, st, d, status);
  else
    MFH_LAUNCH((potrf_kernel<T, 128, 512>), dim3(ndesc), dim3(512), 0, st, d, status);
}
template <typename T>
void launch_skreg_full(const SkRegDesc<T>* d, int ndesc, double eps, int adaptive, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  if constexpr (sizeof(T) == 8)
    MFH_LAUNCH((skreg_kernel<T, 2, 16, true, 1024>), dim3(ndesc), dim3(1024), 0, st, d, eps, adaptive, status);
  else
    MFH_LAUNCH((skreg_kernel<T, 4, 16, true, 1024>), dim3(ndesc), dim3(1024), 0, st, d, eps, adaptive, status);
}
template <typename T>
void launch_skreg_hat(const SkRegDesc<T>* d, int ndesc, double eps, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  if constexpr (sizeof(T) == 8)
    MFH_LAUNCH((skreg_kernel<T, 2, 8, false, 1024>), dim3(ndesc), dim3(1024), 0, st, d, eps, 0, status);
  else
    MFH_LAUNCH((skreg_kernel<T, 3, 24, false, 512>), dim3(ndesc), dim3(512), 0, st, d, eps, 0, status);
}
template <typename T>
void launch_skelfac(const SkelFacDesc<T>* d, int ndesc, int wgs, int rmax, hipStream_t st) {
  if (ndesc <= 0 || wgs <= 0) return;
  MFH_LAUNCH(skelfac_kernel<T>, dim3(wgs), dim3(kSkelFacThreads), skelfac_lds<T>(rmax), st, d, ndesc, rmax);
}
template <typename T>
void launch_phase2(const Phase2Desc<T>* d, int ndesc, int maxrc, double eps, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  MFH_LAUNCH(phase2_kernel<T>, dim3(ndesc), dim3(1024), (size_t)maxrc, st, d, eps, status);
}
template <typename T>
int phase2_coop_wcols(int nr) {
  const long per_col = (long)nr * sizeof(T) + sizeof(T) + 1;
  const long fixed = (long)nr * (sizeof(T) + 1) + 64;
  const long w = (kPhase2CoopLds - fixed) / per_col;
  return w >= 1 ? (int)w : 0;
}
template <typename T>
size_t phase2_coop_lds(int nr, int wcols, bool slice_lds) {
  return (slice_lds ? (size_t)nr * wcols * sizeof(T) : 0) + (size_t)nr * sizeof(T) + (size_t)wcols * sizeof(T) +
         nr + wcols + 16;
}
template <typename T>
int phase2_coop_capacity(size_t lds, bool slice_lds) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  // the answer depends only on (device, mode, LDS): asked once, then kept
  static std::mutex mu;
  static std::map<std::tuple<int, bool, size_t>, int> known;
  const auto key = std::make_tuple(dev, slice_lds, lds);
  {
    std::lock_guard<std::mutex> g(mu);
    const auto it = known.find(key);
    if (it != known.end()) return it->second;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* k = slice_lds ? reinterpret_cast<const void*>(phase2_coop_kernel<T, true>)
                            : reinterpret_cast<const void*>(phase2_coop_kernel<T, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kCoopThreads, lds) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(mu);
  known[key] = per * cus;
  return per * cus;
}
// One multi-workgroup phase-2 launch runs at a time on a device: two
// spin-barrier launches on different streams could otherwise each hold
// resources the other's missing workgroups need.  Before a launch the host
// waits for the device's previous one unless both are on one stream (which
// orders them already).  The grid never exceeds the resident capacity, so on
// its own a launch always gets all its workgroups resident once other
// streams' (finite) kernels drain; the bounded barrier poll turns any stall
// into status bit 8.
template <typename T>
hipError_t launch_phase2_coop(const Phase2CoopDesc<T>* d, int ndesc, int wgs, size_t lds, bool slice_lds,
                              double eps, int* status, long long wait_ticks, hipStream_t st) {
  if (ndesc <= 0 || wgs <= 0) return hipSuccess;
  struct Last {
    hipEvent_t ev = nullptr;
    hipStream_t st = nullptr;
    bool pending = false;
  };
  static std::mutex mu;
  static std::map<int, Last> last;   // by device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  Last& L = last[dev];
  if (!L.ev) {
    e = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (L.pending && L.st != st) {
    e = hipEventSynchronize(L.ev);
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // what follows reports this launch's error only
  if (slice_lds)
    MFH_LAUNCH((phase2_coop_kernel<T, true>), dim3(wgs), dim3(kCoopThreads), lds, st, d, ndesc, eps, status,
               wait_ticks);
  else
    MFH_LAUNCH((phase2_coop_kernel<T, false>), dim3(wgs), dim3(kCoopThreads), lds, st, d, ndesc, eps, status,
               wait_ticks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipEventRecord(L.ev, st);
  L.st = st;
  L.pending = e == hipSuccess;
  return e;
}
template <typename T>
void launch_gather(const GatherDesc<T>* d, int ndesc, int tiles, const GatherFront<T>* fronts, const int* rowptr,
                   const int* colind, const double* vals, const int* perm, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH(gather_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc, fronts, rowptr, colind, vals, perm);
}
template <typename T>
void launch_cross(const CrossDesc<T>* d, int ndesc, int maxrc, double eps, const int* rowptr, const int* colind,
                  const double* vals, const int* perm, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  MFH_LAUNCH(cross_kernel<T>, dim3(ndesc), dim3(kCrossThreads), (size_t)maxrc, st, d, eps, rowptr, colind, vals, perm,
             status);
}
template <typename T>
void launch_extadd_c(const ExtAddCDesc<T>* d, int ndesc, int tiles, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH(extadd_c_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc);
}
template <typename T>
void launch_extadd(const ExtAddDesc<T>* d, int ndesc, int tiles, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH(extadd_kernel<T>, dim3(tiles), dim3(256), 0, st, d, ndesc);
}
template <typename S, typename D>
void launch_copy(const CopyDesc<S, D>* d, int ndesc, int tiles, hipStream_t st) {
  if (ndesc <= 0 || tiles <= 0) return;
  MFH_LAUNCH((copy_kernel<S, D>), dim3(tiles), dim3(256), 0, st, d, ndesc);
}
template <typename T>
void launch_cap(const CapDesc<T>* d, int ndesc, hipStream_t st) {
  if (ndesc <= 0) return;
  MFH_LAUNCH(cap_kernel<T>, dim3(ndesc), dim3(256), 0, st, d);
}
int gj_kind(int nmax) {
  return nmax <= 64 ? PK_GJ64 : nmax <= 128 ? PK_GJ128 : nmax <= 192 ? PK_GJ192 : PK_GJWIDE;
}
void launch_gj_inverse(const InvDesc* d, int ndesc, int nmax, int* status, hipStream_t st) {
  if (ndesc <= 0) return;
  switch (gj_kind(nmax)) {
    case PK_GJ64: MFH_LAUNCH((gj_kernel<1, 16, 256>), dim3(ndesc), dim3(256), 0, st, d, status); break;
    case PK_GJ128: MFH_LAUNCH((gj_kernel<2, 16, 512>), dim3(ndesc), dim3(512), 0, st, d, status); break;
    case PK_GJ192: MFH_LAUNCH((gj_kernel<3, 16, 768>), dim3(ndesc), dim3(768), 0, st, d, status); break;
    default: MFH_LAUNCH(gj_wide_kernel, dim3(ndesc), dim3(1024), 0, st, d, status); break;
  }
}
__global__ __launch_bounds__(256) void maxabs_kernel(const MaxAbsDesc* __restrict__ descs, double* out) {
  __shared__ double red[kWave];
  const MaxAbsDesc d = descs[blockIdx.x];
  const int64_t tot = (int64_t)d.rows * d.cols;
  double mx = 0.0;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e % d.rows), c = (int)(e / d.rows);
    const double v = fabs(d.p[r + (size_t)c * d.ld]);
    mx = fmax(mx, v != v ? (double)INFINITY : v);   // a NaN is reported as infinity
  }
  mx = block_max(mx, red);
  if (threadIdx.x == 0) out[blockIdx.x] = mx;
}
void launch_maxabs(const MaxAbsDesc* d, int ndesc, double* out, hipStream_t st) {
  if (ndesc <= 0) return;
  MFH_LAUNCH(maxabs_kernel, dim3(ndesc), dim3(256), 0, st, d, out);
}
template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t st) {
  if (n <= 0) return;
  MFH_LAUNCH(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void launch_asm_map(const int* rowptr, const int* colind, const int* iperm, const int* owner, const AsmFront* fr,
                    const int* upd, int n, int64_t* dest, signed char* lvl, hipStream_t st) {
  if (n <= 0) return;
  MFH_LAUNCH(asm_map_kernel, dim3((n + 255) / 256), dim3(256), 0, st, rowptr, colind, iperm, owner, fr, upd, n, dest,
             lvl);
}
void launch_readback(const int* a, int na, const int* b, int nb, const int* c, int* out, hipStream_t st) {
  const int n = na + nb + 1;
  MFH_LAUNCH(readback_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a, na, b, nb, c, out);
}
template <typename T>
void launch_assemble(T* ws, const int64_t* dest, const signed char* lvl, const double* vals, int64_t nnz, int h,
                     hipStream_t st) {
  if (nnz <= 0) return;
  MFH_LAUNCH(assemble_kernel<T>, dim3(grid_for(nnz)), dim3(256), 0, st, ws, dest, lvl, vals, nnz, h);
}
template <typename T>
void launch_vec_asm(const VecAsmDesc<T>* d, int ndesc, int nrhs, hipStream_t st) {
  if (ndesc <= 0) return;
  MFH_LAUNCH(vec_asm_kernel<T>, dim3(ndesc, nrhs), dim3(256), 0, st, d, nrhs);
}
template <typename T>
void launch_perm_in(const double* r, T* xn, const int* perm, int N, int nrhs, hipStream_t st) {
  MFH_LAUNCH(perm_in_kernel<T>, dim3(grid_for((int64_t)N * nrhs)), dim3(256), 0, st, r, xn, perm, N, nrhs);
}
template <typename T>
void launch_perm_out(const T* xn, double* z, const int* iperm, int N, int nrhs, hipStream_t st) {
  MFH_LAUNCH(perm_out_kernel<T>, dim3(grid_for((int64_t)N * nrhs)), dim3(256), 0, st, xn, z, iperm, N, nrhs);
}

void launch_spmv(const int* rowptr, const int* colind, const double* vals, const double* x, double* y, int n,
                 int nrhs, double alpha, double beta, hipStream_t st, const int* win) {
  MFH_LAUNCH(spmv_kernel, dim3((int)(((int64_t)n * kSpmvLanes + 255) / 256)), dim3(256), 0, st, rowptr, colind,
             vals, x, y, n, nrhs, alpha, beta, win);
}
void launch_mdot(const double* X, int64_t xstride, int nv, const double* w, int n, int nrhs, double* partial,
                 double* out, int accumulate, hipStream_t st, const int* win) {
  const int nchunk = mdot_chunks(nrhs);
  MFH_LAUNCH(mdot_partial_kernel, dim3(nchunk, nrhs, (nv + kMdotGroup - 1) / kMdotGroup), dim3(256), 0, st, X,
             xstride, nv, w, n, nrhs, partial, win);
  MFH_LAUNCH(mdot_reduce_kernel, dim3((nv * nrhs + 3) / 4), dim3(256), 0, st, partial, nchunk, nv, nrhs, out,
             accumulate);
}
void launch_cg_xr(double* x, double* r, double* rprev, const double* p, const double* q, const double* rz,
                  const double* pq, const int* act, int n, int nrhs, hipStream_t st) {
  MFH_LAUNCH(cg_xr_kernel, dim3(grid_for((int64_t)n * nrhs)), dim3(256), 0, st, x, r, rprev, p, q, rz, pq, act, n,
             nrhs);
}
void launch_cg_p(double* p, const double* z, const double* rzn, const double* rzo, const double* rz, const int* act,
                 int n, int nrhs, hipStream_t st) {
  MFH_LAUNCH(cg_p_kernel, dim3(grid_for((int64_t)n * nrhs)), dim3(256), 0, st, p, z, rzn, rzo, rz, act, n, nrhs);
}
// per-column launches: as many workgroups in all as the flat form had
inline dim3 col_grid(int n, int nrhs) { return dim3(grid_for(n, 256, std::max(1, 8192 / nrhs)), nrhs); }
void launch_maxpy(const double* X, int64_t xstride, int nv, const double* coef, double* w, int n, int nrhs,
                  double sign, hipStream_t st, const int* win) {
  MFH_LAUNCH(maxpy_kernel, col_grid(n, nrhs), dim3(256), 0, st, X, xstride, nv, coef, w, n, nrhs, sign, win);
}
void launch_scale_cols(const double* w, double* v, const double* norms, int n, int nrhs, hipStream_t st,
                       const int* win) {
  MFH_LAUNCH(scale_cols_kernel, col_grid(n, nrhs), dim3(256), 0, st, w, v, norms, n, nrhs, win);
}
void launch_xupdate(const double* Z, int64_t zstride, int nv, const double* y, double* x, int n, int nrhs,
                    hipStream_t st, const int* win) {
  MFH_LAUNCH(xupdate_kernel, col_grid(n, nrhs), dim3(256), 0, st, Z, zstride, nv, y, x, n, nrhs, win);
}
void launch_axpby(const double* a, const double* b, double* c, double alpha, double beta, int64_t n, hipStream_t st) {
  MFH_LAUNCH(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, st, a, b, c, alpha, beta, n);
}

#define MFH_INST(T)                                                                              \
  template void launch_gemm<T>(const GemmDesc<T>*, int, int, hipStream_t, int);                  \
  template void launch_gemm_reduce<T>(const GemmDesc<T>*, int, int, hipStream_t);                \
  template void launch_gemm_fold<T>(const GemmDesc<T>*, const FoldDesc<T>*, int, int, hipStream_t); \
  template void launch_potrf<T>(const PotrfDesc<T>*, int, int, int*, hipStream_t);               \
  template void launch_skreg_full<T>(const SkRegDesc<T>*, int, double, int, int*, hipStream_t);  \
  template void launch_skreg_hat<T>(const SkRegDesc<T>*, int, double, int*, hipStream_t);        \
  template void launch_skelfac<T>(const SkelFacDesc<T>*, int, int, int, hipStream_t);            \
  template void launch_phase2<T>(const Phase2Desc<T>*, int, int, double, int*, hipStream_t);     \
  template int phase2_coop_wcols<T>(int);                                                         \
  template size_t phase2_coop_lds<T>(int, int, bool);                                             \
  template int phase2_coop_capacity<T>(size_t, bool);                                             \
  template hipError_t launch_phase2_coop<T>(const Phase2CoopDesc<T>*, int, int, size_t, bool, double, int*, long long, \
                                            hipStream_t);                                         \
  template void launch_extadd<T>(const ExtAddDesc<T>*, int, int, hipStream_t);                   \
  template void launch_extadd_c<T>(const ExtAddCDesc<T>*, int, int, hipStream_t);                 \
  template void launch_cross<T>(const CrossDesc<T>*, int, int, double, const int*, const int*, const double*, \
                                const int*, int*, hipStream_t);                                   \
  template void launch_gather<T>(const GatherDesc<T>*, int, int, const GatherFront<T>*, const int*, \
                                 const int*, const double*, const int*, hipStream_t);              \
  template void launch_cap<T>(const CapDesc<T>*, int, hipStream_t);                              \
  template void launch_fill<T>(T*, int64_t, T, hipStream_t);                                     \
  template void launch_assemble<T>(T*, const int64_t*, const signed char*, const double*, int64_t, int, \
                                   hipStream_t);                                                 \
  template void launch_vec_asm<T>(const VecAsmDesc<T>*, int, int, hipStream_t);                  \
  template void launch_perm_in<T>(const double*, T*, const int*, int, int, hipStream_t);         \
  template void launch_perm_out<T>(const T*, double*, const int*, int, int, hipStream_t);

MFH_INST(float)
MFH_INST(double)
template void launch_copy<float, float>(const CopyDesc<float, float>*, int, int, hipStream_t);
template void launch_copy<double, double>(const CopyDesc<double, double>*, int, int, hipStream_t);
template void launch_copy<float, double>(const CopyDesc<float, double>*, int, int, hipStream_t);
template void launch_copy<double, float>(const CopyDesc<double, float>*, int, int, hipStream_t);
template void launch_fill<int>(int*, int64_t, int, hipStream_t);
template void launch_fill<unsigned long long>(unsigned long long*, int64_t, unsigned long long, hipStream_t);

}  // namespace mfh
