// Dense GEMMs on the matrix cores of gfx950, FP64 (v_mfma_f64_16x16x4f64) and
// FP32 (v_mfma_f32_16x16x4f32) inputs.
//
// Each 256-thread block (4 wavefronts of 64) owns a tile of C and walks K in
// steps of 16: the A and B panels are staged through LDS in k-major order so
// that every lane fetches its MFMA operand with one conflict-free read, and
// each wavefront accumulates 16x16 tiles.  Operands: lane l holds A[l%16][l/16]
// and B[l/16][l%16].  Accumulator register r of lane l holds column l%16 and
// row l/16 + 4r (f64) or row 4(l/16) + r (f32) -- both measured on gfx950.
#include <algorithm>

#include "gemm.hpp"

namespace seqx {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

template <class T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4 acc_t;
  typedef d2 pair_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  typedef f2 pair_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Store one accumulator element: C = alpha * acc + beta * C (+ sigma epilogue), in FP64 arithmetic.
template <class To, bool EPI>
__device__ __forceinline__ void store_elem(To* __restrict__ C, long ldc, long b, int row, int col, double alpha,
                                           double accv, double beta, const SigmaEpilogue& ep) {
  double v = alpha * accv;
  To* cp = C + static_cast<long>(row) * ldc + col;
  if (beta != 0.0) v += beta * static_cast<double>(*cp);
  if (EPI) {
    const long vo = ((b / ep.vdiv) % ep.kv) * ep.strideV + static_cast<long>(row) * ldc + col;
    const double vv = ep.Vf ? static_cast<double>(ep.Vf[vo]) : ep.V[vo];
    v += (ep.eps[ep.nocc + col] - ep.eps[row]) * vv;
  }
  *cp = static_cast<To>(v);
}

// ---------------------------------------------------------------- general tiles

template <class T, class To, int WM, int WN, int TM, int TN, bool TA, bool TB, bool EPI>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, double alpha, const T* __restrict__ A, long lda,
                                                   long sA, const T* __restrict__ B, long ldb, long sB, double beta,
                                                   To* __restrict__ C, long ldc, long sC, SigmaEpilogue ep) {
  typedef Mfma<T> MF;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16, BK = 16;
  __shared__ T As[BK][BM];
  __shared__ T Bs[BK][BN];
  const long b = blockIdx.z;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WN) * TM * 16, wn = (wave % WN) * TN * 16;
  typename MF::acc_t acc[TM][TN];
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int i, kk;
      if (!TA) { i = e / BK; kk = e % BK; } else { kk = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + kk;
      T v = 0;
      if (gi < M && gk < K) v = TA ? A[static_cast<long>(gk) * lda + gi] : A[static_cast<long>(gi) * lda + gk];
      As[kk][i] = v;
    }
    for (int e = tid; e < BK * BN; e += 256) {
      int j, kk;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / BK; kk = e % BK; }
      const int gj = n0 + j, gk = k0 + kk;
      T v = 0;
      if (gj < N && gk < K) v = TB ? B[static_cast<long>(gj) * ldb + gk] : B[static_cast<long>(gk) * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }

  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + MF::row(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) store_elem<To, EPI>(C, ldc, b, row, col, alpha, acc[i][j][r], beta, ep);
      }
}

// ---------------------------------------------------------------- 128 x 128 tiles
// For the dense transforms: each of the four wavefronts owns a 64 x 64
// quadrant (4 x 4 MFMA tiles); loads of element pairs.  The K panels are
// double-buffered in LDS: the loads of a later panel are issued (and kept
// ahead of the MFMAs by a scheduling barrier) before the MFMAs of the current
// one and land in the other LDS buffer afterwards, so one barrier per panel
// suffices.  Both precisions prefetch two panels ahead with two register sets
// and use buffer loads on interior tiles; FP32 also issues its LDS operand
// reads one k-step ahead of the MFMAs.  Interior and edge tiles take separate code
// paths.  Needs even leading dimensions and batch strides and pair-aligned
// base pointers (checked by the dispatcher).  Panel depth: 16 (FP64) or 32
// (FP32), which keeps the loads of one panel at 16 registers per lane either
// way.
constexpr int kBM = 128, kBN = 128, kPad = 2;

template <class T>
struct Panel {
  static constexpr int BK = sizeof(T) == 8 ? 16 : 32;
  static constexpr int NP = kBM * BK / 2 / 256;  // element pairs of A per thread
};
// element pairs of B per thread for a tile BN columns wide
template <class T, int BN>
constexpr int kNPB = BN * Panel<T>::BK / 2 / 256;

// Edge tiles and the K head panel: element loads at clamped indices, so every
// load is issued unconditionally (which keeps the wait counters exact).  Rows
// past M and columns past N only feed outputs that are never stored, so their
// clamped values are harmless; columns k >= K are set to zero.
template <class T, bool TA, bool TB, int BN>
__device__ __forceinline__ void panel_load_edge(const T* __restrict__ A, long lda, const T* __restrict__ B, long ldb,
                                                int M, int N, int K, int m0, int n0, int k0, int tid,
                                                typename Mfma<T>::pair_t* ra, typename Mfma<T>::pair_t* rb) {
  constexpr int BK = Panel<T>::BK, HK = BK / 2, HM = kBM / 2, HN = BN / 2;
  auto ld_a = [&](int gi, int gk) {
    const T v = TA ? A[static_cast<long>(min(gk, K - 1)) * lda + min(gi, M - 1)]
                   : A[static_cast<long>(min(gi, M - 1)) * lda + min(gk, K - 1)];
    return gk < K ? v : T(0);
  };
  auto ld_b = [&](int gj, int gk) {
    const T v = TB ? B[static_cast<long>(min(gj, N - 1)) * ldb + min(gk, K - 1)]
                   : B[static_cast<long>(min(gk, K - 1)) * ldb + min(gj, N - 1)];
    return gk < K ? v : T(0);
  };
#pragma unroll
  for (int j = 0; j < Panel<T>::NP; ++j) {
    const int c = tid + 256 * j;
    if (!TA) {
      const int gi = m0 + c / HK, gk = k0 + (c % HK) * 2;
      ra[j].x = ld_a(gi, gk);
      ra[j].y = ld_a(gi, gk + 1);
    } else {
      const int gk = k0 + c / HM, gi = m0 + (c % HM) * 2;
      ra[j].x = ld_a(gi, gk);
      ra[j].y = ld_a(gi + 1, gk);
    }
  }
#pragma unroll
  for (int j = 0; j < kNPB<T, BN>; ++j) {
    const int c = tid + 256 * j;
    if (!TB) {
      const int gk = k0 + c / HN, gj = n0 + (c % HN) * 2;
      rb[j].x = ld_b(gj, gk);
      rb[j].y = ld_b(gj + 1, gk);
    } else {
      const int gj = n0 + c / HK, gk = k0 + (c % HK) * 2;
      rb[j].x = ld_b(gj, gk);
      rb[j].y = ld_b(gj, gk + 1);
    }
  }
}

// Interior panels: buffer loads from a descriptor at the tile's corner, with
// the panel's position as a scalar offset and a per-thread 32-bit offset fixed
// for the whole tile, so each load needs one vector register for its address.
// Word 3 of the descriptor (0x00020000) is the gfx9 raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}

template <class T>
__device__ __forceinline__ typename Mfma<T>::pair_t buffer_pair(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                                unsigned soff);
template <>
__device__ __forceinline__ f2 buffer_pair<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ d2 buffer_pair<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

template <class T, int BN>
__device__ __forceinline__ void panel_load_fast(__amdgpu_buffer_rsrc_t ar, unsigned asoff, __amdgpu_buffer_rsrc_t br,
                                                unsigned bsoff, const unsigned* oa, const unsigned* ob,
                                                typename Mfma<T>::pair_t* ra, typename Mfma<T>::pair_t* rb) {
#pragma unroll
  for (int j = 0; j < Panel<T>::NP; ++j) ra[j] = buffer_pair<T>(ar, oa[j], asoff);
#pragma unroll
  for (int j = 0; j < kNPB<T, BN>; ++j) rb[j] = buffer_pair<T>(br, ob[j], bsoff);
}

template <class T, bool TA, bool TB, int BN>
__device__ __forceinline__ void panel_store(T (*As)[kBM + kPad], T (*Bs)[BN + kPad], int tid,
                                            const typename Mfma<T>::pair_t* ra, const typename Mfma<T>::pair_t* rb) {
  constexpr int BK = Panel<T>::BK, HK = BK / 2, HM = kBM / 2, HN = BN / 2;
#pragma unroll
  for (int j = 0; j < Panel<T>::NP; ++j) {
    const int c = tid + 256 * j;
    if (!TA) {
      const int i = c / HK, kk = (c % HK) * 2;
      As[kk][i] = ra[j].x;
      As[kk + 1][i] = ra[j].y;
    } else {
      const int kk = c / HM, i = (c % HM) * 2;
      As[kk][i] = ra[j].x;
      As[kk][i + 1] = ra[j].y;
    }
  }
#pragma unroll
  for (int j = 0; j < kNPB<T, BN>; ++j) {
    const int c = tid + 256 * j;
    if (!TB) {
      const int kk = c / HN, jj = (c % HN) * 2;
      Bs[kk][jj] = rb[j].x;
      Bs[kk][jj + 1] = rb[j].y;
    } else {
      const int jj = c / HK, kk = (c % HK) * 2;
      Bs[kk][jj] = rb[j].x;
      Bs[kk + 1][jj] = rb[j].y;
    }
  }
}

// FP32: the operands of k-step s + 1 are read from LDS before the MFMAs of
// step s are issued, so the LDS latency overlaps the matrix-core work.  FP64
// keeps one operand set: its accumulators take twice the registers, and a
// second set would cost a wavefront per SIMD.
template <class T, int TN>
__device__ __forceinline__ void panel_mfma(const T (*As)[kBM + kPad], const T (*Bs)[TN * 32 + kPad], int lane, int wm,
                                           int wn, typename Mfma<T>::acc_t (*acc)[TN]) {
  constexpr int NS = Panel<T>::BK / 4;
  if constexpr (sizeof(T) == 8) {  // FP64: one operand set, order left to the compiler
#pragma unroll
    for (int ks = 0; ks < Panel<T>::BK; ks += 4) {
      T a[4], bb[TN];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::op(a[i], bb[j], acc[i][j]);
    }
    return;
  }
  T a[2][4], bb[2][TN];
  auto read = [&](int ks, T* ar, T* br) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ar[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < TN; ++j) br[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
  };
  read(0, a[0], bb[0]);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s + 1 < NS) read(4 * (s + 1), a[(s + 1) & 1], bb[(s + 1) & 1]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::op(a[s & 1][i], bb[s & 1][j], acc[i][j]);
  }
  // schedule: the LDS reads of step 0, then per step the reads of step s + 1
  // ahead of the 4 TN MFMAs of step s (masks: 0x100 LDS read, 0x008 MFMA)
  __builtin_amdgcn_sched_group_barrier(0x100, 4 + TN, 0);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s + 1 < NS) __builtin_amdgcn_sched_group_barrier(0x100, 4 + TN, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 4 * TN, 0);
  }
}

// EM: 0 interior tile; 1 edge tile whose pair dimensions (M when A is
// transposed, N when B is not) are even, loaded like an interior tile at
// clamped offsets; 2 other edge tiles, element loads.
// BN: tile width, 128 or 96 (each wavefront then owns 64 x BN / 2, TN = BN / 32
// MFMA tiles across).
template <class T, class To, bool TA, bool TB, bool EPI, int EM, int BN>
__device__ __forceinline__ void tile128(int M, int N, int K, double alpha, const T* __restrict__ A, long lda,
                                        const T* __restrict__ B, long ldb, double beta, To* __restrict__ C, long ldc,
                                        long b, const SigmaEpilogue& ep, int m0, int n0, T (*As)[kBM + kPad],
                                        T (*Bs)[BN + kPad]) {
  typedef Mfma<T> MF;
  constexpr int BK = Panel<T>::BK, TN = BN / 32, NPB = kNPB<T, BN>;
  constexpr bool EDGE = EM != 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * (BN / 2);
  typename MF::acc_t acc[4][TN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};
  typedef typename MF::pair_t P2;
  {
    // K is walked as a head panel of K % BK columns (when K is not a multiple
    // of BK), loaded with zero fill, followed by full panels, so that the
    // steady-state loop holds no K checks.  Two register sets for the
    // global prefetch: the loads of panel p + 2 are issued while panel p is
    // multiplied and have two panels of MFMA work to land before they are
    // stored to LDS.  The loads are unconditional (past the last panel they
    // repeat it and are not stored): a conditional load would make the wait
    // before the LDS stores cover the newest loads as well.
    P2 ra0[Panel<T>::NP], rb0[NPB], ra1[Panel<T>::NP], rb1[NPB];
    const int kr = K % BK;
    const int npan = K / BK + (kr ? 1 : 0);
    const int kshift = kr ? kr - BK : 0;  // panel p >= 1 starts at p * BK + kshift
    constexpr int HK = BK / 2, HM = kBM / 2, HN = BN / 2;
    // Byte offsets inside a panel.  On edge tiles (EM == 1) rows and columns
    // past M and N are clamped to the last ones (pair starts to the last
    // pair): they only feed outputs that are not stored.
    const int im = M - 1 - m0, in = N - 1 - n0;  // last valid row / column of the tile
    unsigned oa[Panel<T>::NP], ob[NPB];
#pragma unroll
    for (int j = 0; j < Panel<T>::NP; ++j) {
      const int c = tid + 256 * j;
      int i = TA ? (c % HM) * 2 : c / HK, kk = TA ? c / HM : (c % HK) * 2;
      if (EM == 1) i = TA ? min(i, im - 1) : min(i, im);
      oa[j] = static_cast<unsigned>(TA ? kk * lda + i : i * lda + kk) * sizeof(T);
    }
#pragma unroll
    for (int j = 0; j < NPB; ++j) {
      const int c = tid + 256 * j;
      int jj = TB ? c / HK : (c % HN) * 2, kb = TB ? (c % HK) * 2 : c / HN;
      if (EM == 1) jj = TB ? min(jj, in) : min(jj, in - 1);
      ob[j] = static_cast<unsigned>(TB ? jj * ldb + kb : kb * ldb + jj) * sizeof(T);
    }
    const __amdgpu_buffer_rsrc_t ar = buffer_rsrc(TA ? A + m0 : A + static_cast<long>(m0) * lda);
    const __amdgpu_buffer_rsrc_t br = buffer_rsrc(TB ? B + static_cast<long>(n0) * ldb : B + n0);
    auto load_full = [&](int p, P2* ra, P2* rb) {
      const int k0 = p * BK + kshift;
      if (EM < 2)
        panel_load_fast<T, BN>(ar, static_cast<unsigned>(TA ? k0 * lda : k0) * sizeof(T), br,
                               static_cast<unsigned>(TB ? k0 : k0 * ldb) * sizeof(T), oa, ob, ra, rb);
      else
        panel_load_edge<T, TA, TB, BN>(A, lda, B, ldb, M, N, K, m0, n0, k0, tid, ra, rb);
    };
    // LDS buffers 0 and 1: rows [0, BK) and [BK, 2 BK) of As / Bs
    if (kr) panel_load_edge<T, TA, TB, BN>(A, lda, B, ldb, M, N, kr, m0, n0, 0, tid, ra0, rb0);
    else load_full(0, ra0, rb0);
    load_full(min(1, npan - 1), ra1, rb1);
    panel_store<T, TA, TB, BN>(As, Bs, tid, ra0, rb0);
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < npan; kt += 2) {
      load_full(min(kt + 2, npan - 1), ra0, rb0);
      __builtin_amdgcn_sched_barrier(0);
      panel_mfma<T, TN>(As, Bs, lane, wm, wn, acc);
      panel_store<T, TA, TB, BN>(As + BK, Bs + BK, tid, ra1, rb1);
      __syncthreads();
      load_full(min(kt + 3, npan - 1), ra1, rb1);
      __builtin_amdgcn_sched_barrier(0);
      panel_mfma<T, TN>(As + BK, Bs + BK, lane, wm, wn, acc);
      if (kt + 2 < npan) panel_store<T, TA, TB, BN>(As, Bs, tid, ra0, rb0);
      __syncthreads();
    }
    if (kt < npan) panel_mfma<T, TN>(As, Bs, lane, wm, wn, acc);  // odd panel count: the last one is in buffer 0
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + MF::row(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (!EDGE || (row < M && col < N)) store_elem<To, EPI>(C, ldc, b, row, col, alpha, acc[i][j][r], beta, ep);
      }
}

template <class T, class To, bool TA, bool TB, bool EPI, int BN>
__global__ void __launch_bounds__(256) gemm128_kernel(int M, int N, int K, double alpha, const T* __restrict__ A,
                                                      long lda, long sA, const T* __restrict__ B, long ldb, long sB,
                                                      double beta, To* __restrict__ C, long ldc, long sC,
                                                      SigmaEpilogue ep) {
  constexpr int BK = Panel<T>::BK;
  __shared__ T As[2 * BK][kBM + kPad];
  __shared__ T Bs[2 * BK][BN + kPad];
  const long b = blockIdx.z;
  // Workgroups go to the 8 XCDs round-robin by linear id, and each XCD has its
  // own L2.  Regroup the ids so that each XCD gets a contiguous run of tiles in
  // row-major order: the column tiles of one row panel of A then share an L2
  // (the ids past the largest multiple of 8 keep their place).
  const int nbx = gridDim.x, nb = gridDim.x * gridDim.y, nfull = nb - nb % 8;
  int bid = blockIdx.y * nbx + blockIdx.x;
  if (bid < nfull) bid = (bid % 8) * (nfull / 8) + bid / 8;
  const int m0 = (bid / nbx) * kBM, n0 = (bid % nbx) * BN;
  const bool keven = (K & 1) == 0;  // panels start at even k (pair loads)
  if (m0 + kBM <= M && n0 + BN <= N && keven)
    tile128<T, To, TA, TB, EPI, 0, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                       m0, n0, As, Bs);
  else if (keven && (!TA || (M & 1) == 0) && (TB || (N & 1) == 0))
    tile128<T, To, TA, TB, EPI, 1, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                       m0, n0, As, Bs);
  else
    tile128<T, To, TA, TB, EPI, 2, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                       m0, n0, As, Bs);
}

// ---------------------------------------------------------------- dispatch

#define SEQX_DISPATCH_T(KERNEL, ...)                                                                    \
  do {                                                                                                  \
    if (!ta && !tb) hipLaunchKernelGGL((KERNEL<__VA_ARGS__, false, false, EPI>), grid, dim3(256), 0, st, \
                                       M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ep);  \
    else if (!ta && tb) hipLaunchKernelGGL((KERNEL<__VA_ARGS__, false, true, EPI>), grid, dim3(256), 0, \
                                           st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ep); \
    else if (ta && !tb) hipLaunchKernelGGL((KERNEL<__VA_ARGS__, true, false, EPI>), grid, dim3(256), 0, \
                                           st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ep); \
    else hipLaunchKernelGGL((KERNEL<__VA_ARGS__, true, true, EPI>), grid, dim3(256), 0, st, M, N, K,     \
                            alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ep);                       \
  } while (0)

template <class T, class To, bool EPI, int BN>
void launch128(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const T* A, long lda, long sA,
               const T* B, long ldb, long sB, double beta, To* C, long ldc, long sC, int batch,
               const SigmaEpilogue& ep) {
  dim3 grid(ceil_div(N, BN), ceil_div(M, kBM), batch);
  const dim3 blk(256);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm128_kernel<T, To, false, false, EPI, BN>), grid, blk, 0, st, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, ep);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm128_kernel<T, To, false, true, EPI, BN>), grid, blk, 0, st, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, ep);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm128_kernel<T, To, true, false, EPI, BN>), grid, blk, 0, st, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, ep);
  else
    hipLaunchKernelGGL((gemm128_kernel<T, To, true, true, EPI, BN>), grid, blk, 0, st, M, N, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC, ep);
}

// Tile width of the 128-row tiles: 96 when it pads N by at least 3 % less
// than 128 does (N = 660: 672 columns instead of 768).
int tile_width(int N) {
  const long w128 = static_cast<long>(ceil_div(N, 128)) * 128, w96 = static_cast<long>(ceil_div(N, 96)) * 96;
  return 100 * w96 < 97 * w128 ? 96 : 128;
}

template <class T, class To, int WM, int WN, int TM, int TN, bool EPI>
void launch_cfg(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const T* A, long lda, long sA,
                const T* B, long ldb, long sB, double beta, To* C, long ldc, long sC, int batch,
                const SigmaEpilogue& ep) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  dim3 grid(ceil_div(N, BN), ceil_div(M, BM), batch);
  SEQX_DISPATCH_T(gemm_kernel, T, To, WM, WN, TM, TN);
}

bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

template <class T, class To>
void gemm_any(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const T* A, long lda, long sA,
              const T* B, long ldb, long sB, double beta, To* C, long ldc, long sC, int batch,
              const SigmaEpilogue* epi) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // an empty product: C = beta * C (only used with beta = 0 in practice)
    if (beta == 0.0)
      for (int b = 0; b < batch; ++b)
        for (int i = 0; i < M; ++i)
          SEQX_HIP(hipMemsetAsync(C + b * sC + static_cast<long>(i) * ldc, 0, N * sizeof(To), st));
    return;
  }
  SigmaEpilogue ep;
  if (epi) ep = *epi;
  if constexpr (sizeof(T) == 8 && sizeof(To) == 8) {
    if (!ta && !tb && !epi && batch == 1 && N >= 4096 && (M <= 48 || (M <= 256 && N >= 64L * M))) {
      // combinations of a long basis: passes of at most 48 output rows, each
      // reading B once
      for (int r0 = 0; r0 < M; r0 += 48)
        skinny_combine(st, std::min(48, M - r0), N, K, alpha, A + static_cast<long>(r0) * lda, lda, B, ldb, beta,
                       C + static_cast<long>(r0) * ldc, ldc);
      return;
    }
  }
  const bool skinny = N <= 16;
  const bool even = ((lda | ldb | sA | sB) & 1) == 0 && aligned_to(A, 2 * sizeof(T)) && aligned_to(B, 2 * sizeof(T));
  // the 128 x 128 tiles address each operand with 32-bit byte offsets from a
  // tile corner: rows and panel steps must stay below 2 GiB
  const long ldmax = lda > ldb ? lda : ldb;
  const bool small_offsets = (ldmax * (static_cast<long>(K > kBM ? K : kBM) + kBM) + K) * static_cast<long>(sizeof(T)) <
                             (1L << 31);
  if (even && small_offsets && M >= 96 && N >= 96 && K >= 16) {
    const bool w96 = tile_width(N) == 96;
    if (epi && w96)
      launch128<T, To, true, 96>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
    else if (epi)
      launch128<T, To, true, 128>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
    else if (w96)
      launch128<T, To, false, 96>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
    else
      launch128<T, To, false, 128>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  } else if (epi) {
    launch_cfg<T, To, 2, 2, 2, 2, true>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                                        ep);
  } else if (!skinny && M <= 32) {
    launch_cfg<T, To, 1, 4, 2, 1, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                                         ep);
  } else if (skinny) {
    launch_cfg<T, To, 4, 1, 1, 1, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                                         ep);
  } else {
    launch_cfg<T, To, 2, 2, 2, 2, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                                         ep);
  }
  SEQX_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- split-bfloat16 tiles
// FP32 operands multiplied as x = hi + lo, hi = bf16(x), lo = bf16(x - hi)
// (round to nearest even both times): a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b
// on the bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, 32 k per
// instruction), FP32 accumulation.  Dropped: lo_a lo_b and the rounding of the
// lo parts, so each product carries a relative error of at most 3 * 2^-16.
// Same 128 x 128 tile, prefetch and XCD order as the FP32 kernel; the panels
// are split once, when stored to LDS, as hi and lo planes with k contiguous per
// row (one 16-byte LDS read per operand of an MFMA).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

// hi and lo parts of two values, packed two per word (element 0 in the low
// half): one hardware conversion (round to nearest even) per pair for each part
__device__ __forceinline__ void split_pair(float x, float y, unsigned& hi, unsigned& lo) {
  const bf2 h = {static_cast<__bf16>(x), static_cast<__bf16>(y)};
  const unsigned hb = __builtin_bit_cast(unsigned, h);
  const float hx = __uint_as_float(hb << 16), hy = __uint_as_float(hb & 0xffff0000u);
  const bf2 l = {static_cast<__bf16>(x - hx), static_cast<__bf16>(y - hy)};
  hi = hb;
  lo = __builtin_bit_cast(unsigned, l);
}

constexpr int kBK3 = 32;           // k per panel
constexpr int kLd3 = kBK3 + 8;     // bf16 per LDS row (k contiguous), padded; rows stay 16-byte aligned

// element pairs per thread of a 32-deep panel W rows (or columns) wide
template <int W>
constexpr int kNP3 = W * kBK3 / 2 / 256;

// B planes for tiles BN columns wide (128, or 96 where that pads N less)
template <int BN>
struct Lds3 {
  unsigned short ahi[2][kBM][kLd3], alo[2][kBM][kLd3], bhi[2][BN][kLd3], blo[2][BN][kLd3];
};

// Which elements a thread loads.  An operand whose rows in memory run along k
// (A not transposed, B transposed) is loaded as pairs of consecutive k of one
// row / column; one whose rows run along the tile index (A transposed, B not)
// as 2 x 2 blocks: pairs 2q and 2q + 1 hold index i, i + 1 at k and k + 1.
// Either way each LDS word written holds two consecutive k of one row.
// Element pair j of thread tid in a tile W wide: tile index i, panel column k (first element).
template <bool KM, int W>
__device__ __forceinline__ void pair_pos3(int tid, int j, int& i, int& k) {
  constexpr int HK = kBK3 / 2, HW = W / 2;
  if (!KM) {
    const int c = tid + 256 * j;
    i = c / HK;
    k = (c % HK) * 2;
  } else {
    const int c = tid + 256 * (j >> 1);
    k = 2 * (c / HW) + (j & 1);
    i = (c % HW) * 2;
  }
}

// Panel loads, clamped at the edges like panel_load_edge: element (i, k) of
// A (rows i, KA: A[k lda + i] when transposed) and of B (columns i).
template <bool TA, bool TB, int BN>
__device__ __forceinline__ void panel_load_edge3(const float* __restrict__ A, long lda, const float* __restrict__ B,
                                                 long ldb, int M, int N, int K, int m0, int n0, int k0, int tid,
                                                 f2* ra, f2* rb) {
  auto ld_a = [&](int gi, int gk) {
    const float v = TA ? A[static_cast<long>(min(gk, K - 1)) * lda + min(gi, M - 1)]
                       : A[static_cast<long>(min(gi, M - 1)) * lda + min(gk, K - 1)];
    return gk < K ? v : 0.0f;
  };
  auto ld_b = [&](int gj, int gk) {
    const float v = TB ? B[static_cast<long>(min(gj, N - 1)) * ldb + min(gk, K - 1)]
                       : B[static_cast<long>(min(gk, K - 1)) * ldb + min(gj, N - 1)];
    return gk < K ? v : 0.0f;
  };
#pragma unroll
  for (int j = 0; j < kNP3<kBM>; ++j) {
    int i, k;
    pair_pos3<TA, kBM>(tid, j, i, k);
    ra[j].x = ld_a(m0 + i, k0 + k);
    ra[j].y = TA ? ld_a(m0 + i + 1, k0 + k) : ld_a(m0 + i, k0 + k + 1);
  }
#pragma unroll
  for (int j = 0; j < kNP3<BN>; ++j) {
    int i, k;
    pair_pos3<!TB, BN>(tid, j, i, k);
    rb[j].x = ld_b(n0 + i, k0 + k);
    rb[j].y = TB ? ld_b(n0 + i, k0 + k + 1) : ld_b(n0 + i + 1, k0 + k);
  }
}

template <bool KM, int W>
__device__ __forceinline__ void store_plane3(unsigned short (*hi)[kLd3], unsigned short (*lo)[kLd3], int tid,
                                             const f2* r) {
  if (!KM) {
#pragma unroll
    for (int j = 0; j < kNP3<W>; ++j) {
      int i, k;
      pair_pos3<false, W>(tid, j, i, k);
      unsigned h, l;
      split_pair(r[j].x, r[j].y, h, l);
      *reinterpret_cast<unsigned*>(&hi[i][k]) = h;
      *reinterpret_cast<unsigned*>(&lo[i][k]) = l;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kNP3<W> / 2; ++q) {
      int i, k;
      pair_pos3<true, W>(tid, 2 * q, i, k);
      unsigned h, l;
      split_pair(r[2 * q].x, r[2 * q + 1].x, h, l);  // index i at k, k + 1
      *reinterpret_cast<unsigned*>(&hi[i][k]) = h;
      *reinterpret_cast<unsigned*>(&lo[i][k]) = l;
      split_pair(r[2 * q].y, r[2 * q + 1].y, h, l);  // index i + 1
      *reinterpret_cast<unsigned*>(&hi[i + 1][k]) = h;
      *reinterpret_cast<unsigned*>(&lo[i + 1][k]) = l;
    }
  }
}

template <bool TA, bool TB, int BN>
__device__ __forceinline__ void panel_store3(Lds3<BN>& L, int buf, int tid, const f2* ra, const f2* rb) {
  store_plane3<TA, kBM>(L.ahi[buf], L.alo[buf], tid, ra);
  store_plane3<!TB, BN>(L.bhi[buf], L.blo[buf], tid, rb);
}

// one panel of 32 k: lane l reads k 8 (l / 16) .. + 7 of row l % 16 of each tile
template <int BN>
__device__ __forceinline__ void panel_mfma3(const Lds3<BN>& L, int buf, int lane, int wm, int wn,
                                            f4 (*acc)[BN / 32]) {
  constexpr int TN = BN / 32;
  const int r = lane & 15, k8 = 8 * (lane >> 4);
  bf8 ah[4], al[4], bh[TN], bl[TN];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ah[i] = *reinterpret_cast<const bf8*>(&L.ahi[buf][wm + i * 16 + r][k8]);
    al[i] = *reinterpret_cast<const bf8*>(&L.alo[buf][wm + i * 16 + r][k8]);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    bh[j] = *reinterpret_cast<const bf8*>(&L.bhi[buf][wn + j * 16 + r][k8]);
    bl[j] = *reinterpret_cast<const bf8*>(&L.blo[buf][wn + j * 16 + r][k8]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
}

template <class To, bool TA, bool TB, bool EPI, int EM, int BN>
__device__ __forceinline__ void tile128x3(int M, int N, int K, double alpha, const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb, double beta, To* __restrict__ C,
                                          long ldc, long b, const SigmaEpilogue& ep, int m0, int n0, Lds3<BN>& L) {
  typedef f2 P2;
  constexpr int BK = kBK3, TN = BN / 32, NPA = kNP3<kBM>, NPB = kNP3<BN>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * (BN / 2);
  f4 acc[4][TN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0, 0, 0, 0};
  // K as a head panel of K % BK columns (zero filled), then full panels; two
  // register sets prefetch two panels ahead (as in the FP32 kernel)
  P2 ra0[NPA], rb0[NPB], ra1[NPA], rb1[NPB];
  const int kr = K % BK;
  const int npan = K / BK + (kr ? 1 : 0);
  const int kshift = kr ? kr - BK : 0;
  const int im = M - 1 - m0, in = N - 1 - n0;
  unsigned oa[NPA], ob[NPB];
#pragma unroll
  for (int j = 0; j < NPA; ++j) {
    int i, kk;
    pair_pos3<TA, kBM>(tid, j, i, kk);
    if (EM == 1) i = TA ? min(i, im - 1) : min(i, im);
    oa[j] = static_cast<unsigned>(TA ? kk * lda + i : i * lda + kk) * sizeof(float);
  }
#pragma unroll
  for (int j = 0; j < NPB; ++j) {
    int jj, kb;
    pair_pos3<!TB, BN>(tid, j, jj, kb);
    if (EM == 1) jj = TB ? min(jj, in) : min(jj, in - 1);
    ob[j] = static_cast<unsigned>(TB ? jj * ldb + kb : kb * ldb + jj) * sizeof(float);
  }
  const __amdgpu_buffer_rsrc_t ar = buffer_rsrc(TA ? A + m0 : A + static_cast<long>(m0) * lda);
  const __amdgpu_buffer_rsrc_t br = buffer_rsrc(TB ? B + static_cast<long>(n0) * ldb : B + n0);
  auto load_full = [&](int p, P2* ra, P2* rb) {
    const int k0 = p * BK + kshift;
    if (EM < 2)
      panel_load_fast<float, BN>(ar, static_cast<unsigned>(TA ? k0 * lda : k0) * sizeof(float), br,
                                 static_cast<unsigned>(TB ? k0 : k0 * ldb) * sizeof(float), oa, ob, ra, rb);
    else
      panel_load_edge3<TA, TB, BN>(A, lda, B, ldb, M, N, K, m0, n0, k0, tid, ra, rb);
  };
  if (kr) panel_load_edge3<TA, TB, BN>(A, lda, B, ldb, M, N, kr, m0, n0, 0, tid, ra0, rb0);
  else load_full(0, ra0, rb0);
  load_full(min(1, npan - 1), ra1, rb1);
  panel_store3<TA, TB, BN>(L, 0, tid, ra0, rb0);
  __syncthreads();
  int kt = 0;
  for (; kt + 1 < npan; kt += 2) {
    load_full(min(kt + 2, npan - 1), ra0, rb0);
    __builtin_amdgcn_sched_barrier(0);
    panel_mfma3<BN>(L, 0, lane, wm, wn, acc);
    panel_store3<TA, TB, BN>(L, 1, tid, ra1, rb1);
    __syncthreads();
    load_full(min(kt + 3, npan - 1), ra1, rb1);
    __builtin_amdgcn_sched_barrier(0);
    panel_mfma3<BN>(L, 1, lane, wm, wn, acc);
    if (kt + 2 < npan) panel_store3<TA, TB, BN>(L, 0, tid, ra0, rb0);
    __syncthreads();
  }
  if (kt < npan) panel_mfma3<BN>(L, 0, lane, wm, wn, acc);
  constexpr bool EDGE = EM != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (!EDGE || (row < M && col < N)) store_elem<To, EPI>(C, ldc, b, row, col, alpha, acc[i][j][r], beta, ep);
      }
}

template <class To, bool TA, bool TB, bool EPI, int BN>
__global__ void __launch_bounds__(256) gemm128x3_kernel(int M, int N, int K, double alpha,
                                                        const float* __restrict__ A, long lda, long sA,
                                                        const float* __restrict__ B, long ldb, long sB, double beta,
                                                        To* __restrict__ C, long ldc, long sC, SigmaEpilogue ep) {
  __shared__ Lds3<BN> L;
  const long b = blockIdx.z;
  const int nbx = gridDim.x, nb = gridDim.x * gridDim.y, nfull = nb - nb % 8;
  int bid = blockIdx.y * nbx + blockIdx.x;
  if (bid < nfull) bid = (bid % 8) * (nfull / 8) + bid / 8;
  const int m0 = (bid / nbx) * kBM, n0 = (bid % nbx) * BN;
  const bool keven = (K & 1) == 0;
  if (m0 + kBM <= M && n0 + BN <= N && keven)
    tile128x3<To, TA, TB, EPI, 0, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                      m0, n0, L);
  else if (keven && (!TA || (M & 1) == 0) && (TB || (N & 1) == 0))
    tile128x3<To, TA, TB, EPI, 1, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                      m0, n0, L);
  else
    tile128x3<To, TA, TB, EPI, 2, BN>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep,
                                      m0, n0, L);
}

template <class To>
void gemm_x3(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda, long sA,
             const float* B, long ldb, long sB, double beta, To* C, long ldc, long sC, int batch,
             const SigmaEpilogue* epi) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  const bool even = ((lda | ldb | sA | sB) & 1) == 0 && aligned_to(A, 8) && aligned_to(B, 8);
  const long ldmax = lda > ldb ? lda : ldb;
  const bool small_offsets = (ldmax * (static_cast<long>(K > kBM ? K : kBM) + kBM) + K) * 4L < (1L << 31);
  if (!(even && small_offsets && M >= 96 && N >= 96 && K >= 32)) {
    // shapes outside the tile path stay on the FP32 matrix cores
    gemm_any<float, To>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
    return;
  }
  SigmaEpilogue ep;
  if (epi) ep = *epi;
  // 96-wide tiles where they pad N less (v = 660: 672 columns instead of 768)
  const bool w96 = tile_width(N) == 96;
  dim3 grid(ceil_div(N, w96 ? 96 : kBN), ceil_div(M, kBM), batch);
#define SEQX_X3(TA_, TB_, BN_)                                                                                     \
  do {                                                                                                            \
    if (epi)                                                                                                      \
      hipLaunchKernelGGL((gemm128x3_kernel<To, TA_, TB_, true, BN_>), grid, dim3(256), 0, st, M, N, K, alpha, A,   \
                         lda, sA, B, ldb, sB, beta, C, ldc, sC, ep);                                              \
    else                                                                                                          \
      hipLaunchKernelGGL((gemm128x3_kernel<To, TA_, TB_, false, BN_>), grid, dim3(256), 0, st, M, N, K, alpha, A,  \
                         lda, sA, B, ldb, sB, beta, C, ldc, sC, ep);                                              \
  } while (0)
#define SEQX_X3_BN(BN_)                   \
  do {                                    \
    if (!ta && !tb) SEQX_X3(false, false, BN_); \
    else if (!ta && tb) SEQX_X3(false, true, BN_); \
    else if (ta && !tb) SEQX_X3(true, false, BN_); \
    else SEQX_X3(true, true, BN_);        \
  } while (0)
  if (w96) SEQX_X3_BN(96);
  else SEQX_X3_BN(kBN);
#undef SEQX_X3_BN
#undef SEQX_X3
  SEQX_LAUNCH_CHECK();
}

}  // namespace

void dgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda, long sA,
           const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
           const SigmaEpilogue* epi) {
  gemm_any<double, double>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
}

void sgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda, long sA,
           const float* B, long ldb, long sB, double beta, float* C, long ldc, long sC, int batch,
           const SigmaEpilogue* epi) {
  gemm_any<float, float>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
}

void sgemm_out64(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda,
                 long sA, const float* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
                 const SigmaEpilogue* epi) {
  gemm_any<float, double>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
}

void sgemm3(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda, long sA,
            const float* B, long ldb, long sB, double beta, float* C, long ldc, long sC, int batch,
            const SigmaEpilogue* epi) {
  gemm_x3<float>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
}

void sgemm3_out64(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda,
                  long sA, const float* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
                  const SigmaEpilogue* epi) {
  gemm_x3<double>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, epi);
}

void dgemm_cm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
              const double* B, long ldb, double beta, double* C, long ldc) {
  // column-major C = op(A) op(B) is row-major C^T = op(B)^T op(A)^T
  dgemm(st, tb, ta, N, M, K, alpha, B, ldb, 0, A, lda, 0, beta, C, ldc, 0, 1, nullptr);
}

}  // namespace seqx
