// Batched CIS Davidson (batched outline of the paper's GPU-implementation
// subsection and its Fig. 2) for many small molecules of uneven size.
//
// The paper pads every molecule to the largest and runs dense batched tensor
// operations.  Here nothing is padded: a (molecule, trial vector) pair is a
// work item, and one persistent launch of a fused kernel forms all products of
// an iteration.  Each 256-thread workgroup takes items in a static round-robin
// over a list ordered by molecule size (largest first), and for one item runs
// Eqs. 8-9 end to end:
//   T = C_o V,  R = T C_v^T           (workgroup MFMA GEMMs)
//   F = 2 J(R) - K(R)                 (packed Coulomb, one-centre and pair exchange)
//   Z = F C_v,  A V = C_o^T Z + de V  (workgroup MFMA GEMMs, FP64 epilogue)
// with R, F and T/Z in a per-workgroup slice of global scratch (L2-resident).
// The subspace steps (projection, Jacobi eigensolve, Ritz vectors and
// residuals, preconditioning, collapse, Gram-Schmidt) are one launch each over
// all molecules, with per-molecule flags on the device, so the iteration is a
// fixed sequence of launches (captured once as a HIP graph); the host reads one
// counter per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "batch.hpp"
#include "wave.hpp"
#include "fock_blocks.hpp"
#include "jacobi.hpp"
#include "linalg.hpp"

namespace seqx {

static_assert(kBatchMaxSub <= kJacobiMax, "the batched subspace must fit the LDS eigensolver");

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <class T>
struct WgMfma;
template <>
struct WgMfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct WgMfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Workgroup GEMM (4 wavefronts): out(i, j) = sum_k A(i, k) B(k, j) for i < M,
// j < N, with A(i, k) = A[i sai + k sak] and B(k, j) = B[k sbk + j sbj] (any
// transposition through the strides).  Each wave owns macro tiles of
// (16 TM) x (16 TN) in round-robin; operands come straight from global memory
// (L1/L2) in the MFMA lane layout; store(i, j, value) writes the result.
template <class T, int TM, int TN, class TA, class TB, class Store>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, const TA* __restrict__ A, long sai, long sak,
                                        const TB* __restrict__ B, long sbk, long sbj, Store store) {
  typedef WgMfma<T> MF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int tm = (M + 16 * TM - 1) / (16 * TM), tn = (N + 16 * TN - 1) / (16 * TN);
  const int nwave = blockDim.x >> 6;
  for (int t = wave; t < tm * tn; t += nwave) {
    const int i0 = (t / tn) * 16 * TM, j0 = (t % tn) * 16 * TN;
    typename MF::acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};
    // four k-steps per pass, all loads first (the loads past K read zero, so
    // no remainder loop is needed)
    for (int k0 = 0; k0 < K; k0 += 16) {
      T a[4][TM], b[4][TN];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 4 * q + k4;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int row = i0 + i * 16 + r16;
          a[q][i] = (row < M && k < K) ? static_cast<T>(A[row * sai + k * sak]) : T(0);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = j0 + j * 16 + r16;
          b[q][j] = (col < N && k < K) ? static_cast<T>(B[k * sbk + col * sbj]) : T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[q][i], b[q][j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + i * 16 + MF::row(lane, r), col = j0 + j * 16 + r16;
          if (row < M && col < N) store(row, col, static_cast<double>(acc[i][j][r]));
        }
  }
}

constexpr int kSigThreads = 256;  // threads per work item (512 measured slower: the phases are latency-bound)

// One CIS product A V for one trial vector of one molecule (whole workgroup).
// scr: n*n (R) + n*n (F) + n*v (T, then Z) elements of T; rs, js: LDS [np].
template <class T, int TM, int TN>
__device__ void sigma_item(const MolDesc& md, const T* __restrict__ C, const double* __restrict__ V,
                           double* __restrict__ out, T* __restrict__ scr, double* rs, double* js) {
  const int n = md.n, o = md.o, v = md.v, np = md.np;
  T* R = scr;
  T* F = scr + static_cast<long>(n) * n;
  T* Tz = scr + 2L * n * n;
  // T (n x v) = C[:, :o] V
  wg_gemm<T, TM, TN>(n, v, o, C, n, 1, V, v, 1,
                     [&](int i, int j, double x) { Tz[static_cast<long>(i) * v + j] = static_cast<T>(x); });
  __syncthreads();
  // R (n x n) = T C[:, o:]^T
  wg_gemm<T, TM, TN>(n, n, v, Tz, v, 1, C + o, 1, n,
                     [&](int i, int j, double x) { R[static_cast<long>(i) * n + j] = static_cast<T>(x); });
  __syncthreads();
  // packed same-atom densities r_P and Coulomb J = W r (one wave per row, fixed-order reduction)
  for (int P = threadIdx.x; P < np; P += blockDim.x) {
    const int mu = md.pi_mu[P], nu = md.pi_nu[P];
    const double a = static_cast<double>(R[static_cast<long>(mu) * n + nu]);
    const double b = static_cast<double>(R[static_cast<long>(nu) * n + mu]);
    rs[P] = (mu == nu) ? a : a + b;
  }
  __syncthreads();
  // J[P] = sum_Q W[Q][P] r[Q] (W symmetric): thread P walks column P, so each
  // step reads one row of W coalesced and no cross-lane sum is needed
  for (int P0 = 0; P0 < np; P0 += blockDim.x) {
    const int P = P0 + threadIdx.x;
    const double* Wc = md.W + min(P, np - 1);
    double s0 = 0.0, s1 = 0.0;
    int Q = 0;
    for (; Q + 2 <= np; Q += 2) {
      s0 += Wc[static_cast<long>(Q) * np] * rs[Q];
      s1 += Wc[static_cast<long>(Q + 1) * np] * rs[Q + 1];
    }
    if (Q < np) s0 += Wc[static_cast<long>(Q) * np] * rs[Q];
    if (P < np) js[P] = s0 + s1;
  }
  __syncthreads();
  // F = 2 J(R) - K(R): atom-diagonal blocks, then every atom pair (both orders)
  for (int A = threadIdx.x; A < md.natoms; A += blockDim.x)
    diag_block<kSum, T, T>(md.elems[md.slot[A]], md.ao_off[A], md.pi_off[A], js, 1, R, n, F, static_cast<T*>(nullptr),
                           2.0, -1.0, -1.0);
  for (int p = threadIdx.x; p < md.npairs[0]; p += blockDim.x)
    exchange_pair<4, 4, kSum, T, T>(md.pairs[0][p].x, md.pairs[0][p].y, md.ao_off, md.pi_off, md.W, np, R, n, F,
                                    static_cast<T*>(nullptr), -1.0, -1.0);
  for (int p = threadIdx.x; p < md.npairs[1]; p += blockDim.x)
    exchange_pair<4, 1, kSum, T, T>(md.pairs[1][p].x, md.pairs[1][p].y, md.ao_off, md.pi_off, md.W, np, R, n, F,
                                    static_cast<T*>(nullptr), -1.0, -1.0);
  for (int p = threadIdx.x; p < md.npairs[2]; p += blockDim.x)
    exchange_pair<1, 1, kSum, T, T>(md.pairs[2][p].x, md.pairs[2][p].y, md.ao_off, md.pi_off, md.W, np, R, n, F,
                                    static_cast<T*>(nullptr), -1.0, -1.0);
  __syncthreads();
  // Z (n x v) = F C[:, o:]
  wg_gemm<T, TM, TN>(n, v, n, F, n, 1, C + o, n, 1,
                     [&](int i, int j, double x) { Tz[static_cast<long>(i) * v + j] = static_cast<T>(x); });
  __syncthreads();
  // A V (o x v) = C[:, :o]^T Z + (eps_a - eps_i) V, the diagonal term in FP64
  const double* eps = md.eps;
  wg_gemm<T, TM, TN>(o, v, n, C, 1, n, Tz, v, 1, [&](int i, int j, double x) {
    const long ij = static_cast<long>(i) * v + j;
    out[ij] = x + (eps[o + j] - eps[i]) * V[ij];
  });
  __syncthreads();
}

// counters: [0] number of items, [1] active molecules, [2] iteration
template <class T>
__global__ void __launch_bounds__(kSigThreads) sigma_items_kernel(const MolDesc* __restrict__ mols,
                                                          const int2* __restrict__ items, const int* __restrict__ counters,
                                                          const double* __restrict__ Vp, double* __restrict__ AVp,
                                                          T* __restrict__ scratch, long scratch_stride,
                                                          long long* __restrict__ stamps) {
  __shared__ double rs[kBatchMaxNp];
  __shared__ double js[kBatchMaxNp];
  if (threadIdx.x == 0) stamps[2 * blockIdx.x] = static_cast<long long>(wall_clock64());
  const int nit = counters[0];
  T* scr = scratch + blockIdx.x * scratch_stride;
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    const int2 item = items[it];
    const MolDesc md = mols[item.x];
    const T* C = sizeof(T) == 4 ? reinterpret_cast<const T*>(md.C32) : reinterpret_cast<const T*>(md.C64);
    const double* V = Vp + md.vbase + item.y * md.nov;
    double* out = AVp + md.vbase + item.y * md.nov;
    switch (md.variant) {
      case 0: sigma_item<T, 1, 1>(md, C, V, out, scr, rs, js); break;
      case 1: sigma_item<T, 2, 1>(md, C, V, out, scr, rs, js); break;
      default: sigma_item<T, 2, 2>(md, C, V, out, scr, rs, js); break;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) stamps[2 * blockIdx.x + 1] = static_cast<long long>(wall_clock64());
}

// Span of the last sigma launch (latest end - earliest start over its
// workgroups, device wall-clock ticks), added to acc[0]; fixed-order reduction.
__global__ void __launch_bounds__(256) stamp_span_kernel(int G, const long long* __restrict__ stamps,
                                                         long long* acc) {
  __shared__ long long lo[256], hi[256];
  long long a = 0x7fffffffffffffffLL, b = 0;
  for (int i = threadIdx.x; i < G; i += 256) {
    a = min(a, stamps[2 * i]);
    b = max(b, stamps[2 * i + 1]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
      hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += hi[0] - lo[0];
}

// ---------------------------------------------------------------- subspace kernels

__device__ __forceinline__ double wave_sum(double s) { return wave_sum64(s); }

// fixed-order block sum over 256 threads (result valid in every thread)
__device__ double block_sum(double s, double* red) {  // 256 threads; fixed order
  s = wave_sum64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Gap guess: unit vectors at the ng = min(nov, 2K) smallest eps_a - eps_i
// (ties by flat index i*v + a), found by ng rounds of lexicographic minimum.
__global__ void __launch_bounds__(256) guess_kernel(int nmol, const MolDesc* __restrict__ mols, int K,
                                                    double* __restrict__ Vp, int* S, int* knew, int* active, int* conv,
                                                    int* coll, int* qcol, int* evn) {
  __shared__ double bg[256];
  __shared__ long bi[256];
  const int m = blockIdx.x;
  const MolDesc md = mols[m];
  const long nov = md.nov;
  const int ng = static_cast<int>(nov < 2L * K ? nov : 2L * K);
  double* V = Vp + md.vbase;
  for (long x = threadIdx.x; x < ng * nov; x += 256) V[x] = 0.0;
  __syncthreads();
  double lg = -1e300;
  long li = -1;
  for (int r = 0; r < ng; ++r) {
    double g = 1e300;
    long gi = nov;
    for (long x = threadIdx.x; x < nov; x += 256) {
      const double d = md.eps[md.o + x % md.v] - md.eps[x / md.v];
      const bool after = d > lg || (d == lg && x > li);
      if (after && (d < g || (d == g && x < gi))) {
        g = d;
        gi = x;
      }
    }
    bg[threadIdx.x] = g;
    bi[threadIdx.x] = gi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) {
        const double g2 = bg[threadIdx.x + h];
        const long i2 = bi[threadIdx.x + h];
        if (g2 < bg[threadIdx.x] || (g2 == bg[threadIdx.x] && i2 < bi[threadIdx.x])) {
          bg[threadIdx.x] = g2;
          bi[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    lg = bg[0];
    li = bi[0];
    if (threadIdx.x == 0) V[r * nov + li] = 1.0;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S[m] = 0;
    knew[m] = ng;
    active[m] = 1;
    conv[m] = 0;
    coll[m] = 0;
    qcol[m] = 0;
    evn[m] = 0;
  }
}

// Work list of the iteration: items (m, S_m + j), j < knew_m, molecules in
// the size order `order` (largest first); block-wide exclusive scan.
__global__ void __launch_bounds__(256) items_kernel(int nmol, const MolDesc* __restrict__ mols,
                                                    const int* __restrict__ order, const int* __restrict__ S,
                                                    const int* __restrict__ knew, const int* __restrict__ active,
                                                    int2* __restrict__ items, int* counters, long long* nsig) {
  __shared__ int part[256];
  __shared__ long long fl[256];
  const int per = (nmol + 255) / 256;
  const int b0 = threadIdx.x * per, b1 = min(nmol, b0 + per);
  int cnt = 0;
  long long flops = 0;  // algorithmic transform flops of the items: 4 n v (n + o) each
  for (int q = b0; q < b1; ++q) {
    const int m = order[q];
    if (active[m]) {
      cnt += knew[m];
      const long long n = mols[m].n, o = mols[m].o, v = mols[m].v;
      flops += knew[m] * 4LL * n * v * (n + o);
    }
  }
  part[threadIdx.x] = cnt;
  fl[threadIdx.x] = flops;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) fl[threadIdx.x] += fl[threadIdx.x + h];
    __syncthreads();
  }
  for (int h = 1; h < 256; h <<= 1) {  // inclusive Hillis-Steele scan
    const int add = threadIdx.x >= h ? part[threadIdx.x - h] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int pos = part[threadIdx.x] - cnt;
  for (int q = b0; q < b1; ++q) {
    const int m = order[q];
    if (!active[m]) continue;
    for (int j = 0; j < knew[m]; ++j) items[pos++] = make_int2(m, S[m] + j);
  }
  if (threadIdx.x == 255) {
    counters[0] = part[255];
    nsig[0] += part[255];
    nsig[2] += fl[0];
  }
}

// Subspace steps of a molecule are split over kXChunks blocks along the nov
// entries, so that the largest molecules spread over several CUs; partial
// inner products go to per-chunk slots and are summed in a fixed order.
constexpr int kXChunks = 8;
constexpr int kPartStride = kBatchMaxSub * 2 * kBatchMaxRoots;  // one chunk's [s][j] partials

__device__ __forceinline__ long chunk_begin(long nov, int ch) { return nov * ch / kXChunks; }

// Inner products over x in [x0, x1) of up to 16 vectors b_u (nb of them) with
// the rows s0, s0 + 1 of V (rows past ns repeat the last), one wavefront: each
// V element is read once, the b_u stay in L1/L2.  Results in every lane: d[i][u].
__device__ __forceinline__ void wave_dots2x16(const double* __restrict__ V, long nov, int s0, int ns, long x0,
                                              long x1, const double* const* b, int nb,
                                              double (*d)[kBatchMaxRoots]) {
  const int lane = threadIdx.x & 63;
  const double* a0 = V + static_cast<long>(min(s0, ns - 1)) * nov;
  const double* a1 = V + static_cast<long>(min(s0 + 1, ns - 1)) * nov;
  double acc[2][kBatchMaxRoots];
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u) acc[0][u] = acc[1][u] = 0.0;
  for (long x = x0 + lane; x < x1; x += 64) {
    const double v0 = a0[x], v1 = a1[x];
#pragma unroll
    for (int u = 0; u < kBatchMaxRoots; ++u)
      if (u < nb) {
        const double bx = b[u][x];
        acc[0][u] += v0 * bx;
        acc[1][u] += v1 * bx;
      }
  }
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u)
    if (u < nb) {
      d[0][u] = wave_sum(acc[0][u]);
      d[1][u] = wave_sum(acc[1][u]);
    }
}

// New columns of M = V^T A V, first half: block (m, c) forms the partial
// inner products over chunk c of every new product A V_j (j < knew_m, in
// groups of 16) with every basis row s < S_m + knew_m.
__global__ void __launch_bounds__(256) project_part_kernel(const MolDesc* __restrict__ mols,
                                                           const double* __restrict__ Vp,
                                                           const double* __restrict__ AVp, const int* __restrict__ S,
                                                           const int* __restrict__ knew,
                                                           const int* __restrict__ active, double* __restrict__ part) {
  const int m = blockIdx.x, ch = blockIdx.y;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov, x0 = chunk_begin(nov, ch), x1 = chunk_begin(nov, ch + 1);
  const int S0 = S[m], kn = knew[m], ns = S0 + kn;
  const double* V = Vp + md.vbase;
  double* P = part + (static_cast<long>(m) * kXChunks + ch) * kPartStride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j0 = 0; j0 < kn; j0 += kBatchMaxRoots) {
    const int nb = min(kBatchMaxRoots, kn - j0);
    const double* b[kBatchMaxRoots];
#pragma unroll
    for (int u = 0; u < kBatchMaxRoots; ++u) b[u] = AVp + md.vbase + static_cast<long>(S0 + j0 + min(u, nb - 1)) * nov;
    for (int s0 = 2 * wave; s0 < ns; s0 += 8) {
      double d[2][kBatchMaxRoots];
      wave_dots2x16(V, nov, s0, ns, x0, x1, b, nb, d);
      if (lane == 0)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int u = 0; u < kBatchMaxRoots; ++u)
            if (u < nb && s0 + i < ns) P[(s0 + i) * 2 * kBatchMaxRoots + j0 + u] = d[i][u];
    }
  }
}

// Second half: sum the chunks in order and write both triangles of the new
// columns (column-major, ld Smax).  S is advanced by advance_kernel afterwards.
__global__ void __launch_bounds__(256) project_kernel(int Smax, const double* __restrict__ part,
                                                      double* __restrict__ Mp, const int* __restrict__ S,
                                                      const int* __restrict__ knew, const int* __restrict__ active) {
  const int m = blockIdx.x;
  if (!active[m]) return;
  const int S0 = S[m], kn = knew[m], ns = S0 + kn;
  double* M = Mp + static_cast<long>(m) * Smax * Smax;
  const double* P = part + static_cast<long>(m) * kXChunks * kPartStride;
  for (int idx = threadIdx.x; idx < ns * kn; idx += 256) {
    const int sidx = idx / kn, jn = idx % kn, j = S0 + jn;
    if (sidx > j) continue;
    double d = 0.0;
    for (int c = 0; c < kXChunks; ++c) d += P[c * kPartStride + sidx * 2 * kBatchMaxRoots + jn];
    M[sidx + static_cast<long>(j) * Smax] = d;
    M[j + static_cast<long>(sidx) * Smax] = d;
  }
}

__global__ void advance_kernel(int nmol, int* S, const int* __restrict__ knew, const int* __restrict__ active) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nmol && active[m]) S[m] += knew[m];
}

// Symmetric eigensolve of the S x S projected matrix of each molecule
// (Jacobi in LDS, jacobi.hpp).  Eigenvalues ascending in eval, eigenvectors
// as columns of evec (ld Smax).  Warm start: the leading evn x evn block of M
// is unchanged since the last eigensolve, whose eigenvectors are still in
// evec, so M is first rotated into that basis (extended by the identity for
// the new columns) and Jacobi continues from the nearly diagonal result,
// accumulating onto the same basis.
constexpr int kEigThreads = 256;  // measured faster than one wavefront per molecule

__global__ void __launch_bounds__(kEigThreads) eig_kernel(int Smax, const double* __restrict__ Mp,
                                                          const int* __restrict__ S, const int* __restrict__ active,
                                                          int* __restrict__ evn, double* __restrict__ evec,
                                                          double* __restrict__ eval) {
  __shared__ JacobiLds L;
  const int m = blockIdx.x;
  if (!active[m]) return;
  const int n = S[m];
  const int p = min(evn[m], n);
  const double* M = Mp + static_cast<long>(m) * Smax * Smax;
  double* ev = evec + static_cast<long>(m) * Smax * Smax;
  constexpr int kPer = (kJacobiMax * kJacobiMax + kEigThreads - 1) / kEigThreads;
  for (int idx = threadIdx.x; idx < n * n; idx += kEigThreads) {
    const int i = idx / n, j = idx % n;
    L.A[i][j] = M[i + static_cast<long>(j) * Smax];
    L.Q[i][j] = (i < p && j < p) ? ev[i + static_cast<long>(j) * Smax] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (p > 0) {
    // T = M Q (only the first p columns change), then A = Q^T T (only the first p rows change)
    double t[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + kEigThreads * e;
      t[e] = 0.0;
      if (idx < n * n) {
        const int i = idx / n, j = idx % n;
        if (j < p) {
          for (int k = 0; k < p; ++k) t[e] += L.A[i][k] * L.Q[k][j];
        } else {
          t[e] = L.A[i][j];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + kEigThreads * e;
      if (idx < n * n) L.A[idx / n][idx % n] = t[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + kEigThreads * e;
      t[e] = 0.0;
      if (idx < n * n) {
        const int i = idx / n, j = idx % n;
        if (i < p) {
          for (int k = 0; k < p; ++k) t[e] += L.Q[k][i] * L.A[k][j];
        } else {
          t[e] = L.A[i][j];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + kEigThreads * e;
      if (idx < n * n) L.A[idx / n][idx % n] = t[e];
    }
    __syncthreads();
  }
  jacobi_lds<kEigThreads>(n, L, true);
  for (int idx = threadIdx.x; idx < n * n; idx += kEigThreads) {
    const int r = idx / n, i = idx % n;
    ev[i + static_cast<long>(r) * Smax] = L.Q[i][L.perm[r]];
  }
  for (int r = threadIdx.x; r < n; r += kEigThreads) eval[static_cast<long>(m) * Smax + r] = L.A[L.perm[r]][L.perm[r]];
  if (threadIdx.x == 0) evn[m] = n;
}

// Ritz vectors of molecule m, X_j = sum_s evec(s, j) V_s, and residuals
// r_j = A X_j - w_j X_j into Wc, for all K roots in one pass over V and A V
// (each basis element read once); block (m, c) takes chunk c of the nov
// entries and leaves its partial sums of |r_j|^2 in rpart[m][c][j].
__global__ void __launch_bounds__(256) ritz_kernel(const MolDesc* __restrict__ mols, int K, int Smax,
                                                   const double* __restrict__ Vp, const double* __restrict__ AVp,
                                                   const double* __restrict__ evec, const double* __restrict__ eval,
                                                   const int* __restrict__ S, const int* __restrict__ active,
                                                   double* __restrict__ Xp, double* __restrict__ Wcp,
                                                   double* __restrict__ omega, double* __restrict__ rpart) {
  __shared__ double c[kBatchMaxRoots][kBatchMaxSub];
  __shared__ double wr[kBatchMaxRoots];
  __shared__ double red[4][kBatchMaxRoots];
  const int m = blockIdx.x, ch = blockIdx.y;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov;
  const int n = S[m];
  for (int idx = threadIdx.x; idx < K * n; idx += 256) {
    const int j = idx / n, sidx = idx % n;
    c[j][sidx] = evec[static_cast<long>(m) * Smax * Smax + sidx + static_cast<long>(j) * Smax];
  }
  if (threadIdx.x < K) wr[threadIdx.x] = eval[static_cast<long>(m) * Smax + threadIdx.x];
  __syncthreads();
  const double* V = Vp + md.vbase;
  const double* AV = AVp + md.vbase;
  double* X = Xp + md.xbase;
  double* Wc = Wcp + md.xbase;
  const long x0 = chunk_begin(nov, ch), x1 = chunk_begin(nov, ch + 1);
  double ss[kBatchMaxRoots];
#pragma unroll
  for (int j = 0; j < kBatchMaxRoots; ++j) ss[j] = 0.0;
  for (long x = x0 + threadIdx.x; x < x1; x += 256) {
    double xv[kBatchMaxRoots], av[kBatchMaxRoots];
#pragma unroll
    for (int j = 0; j < kBatchMaxRoots; ++j) xv[j] = av[j] = 0.0;
    for (int sidx = 0; sidx < n; ++sidx) {
      const double v = V[sidx * nov + x], a = AV[sidx * nov + x];
#pragma unroll
      for (int j = 0; j < kBatchMaxRoots; ++j)
        if (j < K) {
          xv[j] += c[j][sidx] * v;
          av[j] += c[j][sidx] * a;
        }
    }
#pragma unroll
    for (int j = 0; j < kBatchMaxRoots; ++j)
      if (j < K) {
        const double r = av[j] - wr[j] * xv[j];
        X[j * nov + x] = xv[j];
        Wc[j * nov + x] = r;
        ss[j] += r * r;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kBatchMaxRoots; ++j)
    if (j < K) {
      const double t = wave_sum(ss[j]);
      if (lane == 0) red[wave][j] = t;
    }
  __syncthreads();
  if (threadIdx.x < K)
    rpart[(static_cast<long>(m) * kXChunks + ch) * kBatchMaxRoots + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
  if (ch == 0 && threadIdx.x < K) omega[m * K + threadIdx.x] = wr[threadIdx.x];
}

// Convergence and bookkeeping for every molecule; counts the active ones.
__global__ void __launch_bounds__(256) select_kernel(int nmol, int K, int Smax, double tol,
                                                     const double* __restrict__ rpart, double* __restrict__ rnorm,
                                                     const int* __restrict__ S, int* knew, int* active, int* coll,
                                                     int* qcol, int* unc, int* conv, int* counters) {
  __shared__ double red[256];
  const int iter = counters[2] + 1;
  double nact = 0.0;
  for (int m = threadIdx.x; m < nmol; m += 256) {
    if (!active[m]) continue;
    int nu = 0;
    for (int j = 0; j < K; ++j) {
      double r2 = 0.0;
      for (int c = 0; c < kXChunks; ++c) r2 += rpart[(static_cast<long>(m) * kXChunks + c) * kBatchMaxRoots + j];
      const double rn = sqrt(r2);
      rnorm[m * K + j] = rn;
      if (rn > tol) unc[m * K + nu++] = j;
    }
    if (nu == 0) {
      active[m] = 0;
      conv[m] = iter;
      continue;
    }
    knew[m] = nu;
    coll[m] = S[m] + nu > Smax ? 1 : 0;
    qcol[m] = min(2 * K, S[m]);
    nact += 1.0;
  }
  nact = block_sum(nact, red);
  if (threadIdx.x == 0) {
    counters[1] = static_cast<int>(nact);
    counters[2] = iter;
  }
}

// Collapse onto the q lowest Ritz vectors: TV_s = sum_t evec(t, s) V_t (and A V).
__global__ void __launch_bounds__(256) collapse_kernel(const MolDesc* __restrict__ mols, int Smax,
                                                       const double* __restrict__ Vp, const double* __restrict__ AVp,
                                                       const double* __restrict__ evec, const int* __restrict__ S,
                                                       const int* __restrict__ coll, const int* __restrict__ qcol,
                                                       double* __restrict__ TVp, double* __restrict__ TAVp) {
  __shared__ double c[kBatchMaxSub];
  const int m = blockIdx.x, s = blockIdx.y;
  if (!coll[m] || s >= qcol[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov;
  const int n = S[m];
  for (int t = threadIdx.x; t < n; t += 256) c[t] = evec[static_cast<long>(m) * Smax * Smax + t + static_cast<long>(s) * Smax];
  __syncthreads();
  const double* V = Vp + md.vbase;
  const double* AV = AVp + md.vbase;
  double* TV = TVp + md.tbase + s * nov;
  double* TAV = TAVp + md.tbase + s * nov;
  for (long x = threadIdx.x; x < nov; x += 256) {
    double a = 0.0, b = 0.0;
    for (int t = 0; t < n; ++t) {
      a += c[t] * V[t * nov + x];
      b += c[t] * AV[t * nov + x];
    }
    TV[x] = a;
    TAV[x] = b;
  }
}

// Second half of the collapse: copy back, M = diag(lowest q eigenvalues), S = q.
__global__ void __launch_bounds__(256) collapse_copy_kernel(const MolDesc* __restrict__ mols, int Smax,
                                                            const double* __restrict__ TVp,
                                                            const double* __restrict__ TAVp,
                                                            const double* __restrict__ eval, int* S, int* coll,
                                                            const int* __restrict__ qcol, double* __restrict__ Vp,
                                                            double* __restrict__ AVp, double* __restrict__ Mp,
                                                            int* __restrict__ evn) {
  const int m = blockIdx.x, s = blockIdx.y;
  if (!coll[m]) return;
  const int q = qcol[m];
  if (s > q) return;
  const MolDesc md = mols[m];
  const long nov = md.nov;
  if (s < q) {
    for (long x = threadIdx.x; x < nov; x += 256) {
      Vp[md.vbase + s * nov + x] = TVp[md.tbase + s * nov + x];
      AVp[md.vbase + s * nov + x] = TAVp[md.tbase + s * nov + x];
    }
  } else {  // block s == q: the projected matrix (diagonal: no previous eigenvectors to start from)
    if (threadIdx.x == 0) evn[m] = 0;
    double* M = Mp + static_cast<long>(m) * Smax * Smax;
    for (int idx = threadIdx.x; idx < q * q; idx += 256) {
      const int i = idx / q, j = idx % q;
      M[i + static_cast<long>(j) * Smax] = (i == j) ? eval[static_cast<long>(m) * Smax + i] : 0.0;
    }
  }
}

// Corrections of the unconverged roots, first step: precondition the
// residuals in place, r / (w - de) with |w - de| kept >= 1e-8, and leave the
// partial sums of their squared norms per chunk (the norms before deflation).
__global__ void __launch_bounds__(256) precond_kernel(const MolDesc* __restrict__ mols, int K,
                                                      double* __restrict__ Wcp, const int* __restrict__ knew,
                                                      const int* __restrict__ active, const int* __restrict__ unc,
                                                      const double* __restrict__ omega, double* __restrict__ n0part) {
  __shared__ double wu[kBatchMaxRoots];
  __shared__ double red[4][kBatchMaxRoots];
  const int m = blockIdx.x, ch = blockIdx.y;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov, x0 = chunk_begin(nov, ch), x1 = chunk_begin(nov, ch + 1);
  const int nu = knew[m];
  double* w[kBatchMaxRoots];
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u) w[u] = Wcp + md.xbase + unc[m * K + min(u, nu - 1)] * nov;
  if (threadIdx.x < nu) wu[threadIdx.x] = omega[m * K + unc[m * K + threadIdx.x]];
  __syncthreads();
  double n0[kBatchMaxRoots];
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u) n0[u] = 0.0;
  for (long x = x0 + threadIdx.x; x < x1; x += 256) {
    const double de = md.eps[md.o + x % md.v] - md.eps[x / md.v];
#pragma unroll
    for (int u = 0; u < kBatchMaxRoots; ++u)
      if (u < nu) {
        double den = wu[u] - de;
        if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
        const double t = w[u][x] / den;
        w[u][x] = t;
        n0[u] += t * t;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u)
    if (u < nu) {
      const double t = wave_sum(n0[u]);
      if (lane == 0) red[wave][u] = t;
    }
  __syncthreads();
  if (threadIdx.x < nu)
    n0part[(static_cast<long>(m) * kXChunks + ch) * kBatchMaxRoots + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// Classical Gram-Schmidt of the corrections against the basis (its first
// qcol rows after a collapse), one half-pass each: partial inner products
// per chunk ...
__global__ void __launch_bounds__(256) gs_dots_kernel(const MolDesc* __restrict__ mols, int K,
                                                      const double* __restrict__ Vp, const double* __restrict__ Wcp,
                                                      const int* __restrict__ S, const int* __restrict__ knew,
                                                      const int* __restrict__ active, const int* __restrict__ coll,
                                                      const int* __restrict__ qcol, const int* __restrict__ unc,
                                                      double* __restrict__ part) {
  const int m = blockIdx.x, ch = blockIdx.y;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov, x0 = chunk_begin(nov, ch), x1 = chunk_begin(nov, ch + 1);
  const int nb = coll[m] ? qcol[m] : S[m];
  const int nu = knew[m];
  const double* w[kBatchMaxRoots];
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u) w[u] = Wcp + md.xbase + unc[m * K + min(u, nu - 1)] * nov;
  double* P = part + (static_cast<long>(m) * kXChunks + ch) * kPartStride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int s0 = 2 * wave; s0 < nb; s0 += 8) {
    double d[2][kBatchMaxRoots];
    wave_dots2x16(Vp + md.vbase, nov, s0, nb, x0, x1, w, nu, d);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int u = 0; u < kBatchMaxRoots; ++u)
          if (u < nu && s0 + i < nb) P[(s0 + i) * 2 * kBatchMaxRoots + u] = d[i][u];
  }
}

// ... then the update of chunk c: h = the inner products summed over the
// chunks in order, w_u -= sum_s h[s][u] V_s.
__global__ void __launch_bounds__(256) gs_update_kernel(const MolDesc* __restrict__ mols, int K,
                                                        const double* __restrict__ Vp, double* __restrict__ Wcp,
                                                        const int* __restrict__ S, const int* __restrict__ knew,
                                                        const int* __restrict__ active, const int* __restrict__ coll,
                                                        const int* __restrict__ qcol, const int* __restrict__ unc,
                                                        const double* __restrict__ part) {
  __shared__ double h[kBatchMaxSub][kBatchMaxRoots];
  const int m = blockIdx.x, ch = blockIdx.y;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov, x0 = chunk_begin(nov, ch), x1 = chunk_begin(nov, ch + 1);
  const int nb = coll[m] ? qcol[m] : S[m];
  const int nu = knew[m];
  const double* P = part + static_cast<long>(m) * kXChunks * kPartStride;
  for (int idx = threadIdx.x; idx < nb * nu; idx += 256) {
    const int sidx = idx / nu, u = idx % nu;
    double d = 0.0;
    for (int c = 0; c < kXChunks; ++c) d += P[c * kPartStride + sidx * 2 * kBatchMaxRoots + u];
    h[sidx][u] = d;
  }
  __syncthreads();
  const double* V = Vp + md.vbase;
  double* w[kBatchMaxRoots];
#pragma unroll
  for (int u = 0; u < kBatchMaxRoots; ++u) w[u] = Wcp + md.xbase + unc[m * K + min(u, nu - 1)] * nov;
  for (long x = x0 + threadIdx.x; x < x1; x += 256) {
    double t[kBatchMaxRoots];
#pragma unroll
    for (int u = 0; u < kBatchMaxRoots; ++u) t[u] = u < nu ? w[u][x] : 0.0;
    for (int sidx = 0; sidx < nb; ++sidx) {
      const double v = V[sidx * nov + x];
#pragma unroll
      for (int u = 0; u < kBatchMaxRoots; ++u)
        if (u < nu) t[u] -= h[sidx][u] * v;
    }
#pragma unroll
    for (int u = 0; u < kBatchMaxRoots; ++u)
      if (u < nu) w[u][x] = t[u];
  }
}

// Orthonormalise the deflated corrections among themselves (modified
// Gram-Schmidt, twice) and append the survivors (norm above 1e-8 of the
// correction's norm before deflation) to the basis.
__global__ void __launch_bounds__(256) append_kernel(const MolDesc* __restrict__ mols, int K, int Smax,
                                                     double* __restrict__ Vp, double* __restrict__ Wcp, int* S,
                                                     int* knew, int* active, int* coll, const int* __restrict__ qcol,
                                                     const int* __restrict__ unc, int* conv,
                                                     const int* __restrict__ counters,
                                                     const double* __restrict__ n0part) {
  __shared__ double red[256];
  const int m = blockIdx.x;
  if (!active[m]) return;
  const MolDesc md = mols[m];
  const long nov = md.nov;
  const int S0 = coll[m] ? qcol[m] : S[m];
  const int nu = knew[m];
  double* V = Vp + md.vbase;
  int acc = 0;
  for (int u = 0; u < nu; ++u) {
    if (S0 + acc >= Smax) break;
    double* w = Wcp + md.xbase + unc[m * K + u] * nov;
    for (int pass = 0; pass < 2; ++pass)
      for (int t = 0; t < acc; ++t) {
        const double* a = V + static_cast<long>(S0 + t) * nov;
        double d = 0.0;
        for (long x = threadIdx.x; x < nov; x += 256) d += a[x] * w[x];
        d = block_sum(d, red);
        for (long x = threadIdx.x; x < nov; x += 256) w[x] -= d * a[x];
        __syncthreads();
      }
    double nw = 0.0;
    for (long x = threadIdx.x; x < nov; x += 256) nw += w[x] * w[x];
    nw = sqrt(block_sum(nw, red));
    double n02 = 0.0;
    for (int c = 0; c < kXChunks; ++c) n02 += n0part[(static_cast<long>(m) * kXChunks + c) * kBatchMaxRoots + u];
    if (nw > 1e-8 * sqrt(n02) && nw > 1e-14) {
      double* dst = V + static_cast<long>(S0 + acc) * nov;
      const double inv = 1.0 / nw;
      for (long x = threadIdx.x; x < nov; x += 256) dst[x] = w[x] * inv;
      ++acc;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    S[m] = S0;
    coll[m] = 0;
    knew[m] = acc;
    if (acc == 0) {  // no new direction: stop this molecule (flagged by a negative iteration)
      active[m] = 0;
      conv[m] = -counters[2];
    }
  }
}

int bucket_of(int n) { return n < 32 ? 0 : n < 64 ? 1 : n < 96 ? 2 : n < 128 ? 3 : 4; }

double ms_between(hipEvent_t a, hipEvent_t b) {
  float t = 0.f;
  SEQX_HIP(hipEventElapsedTime(&t, a, b));
  return t;
}

}  // namespace

BatchWork::~BatchWork() {
  if (stream) (void)hipStreamDestroy(stream);
}

BatchResult batched_cis(const std::vector<DeviceMolecule*>& mols, const BatchOptions& opt, BatchWork& w,
                        TileTuning& tune, SigmaWork& sig, hipStream_t user_stream) {
  const int nmol = static_cast<int>(mols.size());
  const int K = opt.nroots;
  const bool f32 = opt.precision == kPrecFP32;
  if (opt.precision != kPrecFP32 && opt.precision != kPrecFP64)
    throw Error(kEArg, "batched solve supports FP32 and FP64 products");
  if (K < 1 || K > kBatchMaxRoots) throw Error(kEArg, "batched solve supports 1 to 16 roots");
  int Smax = opt.max_sub > 0 ? opt.max_sub : 8 * K;
  Smax = std::min(std::max(Smax, 3 * K), kBatchMaxSub);
  if (Smax < 3 * K) throw Error(kEArg, "batched solve: subspace cap below 3 * nroots");
  BatchResult res;
  if (!w.stream) SEQX_HIP(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
  hipStream_t st = w.stream;

  // ---- molecule table, ordering and pools
  std::vector<MolDesc> h(nmol);
  long vtot = 0, xtot = 0, ttot = 0, scr = 0;
  int maxnew = 2 * K;
  for (int m = 0; m < nmol; ++m) {
    const DeviceMolecule& d = *mols[m];
    const long nov = static_cast<long>(d.nocc) * d.nvirt;
    if (nov < K) throw Error(kEArg, "nroots exceeds nocc*nvirt of a molecule");
    if (d.np > kBatchMaxNp) throw Error(kEArg, "molecule too large for the batched solver (pair indices > 1536)");
    if (d.C32.n < static_cast<size_t>(d.nao) * d.nao) throw Error(kEState, "FP32 MO coefficients missing");
    MolDesc& md = h[m];
    md.n = d.nao;
    md.o = d.nocc;
    md.v = d.nvirt;
    md.np = d.np;
    md.natoms = d.natoms;
    for (int g = 0; g < 3; ++g) {
      md.npairs[g] = d.npairs[g];
      md.pairs[g] = d.pairs[g].p;
    }
    md.variant = 2;
    md.pad_ = 0;
    md.nov = nov;
    md.vbase = vtot;
    md.xbase = xtot;
    md.tbase = ttot;
    vtot += static_cast<long>(Smax) * nov;
    xtot += static_cast<long>(K) * nov;
    ttot += static_cast<long>(2 * K) * nov;
    md.C32 = d.C32.p;
    md.C64 = d.C.p;
    md.eps = d.eps.p;
    md.W = d.W.p;
    md.slot = d.slot.p;
    md.ao_off = d.ao_off.p;
    md.pi_off = d.pi_off.p;
    md.pi_mu = d.pi_mu.p;
    md.pi_nu = d.pi_nu.p;
    md.elems = d.elems;
    scr = std::max(scr, 2L * d.nao * d.nao + static_cast<long>(d.nao) * d.nvirt);
  }
  std::vector<int> order(nmol);
  for (int m = 0; m < nmol; ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h[a].n > h[b].n; });

  // persistent grid: as many workgroups as fit on the device at once
  int dev = 0, ncu = 0, occ = 0;
  SEQX_HIP(hipGetDevice(&dev));
  SEQX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (f32)
    SEQX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sigma_items_kernel<float>, kSigThreads, 0));
  else
    SEQX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sigma_items_kernel<double>, kSigThreads, 0));
  const int G = std::max(1, ncu * std::max(1, occ));
  const long scr_stride = (scr + 63) / 64 * 64;

  w.mols.ensure(nmol);
  w.order.ensure(nmol);
  for (DBuf<int>* b : {&w.S, &w.knew, &w.active, &w.coll, &w.qcol, &w.conv, &w.evn}) b->ensure(nmol);
  w.unc.ensure(static_cast<size_t>(nmol) * K);
  w.counters.ensure(4);
  w.nsig.ensure(3);
  w.stamps.ensure(2 * static_cast<size_t>(G));
  w.items.ensure(static_cast<size_t>(nmol) * std::max(maxnew, K));
  w.V.ensure(vtot);
  w.AV.ensure(vtot);
  w.X.ensure(xtot);
  w.Wc.ensure(xtot);
  w.TV.ensure(ttot);
  w.TAV.ensure(ttot);
  w.Mp.ensure(static_cast<size_t>(nmol) * Smax * Smax);
  w.evec.ensure(static_cast<size_t>(nmol) * Smax * Smax);
  w.eval.ensure(static_cast<size_t>(nmol) * Smax);
  w.omega.ensure(static_cast<size_t>(nmol) * K);
  w.rnorm.ensure(static_cast<size_t>(nmol) * K);
  w.rpart.ensure(static_cast<size_t>(nmol) * kXChunks * kBatchMaxRoots);
  w.part.ensure(static_cast<size_t>(nmol) * kXChunks * kPartStride);
  w.n0.ensure(static_cast<size_t>(nmol) * kXChunks * kBatchMaxRoots);
  if (f32) w.scratch32.ensure(static_cast<size_t>(G) * scr_stride);
  else w.scratch64.ensure(static_cast<size_t>(G) * scr_stride);

  // order against the caller's stream
  hipEvent_t ev_in, ev_a, ev_b;
  SEQX_HIP(hipEventCreate(&ev_in));
  SEQX_HIP(hipEventCreate(&ev_a));
  SEQX_HIP(hipEventCreate(&ev_b));
  auto destroy_events = [&] {
    for (hipEvent_t e : {ev_in, ev_a, ev_b}) (void)hipEventDestroy(e);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  try {
    SEQX_HIP(hipEventRecord(ev_in, user_stream));
    SEQX_HIP(hipStreamWaitEvent(st, ev_in, 0));
    SEQX_HIP(hipMemcpyAsync(w.order.p, order.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
    std::vector<int> zero4(4, 0);
    SEQX_HIP(hipMemcpyAsync(w.counters.p, zero4.data(), 4 * sizeof(int), hipMemcpyHostToDevice, st));
    const long long z3[3] = {0, 0, 0};
    SEQX_HIP(hipMemcpyAsync(w.nsig.p, z3, 3 * sizeof(long long), hipMemcpyHostToDevice, st));

    auto upload_desc = [&] {
      SEQX_HIP(hipMemcpyAsync(w.mols.p, h.data(), nmol * sizeof(MolDesc), hipMemcpyHostToDevice, st));
    };
    auto launch_sigma = [&] {
      if (f32)
        hipLaunchKernelGGL(sigma_items_kernel<float>, dim3(G), dim3(kSigThreads), 0, st, w.mols.p, w.items.p, w.counters.p,
                           w.V.p, w.AV.p, w.scratch32.p, scr_stride, w.stamps.p);
      else
        hipLaunchKernelGGL(sigma_items_kernel<double>, dim3(G), dim3(kSigThreads), 0, st, w.mols.p, w.items.p, w.counters.p,
                           w.V.p, w.AV.p, w.scratch64.p, scr_stride, w.stamps.p);
      SEQX_LAUNCH_CHECK();
    };

    // ---- autotuner: per size bucket, time each tile variant on the bucket's molecules
    const int pk = f32 ? 0 : 1;
    std::vector<int> bucket(nmol);
    for (int m = 0; m < nmol; ++m) bucket[m] = bucket_of(h[m].n);
    upload_desc();
    hipLaunchKernelGGL(guess_kernel, dim3(nmol), dim3(256), 0, st, nmol, w.mols.p, K, w.V.p, w.S.p, w.knew.p,
                       w.active.p, w.conv.p, w.coll.p, w.qcol.p, w.evn.p);
    SEQX_LAUNCH_CHECK();
    const auto ta0 = std::chrono::steady_clock::now();
    for (int b = 0; b < kNumSizeBuckets; ++b) {
      std::vector<int> mb;
      for (int m = 0; m < nmol; ++m)
        if (bucket[m] == b) mb.push_back(m);
      if (mb.empty()) continue;
      if (!opt.autotune) {
        tune.best[pk][b] = 2;
        continue;
      }
      if (tune.tuned[pk][b]) continue;
      // sample: up to 2 G items of this bucket (the first one or two guess vectors)
      std::vector<int2> it;
      for (int m : mb)
        for (int j = 0; j < std::min<long>(2, h[m].nov) && static_cast<int>(it.size()) < 2 * G; ++j)
          it.push_back(make_int2(m, j));
      const int ni = static_cast<int>(it.size());
      SEQX_HIP(hipMemcpyAsync(w.items.p, it.data(), ni * sizeof(int2), hipMemcpyHostToDevice, st));
      SEQX_HIP(hipMemcpyAsync(w.counters.p, &ni, sizeof(int), hipMemcpyHostToDevice, st));
      double best = 1e300;
      for (int var = 0; var < kNumTileVariants; ++var) {
        for (int m : mb) h[m].variant = var;
        upload_desc();
        launch_sigma();  // warm-up
        SEQX_HIP(hipEventRecord(ev_a, st));
        for (int rep = 0; rep < 3; ++rep) launch_sigma();
        SEQX_HIP(hipEventRecord(ev_b, st));
        SEQX_HIP(hipEventSynchronize(ev_b));
        const double t = ms_between(ev_a, ev_b) / 3.0;
        tune.ms[pk][b][var] = t;
        if (t < best) {
          best = t;
          tune.best[pk][b] = var;
        }
      }
      tune.tuned[pk][b] = true;
    }
    res.t_autotune_ms = 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - ta0).count();
    for (int m = 0; m < nmol; ++m) h[m].variant = tune.best[pk][bucket[m]];
    for (int b = 0; b < kNumSizeBuckets; ++b) res.variant_of_bucket[b] = tune.best[pk][b];
    upload_desc();
    SEQX_HIP(hipMemcpyAsync(w.counters.p, zero4.data(), 4 * sizeof(int), hipMemcpyHostToDevice, st));

    // ---- one iteration as a fixed launch sequence
    const int Q = 2 * K;
    auto iteration = [&](bool timed) {
      hipLaunchKernelGGL(items_kernel, dim3(1), dim3(256), 0, st, nmol, w.mols.p, w.order.p, w.S.p, w.knew.p,
                         w.active.p, w.items.p, w.counters.p, w.nsig.p);
      launch_sigma();
      if (timed) hipLaunchKernelGGL(stamp_span_kernel, dim3(1), dim3(256), 0, st, G, w.stamps.p, w.nsig.p + 1);
      hipLaunchKernelGGL(project_part_kernel, dim3(nmol, kXChunks), dim3(256), 0, st, w.mols.p, w.V.p, w.AV.p,
                         w.S.p, w.knew.p, w.active.p, w.part.p);
      hipLaunchKernelGGL(project_kernel, dim3(nmol), dim3(256), 0, st, Smax, w.part.p, w.Mp.p, w.S.p, w.knew.p,
                         w.active.p);
      hipLaunchKernelGGL(advance_kernel, dim3(ceil_div(nmol, 256)), dim3(256), 0, st, nmol, w.S.p, w.knew.p,
                         w.active.p);
      hipLaunchKernelGGL(eig_kernel, dim3(nmol), dim3(kEigThreads), 0, st, Smax, w.Mp.p, w.S.p, w.active.p,
                         w.evn.p, w.evec.p, w.eval.p);
      hipLaunchKernelGGL(ritz_kernel, dim3(nmol, kXChunks), dim3(256), 0, st, w.mols.p, K, Smax, w.V.p, w.AV.p,
                         w.evec.p, w.eval.p, w.S.p, w.active.p, w.X.p, w.Wc.p, w.omega.p, w.rpart.p);
      hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, st, nmol, K, Smax, opt.tol, w.rpart.p, w.rnorm.p,
                         w.S.p, w.knew.p, w.active.p, w.coll.p, w.qcol.p, w.unc.p, w.conv.p, w.counters.p);
      hipLaunchKernelGGL(collapse_kernel, dim3(nmol, Q), dim3(256), 0, st, w.mols.p, Smax, w.V.p, w.AV.p, w.evec.p,
                         w.S.p, w.coll.p, w.qcol.p, w.TV.p, w.TAV.p);
      hipLaunchKernelGGL(collapse_copy_kernel, dim3(nmol, Q + 1), dim3(256), 0, st, w.mols.p, Smax, w.TV.p, w.TAV.p,
                         w.eval.p, w.S.p, w.coll.p, w.qcol.p, w.V.p, w.AV.p, w.Mp.p, w.evn.p);
      const dim3 chunks(nmol, kXChunks);
      hipLaunchKernelGGL(precond_kernel, chunks, dim3(256), 0, st, w.mols.p, K, w.Wc.p, w.knew.p, w.active.p,
                         w.unc.p, w.omega.p, w.n0.p);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(gs_dots_kernel, chunks, dim3(256), 0, st, w.mols.p, K, w.V.p, w.Wc.p, w.S.p, w.knew.p,
                           w.active.p, w.coll.p, w.qcol.p, w.unc.p, w.part.p);
        hipLaunchKernelGGL(gs_update_kernel, chunks, dim3(256), 0, st, w.mols.p, K, w.V.p, w.Wc.p, w.S.p,
                           w.knew.p, w.active.p, w.coll.p, w.qcol.p, w.unc.p, w.part.p);
      }
      hipLaunchKernelGGL(append_kernel, dim3(nmol), dim3(256), 0, st, w.mols.p, K, Smax, w.V.p, w.Wc.p, w.S.p,
                         w.knew.p, w.active.p, w.coll.p, w.qcol.p, w.unc.p, w.conv.p, w.counters.p, w.n0.p);
      SEQX_LAUNCH_CHECK();
    };
    if (opt.graph) {
      // capture one iteration; if the runtime refuses any step, run eagerly instead
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        try {
          iteration(true);
        } catch (const Error&) {
          ok = false;
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        graph = g;
        ok = ok && e == hipSuccess && graph != nullptr;
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        (void)hipGetLastError();
      }
      if (!ok) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
      }
      res.used_graph = ok;
    }
    SEQX_HIP(hipEventRecord(ev_a, st));
    int it = 0, counters[4] = {0, 0, 0, 0};
    for (it = 1; it <= opt.max_iter; ++it) {
      if (exec) SEQX_HIP(hipGraphLaunch(exec, st));
      else iteration(true);
      SEQX_HIP(hipMemcpyAsync(counters, w.counters.p, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
      SEQX_HIP(hipStreamSynchronize(st));
      if (counters[1] == 0) break;
    }
    SEQX_HIP(hipEventRecord(ev_b, st));
    SEQX_HIP(hipEventSynchronize(ev_b));
    res.t_solve_ms = ms_between(ev_a, ev_b);
    res.iterations = std::min(it, opt.max_iter);
    long long ns[3] = {0, 0, 0};
    res.conv_iter.resize(nmol);
    SEQX_HIP(hipMemcpyAsync(ns, w.nsig.p, 3 * sizeof(long long), hipMemcpyDeviceToHost, st));
    SEQX_HIP(hipMemcpyAsync(res.conv_iter.data(), w.conv.p, nmol * sizeof(int), hipMemcpyDeviceToHost, st));
    SEQX_HIP(hipStreamSynchronize(st));
    res.n_sigma = ns[0];
    res.sigma_flops = static_cast<double>(ns[2]);
    int rate_khz = 0;  // device wall clock (the stamps of the sigma launches)
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && rate_khz > 0)
      res.t_sigma_ms = static_cast<double>(ns[1]) / rate_khz;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    for (int m = 0; m < nmol; ++m)
      if (res.conv_iter[m] <= 0)
        throw Error(kEDavNoConv, res.conv_iter[m] < 0 ? "batched Davidson: no new direction for a molecule"
                                                      : "batched Davidson did not converge in " +
                                                            std::to_string(opt.max_iter) + " iterations");
    // ---- amplitudes and properties per molecule, on the caller's stream
    SEQX_HIP(hipEventRecord(ev_b, st));
    SEQX_HIP(hipStreamWaitEvent(user_stream, ev_b, 0));
    for (int m = 0; m < nmol; ++m) {
      const double* Xm = w.X.p + h[m].xbase;
      finalize_roots(*mols[m], 0, K, w.omega.p + static_cast<long>(m) * K, Xm, Xm, sig, w.fin, user_stream);
      mols[m]->dav_iterations = res.conv_iter[m];
    }
  } catch (...) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamSynchronize(st);
    destroy_events();
    throw;
  }
  destroy_events();
  return res;
}

}  // namespace seqx
