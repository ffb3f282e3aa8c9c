// Learned starting space: features, the 12 -> 128 -> 128 -> 1 SiLU network
// (bfloat16 weights, FP32 activations and accumulation), softmax cross-entropy
// training with Adam, and the top-M P-space guess.
//
// The 128 x 128 layer of the forward pass runs on the bfloat16 matrix cores
// (v_mfma_f32_16x16x16_bf16): the weights are bfloat16 values, and each FP32
// activation enters as a pair of bfloat16 numbers (hi + lo, two MFMAs), which
// keeps about 16 significant bits of the activation.  The backward pass uses
// the FP32 matrix cores with the same bfloat16-valued weights.  Weight
// gradients of every 32-pair tile are written out and summed in a fixed order
// (no atomics), so training is deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <random>

#include "mlp.hpp"

namespace seqx {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float x) {  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_value(float x) { return __uint_as_float(static_cast<unsigned>(bf16_bits(x)) << 16); }
__device__ __forceinline__ float silu(float t) { return t / (1.0f + expf(-t)); }
__device__ __forceinline__ float dsilu(float t) {
  const float s = 1.0f / (1.0f + expf(-t));
  return s * (1.0f + t * (1.0f - s));
}

// ---------------------------------------------------------------- features

// pop[A][x] = sum_{mu in A} C[mu][x]^2
__global__ void pop_kernel(int n, int natoms, const int* __restrict__ ao_off, const double* __restrict__ C,
                           double* __restrict__ pop) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int A = blockIdx.y;
  if (x >= n) return;
  double s = 0.0;
  for (int mu = ao_off[A]; mu < ao_off[A + 1]; ++mu) s += C[static_cast<long>(mu) * n + x] * C[static_cast<long>(mu) * n + x];
  pop[static_cast<long>(A) * n + x] = s;
}

// orbital centroids cent[x] = sum_A pop[A][x] R_A
__global__ void centroid_kernel(int n, int natoms, const double* __restrict__ pop, const double* __restrict__ xyz,
                                double* __restrict__ cent) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  double c[3] = {0, 0, 0};
  for (int A = 0; A < natoms; ++A) {
    const double p = pop[static_cast<long>(A) * n + x];
    for (int d = 0; d < 3; ++d) c[d] += p * xyz[3 * A + d];
  }
  for (int d = 0; d < 3; ++d) cent[3 * x + d] = c[d];
}

__global__ void features_kernel(int n, int o, int natoms, const int* __restrict__ ao_off, const int* __restrict__ slot,
                                const Elem* __restrict__ elems, const double* __restrict__ C,
                                const double* __restrict__ eps, const double* __restrict__ pop,
                                const double* __restrict__ cent, float* __restrict__ out) {
  const int v = n - o;
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (x >= static_cast<long>(o) * v) return;
  const int i = static_cast<int>(x / v), a = o + static_cast<int>(x % v);
  double f3 = 0.0, f8 = 0.0, f9 = 0.0, top[4] = {0, 0, 0, 0};
  for (int A = 0; A < natoms; ++A) {
    double q = 0.0;
    for (int mu = ao_off[A]; mu < ao_off[A + 1]; ++mu) q += C[static_cast<long>(mu) * n + i] * C[static_cast<long>(mu) * n + a];
    const double g = elems[slot[A]].gss;
    f3 += q * q;
    f8 += g * q * q;
    f9 += g * pop[static_cast<long>(A) * n + i] * pop[static_cast<long>(A) * n + a];
    double t = fabs(q);
    for (int k = 0; k < 4; ++k)  // insertion into the descending top four
      if (t > top[k]) {
        const double u = top[k];
        top[k] = t;
        t = u;
      }
  }
  const double d0 = cent[3 * i] - cent[3 * a], d1 = cent[3 * i + 1] - cent[3 * a + 1], d2 = cent[3 * i + 2] - cent[3 * a + 2];
  float* f = out + x * kNumFeatures;
  const double gap = eps[a] - eps[i];
  f[0] = static_cast<float>(gap);
  f[1] = static_cast<float>(eps[o - 1] - eps[i]);
  f[2] = static_cast<float>(eps[a] - eps[o]);
  f[3] = static_cast<float>(f3);
  for (int k = 0; k < 4; ++k) f[4 + k] = static_cast<float>(top[k]);
  f[8] = static_cast<float>(f8);
  f[9] = static_cast<float>(f9);
  f[10] = static_cast<float>(sqrt(d0 * d0 + d1 * d1 + d2 * d2));
  f[11] = static_cast<float>(gap + 2.0 * f8 - f9);
}

// ---------------------------------------------------------------- network

struct TileLds {
  float x[kMlpTile][kNumFeatures];
  float a1[kMlpTile][kWidth + 1];  // pre-activations of layer 1 (then its gradient)
  float a2[kMlpTile][kWidth + 1];  // pre-activations of layer 2 (then its gradient)
  float red[256];
};

// Rows [r0, r0 + rows) of the feature array through layers 1 and 2 (pre-activations into L.a1, L.a2).
__device__ void tile_forward(long r0, int rows, const float* __restrict__ feats, const float* __restrict__ wr,
                             TileLds& L) {
  const float* mu = wr + kOffMu;
  const float* sd = wr + kOffSd;
  for (int idx = threadIdx.x; idx < kMlpTile * kNumFeatures; idx += 256) {
    const int r = idx / kNumFeatures, f = idx % kNumFeatures;
    L.x[r][f] = r < rows ? (feats[(r0 + r) * kNumFeatures + f] - mu[f]) / sd[f] : 0.0f;
  }
  __syncthreads();
  const float* W1 = wr + kOffW1;
  const float* b1 = wr + kOffB1;
  for (int idx = threadIdx.x; idx < kMlpTile * kWidth; idx += 256) {
    const int r = idx / kWidth, k = idx % kWidth;
    float s = b1[k];
    for (int f = 0; f < kNumFeatures; ++f) s += L.x[r][f] * W1[f * kWidth + k];
    L.a1[r][k] = s;
  }
  __syncthreads();
  // layer 2 on the bf16 matrix cores: 2 x 8 output tiles of 16 x 16, four per wave
  const float* W2 = wr + kOffW2;
  const float* b2 = wr + kOffB2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = wave; t < 16; t += 4) {
    const int rt = t / 8, ct = t % 8;
    f4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < kWidth; k0 += 16) {
      s4 ahi, alo, b;
      for (int j = 0; j < 4; ++j) {
        const int kk = k0 + 4 * (lane >> 4) + j;
        const float h = silu(L.a1[rt * 16 + (lane & 15)][kk]);
        const unsigned short hb = bf16_bits(h);
        const float hv = __uint_as_float(static_cast<unsigned>(hb) << 16);
        ahi[j] = static_cast<short>(hb);
        alo[j] = static_cast<short>(bf16_bits(h - hv));
        b[j] = static_cast<short>(bf16_bits(W2[kk * kWidth + ct * 16 + (lane & 15)]));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, b, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, b, acc, 0, 0, 0);
    }
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * (lane >> 4) + r, col = ct * 16 + (lane & 15);
      L.a2[row][col] = acc[r] + b2[col];
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(long npairs, const float* __restrict__ feats,
                                                          const float* __restrict__ wr, float* __restrict__ z) {
  __shared__ TileLds L;
  const long r0 = static_cast<long>(blockIdx.x) * kMlpTile;
  const int rows = static_cast<int>(min<long>(kMlpTile, npairs - r0));
  tile_forward(r0, rows, feats, wr, L);
  const float* w3 = wr + kOffW3;
  const float b3 = wr[kOffB3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < rows; r += 4) {
    float s = silu(L.a2[r][lane]) * w3[lane] + silu(L.a2[r][lane + 64]) * w3[lane + 64];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) z[r0 + r] = s + b3;
  }
}

// Backward pass of one tile (rows of tiles[t]); dz per pair in global memory.
// Writes the tile's weight gradients to part[t][kNumWeights].
__global__ void __launch_bounds__(256) mlp_backward_kernel(const int2* __restrict__ tiles,
                                                           const float* __restrict__ feats,
                                                           const float* __restrict__ wr, const float* __restrict__ dz,
                                                           float* __restrict__ part) {
  __shared__ TileLds L;
  __shared__ float dzs[kMlpTile];
  const int2 tl = tiles[blockIdx.x];
  const long r0 = tl.x;
  const int rows = tl.y;
  tile_forward(r0, rows, feats, wr, L);
  for (int r = threadIdx.x; r < kMlpTile; r += 256) dzs[r] = r < rows ? dz[r0 + r] : 0.0f;
  __syncthreads();
  float* g = part + static_cast<long>(blockIdx.x) * kNumWeights;
  const float* w3 = wr + kOffW3;
  const float* W2 = wr + kOffW2;
  // output layer
  if (threadIdx.x < kWidth) {
    const int k = threadIdx.x;
    float s = 0.0f;
    for (int r = 0; r < kMlpTile; ++r) s += silu(L.a2[r][k]) * dzs[r];
    g[kOffW3 + k] = s;
  }
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int r = 0; r < kMlpTile; ++r) s += dzs[r];
    g[kOffB3] = s;
  }
  __syncthreads();
  // d2 = dz w3^T o silu'(a2), in place of a2
  for (int idx = threadIdx.x; idx < kMlpTile * kWidth; idx += 256) {
    const int r = idx / kWidth, k = idx % kWidth;
    L.a2[r][k] = dzs[r] * w3[k] * dsilu(L.a2[r][k]);
  }
  __syncthreads();
  if (threadIdx.x < kWidth) {
    const int k = threadIdx.x;
    float s = 0.0f;
    for (int r = 0; r < kMlpTile; ++r) s += L.a2[r][k];
    g[kOffB2 + k] = s;
  }
  // dW2[k][n] = sum_r silu(a1[r][k]) d2[r][n]: 8 x 8 tiles of 16 x 16 on the FP32 matrix cores, 16 per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = wave; t < 64; t += 4) {
    const int kt = t / 8, nt = t % 8;
    f4 acc = {0, 0, 0, 0};
    for (int r0k = 0; r0k < kMlpTile; r0k += 4) {
      const int r = r0k + (lane >> 4);
      const float av = silu(L.a1[r][kt * 16 + (lane & 15)]);
      const float bv = L.a2[r][nt * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    for (int rr = 0; rr < 4; ++rr) {
      const int k = kt * 16 + 4 * (lane >> 4) + rr, nn = nt * 16 + (lane & 15);
      g[kOffW2 + k * kWidth + nn] = acc[rr];
    }
  }
  __syncthreads();
  // d1[r][k] = (sum_n d2[r][n] W2[k][n]) silu'(a1[r][k]): 2 x 8 tiles, four per wave
  f4 dacc[4];
  for (int q = 0; q < 4; ++q) {
    const int t = wave + 4 * q, rt = t / 8, kt = t % 8;
    f4 acc = {0, 0, 0, 0};
    for (int n0 = 0; n0 < kWidth; n0 += 4) {
      const int nn = n0 + (lane >> 4);
      const float av = L.a2[rt * 16 + (lane & 15)][nn];
      const float bv = W2[(kt * 16 + (lane & 15)) * kWidth + nn];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    dacc[q] = acc;
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int t = wave + 4 * q, rt = t / 8, kt = t % 8;
    for (int rr = 0; rr < 4; ++rr) {
      const int r = rt * 16 + 4 * (lane >> 4) + rr, k = kt * 16 + (lane & 15);
      L.a1[r][k] = dacc[q][rr] * dsilu(L.a1[r][k]);
    }
  }
  __syncthreads();
  if (threadIdx.x < kWidth) {
    const int k = threadIdx.x;
    float s = 0.0f;
    for (int r = 0; r < kMlpTile; ++r) s += L.a1[r][k];
    g[kOffB1 + k] = s;
  }
  for (int idx = threadIdx.x; idx < kNumFeatures * kWidth; idx += 256) {
    const int f = idx / kWidth, k = idx % kWidth;
    float s = 0.0f;
    for (int r = 0; r < kMlpTile; ++r) s += L.x[r][f] * L.a1[r][k];
    g[kOffW1 + f * kWidth + k] = s;
  }
}

// Softmax cross-entropy of molecule b of the batch (pairs seg[b] .. seg[b+1]):
// loss into lossm[b], dz = (softmax(z) sum(w) - w) / nmol.
__global__ void __launch_bounds__(256) softmax_loss_kernel(int nmol, const long* __restrict__ seg,
                                                           const float* __restrict__ z, const float* __restrict__ w,
                                                           float* __restrict__ dz, double* __restrict__ lossm) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const long s0 = seg[2 * b], s1 = seg[2 * b + 1];
  double mx = -1e300;
  for (long x = s0 + threadIdx.x; x < s1; x += 256) mx = fmax(mx, static_cast<double>(z[x]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  double se = 0.0, sw = 0.0, swz = 0.0;
  for (long x = s0 + threadIdx.x; x < s1; x += 256) {
    se += exp(static_cast<double>(z[x]) - mx);
    sw += w[x];
    swz += static_cast<double>(w[x]) * z[x];
  }
  double tot[3] = {se, sw, swz};
  for (int c = 0; c < 3; ++c) {
    red[threadIdx.x] = tot[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    tot[c] = red[0];
    __syncthreads();
  }
  const double lse = mx + log(tot[0]);
  for (long x = s0 + threadIdx.x; x < s1; x += 256)
    dz[x] = static_cast<float>((exp(static_cast<double>(z[x]) - lse) * tot[1] - w[x]) / nmol);
  if (threadIdx.x == 0) lossm[b] = lse * tot[1] - tot[2];
}

// grad[p] = sum over tiles of part[t][p], fixed order
__global__ void sum_tiles_kernel(int ntiles, const float* __restrict__ part, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNumWeights) return;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += part[static_cast<long>(t) * kNumWeights + p];
  grad[p] = static_cast<float>(s);
}

__device__ __forceinline__ bool is_rounded_weight(int p) {
  return (p >= kOffW1 && p < kOffB1) || (p >= kOffW2 && p < kOffB2) || (p >= kOffW3 && p < kOffB3);
}

// copy the master parameters into the forward copy, rounding the weight matrices to bfloat16
__global__ void round_params_kernel(const float* __restrict__ master, float* __restrict__ wr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNumParams) wr[p] = is_rounded_weight(p) ? bf16_value(master[p]) : master[p];
}

__global__ void adam_kernel(long step, float lr, const float* __restrict__ grad, float* master, float* m1, float* m2,
                            float* wr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNumWeights) return;
  const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
  const float g = grad[p];
  m1[p] = b1 * m1[p] + (1.0f - b1) * g;
  m2[p] = b2 * m2[p] + (1.0f - b2) * g * g;
  const float mh = m1[p] / (1.0f - powf(b1, static_cast<float>(step)));
  const float vh = m2[p] / (1.0f - powf(b2, static_cast<float>(step)));
  master[p] -= lr * mh / (sqrtf(vh) + e);
  wr[p] = is_rounded_weight(p) ? bf16_value(master[p]) : master[p];
}

// target w = (1/K) sum_n X[n]^2 of one molecule
__global__ void target_kernel(long nov, int K, const double* __restrict__ X, float* __restrict__ w) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (x >= nov) return;
  double s = 0.0;
  for (int n = 0; n < K; ++n) s += X[n * nov + x] * X[n * nov + x];
  w[x] = static_cast<float>(s / K);
}

// mean and standard deviation of every feature over all rows (fixed order, one block per feature)
__global__ void __launch_bounds__(256) feature_stats_kernel(long npairs, const float* __restrict__ feats,
                                                            float* __restrict__ musd) {
  __shared__ double red[256];
  const int f = blockIdx.x;
  double s = 0.0;
  for (long x = threadIdx.x; x < npairs; x += 256) s += feats[x * kNumFeatures + f];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double mean = red[0] / npairs;
  __syncthreads();
  double q = 0.0;
  for (long x = threadIdx.x; x < npairs; x += 256) {
    const double d = feats[x * kNumFeatures + f] - mean;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    musd[f] = static_cast<float>(mean);
    musd[kNumFeatures + f] = static_cast<float>(fmax(sqrt(red[0] / npairs), 1e-6));
  }
}

// M best pairs by (score descending, index ascending); learned = 0 scores by
// -gap.  Stage 1: every workgroup keeps the M best of its contiguous chunk
// (M rounds of a lexicographic workgroup maximum); stage 2: one workgroup
// picks the M best of the candidates.  Both stages visit candidates in index
// order, so ties go to the lower flat index.
__device__ __forceinline__ bool better(double s, long i, double t, long j) { return s > t || (s == t && i < j); }

__device__ void topm_block(long n0, long n1, int M, const double* cs, const long* ci, int learned_src,
                           const float* __restrict__ z, const double* __restrict__ eps, int v, int o,
                           double* outs, long* outi, double* bs, long* bi) {
  double ls = 1e300;
  long li = -1;
  for (int r = 0; r < M; ++r) {
    double best = -1e300;
    long bidx = 0x7fffffffffffffffL;
    for (long x = n0 + threadIdx.x; x < n1; x += 256) {
      double sc;
      long id;
      if (cs) {
        sc = cs[x];
        id = ci[x];
      } else {
        sc = learned_src ? static_cast<double>(z[x]) : -(eps[o + x % v] - eps[x / v]);
        id = x;
      }
      if (id < 0) continue;
      if (better(ls, li, sc, id) && better(sc, id, best, bidx)) {
        best = sc;
        bidx = id;
      }
    }
    bs[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h && better(bs[threadIdx.x + h], bi[threadIdx.x + h], bs[threadIdx.x], bi[threadIdx.x])) {
        bs[threadIdx.x] = bs[threadIdx.x + h];
        bi[threadIdx.x] = bi[threadIdx.x + h];
      }
      __syncthreads();
    }
    ls = bs[0];
    li = bi[0];
    if (threadIdx.x == 0) {
      outs[r] = ls;
      outi[r] = li < 0x7fffffffffffffffL ? li : -1;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) topm_stage1_kernel(long nov, long chunk, int v, int o, int M, int learned,
                                                          const float* __restrict__ z, const double* __restrict__ eps,
                                                          double* __restrict__ cs, long* __restrict__ ci) {
  __shared__ double bs[256];
  __shared__ long bi[256];
  const long n0 = blockIdx.x * chunk, n1 = min(nov, n0 + chunk);
  topm_block(n0, n1, M, nullptr, nullptr, learned, z, eps, v, o, cs + static_cast<long>(blockIdx.x) * M,
             ci + static_cast<long>(blockIdx.x) * M, bs, bi);
}

__global__ void __launch_bounds__(256) topm_stage2_kernel(long ncand, int M, const double* __restrict__ cs,
                                                          const long* __restrict__ ci, double* __restrict__ ws,
                                                          long* __restrict__ wi, int* __restrict__ sel) {
  __shared__ double bs[256];
  __shared__ long bi[256];
  topm_block(0, ncand, M, cs, ci, 0, nullptr, nullptr, 1, 0, ws, wi, bs, bi);
  for (int r = threadIdx.x; r < M; r += 256) sel[r] = static_cast<int>(wi[r]);
}

__global__ void unit_rows_kernel(long nov, int M, const int* __restrict__ sel, double* __restrict__ V) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const int r = blockIdx.y;
  if (x < nov) V[r * nov + x] = (x == sel[r]) ? 1.0 : 0.0;
}

}  // namespace

void Mlp::set(const float* host, hipStream_t st) {
  master.ensure(kNumParams);
  wr.ensure(kNumParams);
  m1.ensure(kNumWeights);
  m2.ensure(kNumWeights);
  SEQX_HIP(hipMemcpyAsync(master.p, host, kNumParams * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<float> zero(kNumWeights, 0.0f);
  SEQX_HIP(hipMemcpyAsync(m1.p, zero.data(), kNumWeights * sizeof(float), hipMemcpyHostToDevice, st));
  SEQX_HIP(hipMemcpyAsync(m2.p, zero.data(), kNumWeights * sizeof(float), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(round_params_kernel, dim3(ceil_div(kNumParams, 256)), dim3(256), 0, st, master.p, wr.p);
  SEQX_LAUNCH_CHECK();
  SEQX_HIP(hipStreamSynchronize(st));
  step = 0;
  ready = true;
}

void Mlp::get(float* host, hipStream_t st) const {
  if (!ready) throw Error(kEState, "no network parameters");
  SEQX_HIP(hipMemcpyAsync(host, master.p, kNumParams * sizeof(float), hipMemcpyDeviceToHost, st));
  SEQX_HIP(hipStreamSynchronize(st));
}

void mlp_features(const DeviceMolecule& m, float* out, MlpWork& w, hipStream_t st) {
  const int n = m.nao, o = m.nocc, na = m.natoms;
  const long nov = static_cast<long>(o) * m.nvirt;
  w.pop.ensure(static_cast<size_t>(na) * n);
  w.cent.ensure(3 * static_cast<size_t>(n));
  hipLaunchKernelGGL(pop_kernel, dim3(ceil_div(n, 256), na), dim3(256), 0, st, n, na, m.ao_off.p, m.C.p, w.pop.p);
  hipLaunchKernelGGL(centroid_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, na, w.pop.p, m.xyz.p, w.cent.p);
  hipLaunchKernelGGL(features_kernel, dim3(ceil_div(nov, 256)), dim3(256), 0, st, n, o, na, m.ao_off.p, m.slot.p,
                     m.elems, m.C.p, m.eps.p, w.pop.p, w.cent.p, out);
  SEQX_LAUNCH_CHECK();
}

void mlp_scores(const Mlp& net, long npairs, const float* feats, float* z, hipStream_t st) {
  if (!net.ready) throw Error(kEState, "no network parameters: load or train one first");
  if (npairs <= 0) return;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(static_cast<unsigned>(ceil_div(npairs, kMlpTile))), dim3(256), 0, st,
                     npairs, feats, net.wr.p, z);
  SEQX_LAUNCH_CHECK();
}

namespace {

// one optimisation step's gradient over the molecules `batch` (pair ranges in seg_all)
double batch_loss_grad(const Mlp& net, const float* feats, const float* w, const std::vector<long>& ranges,
                       float* grad, MlpWork& work, hipStream_t st) {
  const int nb = static_cast<int>(ranges.size() / 2);
  std::vector<int2> tiles;
  long maxp = 0;
  for (int b = 0; b < nb; ++b) {
    for (long r = ranges[2 * b]; r < ranges[2 * b + 1]; r += kMlpTile)
      tiles.push_back(make_int2(static_cast<int>(r), static_cast<int>(std::min<long>(kMlpTile, ranges[2 * b + 1] - r))));
    maxp = std::max(maxp, ranges[2 * b + 1]);
  }
  const int nt = static_cast<int>(tiles.size());
  work.tiles.ensure(nt);
  work.seg.ensure(2 * nb);
  work.part.ensure(static_cast<size_t>(nt) * kNumWeights);
  work.lossm.ensure(nb);
  work.z.ensure(maxp);
  work.dz.ensure(maxp);
  SEQX_HIP(hipMemcpyAsync(work.tiles.p, tiles.data(), nt * sizeof(int2), hipMemcpyHostToDevice, st));
  SEQX_HIP(hipMemcpyAsync(work.seg.p, ranges.data(), 2 * nb * sizeof(long), hipMemcpyHostToDevice, st));
  for (int b = 0; b < nb; ++b) {
    const long r0 = ranges[2 * b], np = ranges[2 * b + 1] - r0;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(static_cast<unsigned>(ceil_div(np, kMlpTile))), dim3(256), 0, st, np,
                       feats + r0 * kNumFeatures, net.wr.p, work.z.p + r0);
  }
  hipLaunchKernelGGL(softmax_loss_kernel, dim3(nb), dim3(256), 0, st, nb, work.seg.p, work.z.p, w, work.dz.p,
                     work.lossm.p);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(nt), dim3(256), 0, st, work.tiles.p, feats, net.wr.p, work.dz.p,
                     work.part.p);
  hipLaunchKernelGGL(sum_tiles_kernel, dim3(ceil_div(kNumWeights, 256)), dim3(256), 0, st, nt, work.part.p, grad);
  SEQX_LAUNCH_CHECK();
  std::vector<double> lm(nb);
  SEQX_HIP(hipMemcpyAsync(lm.data(), work.lossm.p, nb * sizeof(double), hipMemcpyDeviceToHost, st));
  SEQX_HIP(hipStreamSynchronize(st));
  double L = 0.0;
  for (double x : lm) L += x;
  return L / nb;
}

}  // namespace

double mlp_loss_grad(const Mlp& net, long npairs, const float* feats, const float* w, int nmol, const long* seg,
                     float* grad, MlpWork& work, hipStream_t st) {
  if (!net.ready) throw Error(kEState, "no network parameters");
  if (nmol < 1 || seg[0] != 0 || seg[nmol] != npairs) throw Error(kEArg, "bad molecule segmentation");
  std::vector<long> ranges(2 * nmol);
  for (int b = 0; b < nmol; ++b) {
    if (seg[b + 1] <= seg[b]) throw Error(kEArg, "empty molecule in segmentation");
    ranges[2 * b] = seg[b];
    ranges[2 * b + 1] = seg[b + 1];
  }
  return batch_loss_grad(net, feats, w, ranges, grad, work, st);
}

void mlp_train(Mlp& net, const std::vector<DeviceMolecule*>& mols, const TrainOptions& opt, TrainLog& log,
               MlpWork& work, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  const int nmol = static_cast<int>(mols.size());
  if (nmol < 1) throw Error(kEArg, "empty training set");
  std::vector<long> off(nmol + 1, 0);
  for (int m = 0; m < nmol; ++m) {
    const DeviceMolecule& d = *mols[m];
    if (d.nroots < 1 || d.theory != 0) throw Error(kEState, "training molecules need solved CIS roots");
    off[m + 1] = off[m] + static_cast<long>(d.nocc) * d.nvirt;
  }
  const long np = off[nmol];
  work.feats.ensure(static_cast<size_t>(np) * kNumFeatures);
  work.w.ensure(np);
  for (int m = 0; m < nmol; ++m) {
    const DeviceMolecule& d = *mols[m];
    const long nov = off[m + 1] - off[m];
    mlp_features(d, work.feats.p + off[m] * kNumFeatures, work, st);
    hipLaunchKernelGGL(target_kernel, dim3(static_cast<unsigned>(ceil_div(nov, 256))), dim3(256), 0, st, nov,
                       d.nroots, d.X.p, work.w.p + off[m]);
  }
  SEQX_LAUNCH_CHECK();
  if (opt.init || !net.ready) {
    // fan-in scaled uniform weights from the seed, zero biases, standardisation from the training features
    std::vector<float> p(kNumParams, 0.0f);
    std::mt19937_64 rng(opt.seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    const double l1 = std::sqrt(6.0 / kNumFeatures), l2 = std::sqrt(6.0 / kWidth);
    for (int i = 0; i < kNumFeatures * kWidth; ++i) p[kOffW1 + i] = static_cast<float>(l1 * u(rng));
    for (int i = 0; i < kWidth * kWidth; ++i) p[kOffW2 + i] = static_cast<float>(l2 * u(rng));
    for (int i = 0; i < kWidth; ++i) p[kOffW3 + i] = static_cast<float>(l2 * u(rng));
    DBuf<float> musd(2 * kNumFeatures);
    hipLaunchKernelGGL(feature_stats_kernel, dim3(kNumFeatures), dim3(256), 0, st, np, work.feats.p, musd.p);
    SEQX_LAUNCH_CHECK();
    SEQX_HIP(hipMemcpyAsync(p.data() + kOffMu, musd.p, 2 * kNumFeatures * sizeof(float), hipMemcpyDeviceToHost, st));
    SEQX_HIP(hipStreamSynchronize(st));
    net.set(p.data(), st);
  }
  work.grad.ensure(kNumWeights);
  std::vector<int> order(nmol);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 shuf(opt.seed ^ 0x9E3779B97F4A7C15ULL);
  const int B = std::max(1, std::min(opt.batch, nmol));
  log.loss.clear();
  for (int e = 0; e < opt.epochs; ++e) {
    std::shuffle(order.begin(), order.end(), shuf);
    double el = 0.0;
    int nsteps = 0;
    for (int b0 = 0; b0 < nmol; b0 += B) {
      std::vector<long> ranges;
      for (int b = b0; b < std::min(nmol, b0 + B); ++b) {
        ranges.push_back(off[order[b]]);
        ranges.push_back(off[order[b] + 1]);
      }
      el += batch_loss_grad(net, work.feats.p, work.w.p, ranges, work.grad.p, work, st);
      ++nsteps;
      ++net.step;
      hipLaunchKernelGGL(adam_kernel, dim3(ceil_div(kNumWeights, 256)), dim3(256), 0, st, net.step,
                         static_cast<float>(opt.lr), work.grad.p, net.master.p, net.m1.p, net.m2.p, net.wr.p);
      SEQX_LAUNCH_CHECK();
    }
    log.loss.push_back(el / nsteps);
  }
  SEQX_HIP(hipStreamSynchronize(st));
  log.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void pspace_guess(const Mlp* net, const DeviceMolecule& m, int M, bool learned, double* V, MlpWork& w,
                  hipStream_t st) {
  const long nov = static_cast<long>(m.nocc) * m.nvirt;
  if (M < 1 || M > nov) throw Error(kEArg, "P-space size out of range");
  w.sel.ensure(M);
  if (learned) {
    if (!net || !net->ready) throw Error(kEState, "learned guess needs a loaded or trained network");
    w.feats.ensure(static_cast<size_t>(nov) * kNumFeatures);
    w.z.ensure(nov);
    mlp_features(m, w.feats.p, w, st);
    mlp_scores(*net, nov, w.feats.p, w.z.p, st);
  }
  const long chunk = std::max<long>(1024, ceil_div(nov, 512));
  const int nblk = static_cast<int>(ceil_div(nov, chunk));
  w.cand.ensure(static_cast<size_t>(nblk) * M + M);
  w.candi.ensure(static_cast<size_t>(nblk) * M + M);
  hipLaunchKernelGGL(topm_stage1_kernel, dim3(nblk), dim3(256), 0, st, nov, chunk, m.nvirt, m.nocc, M,
                     learned ? 1 : 0, learned ? w.z.p : nullptr, m.eps.p, w.cand.p, w.candi.p);
  hipLaunchKernelGGL(topm_stage2_kernel, dim3(1), dim3(256), 0, st, static_cast<long>(nblk) * M, M, w.cand.p,
                     w.candi.p, w.cand.p + static_cast<long>(nblk) * M, w.candi.p + static_cast<long>(nblk) * M,
                     w.sel.p);
  hipLaunchKernelGGL(unit_rows_kernel, dim3(static_cast<unsigned>(ceil_div(nov, 256)), M), dim3(256), 0, st, nov, M,
                     w.sel.p, V);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
