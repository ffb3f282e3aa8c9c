// Davidson iteration for CIS (Eq. 7) and TDHF (Eq. 2) on one GPU.
//
// The paper's outline (GPU-implementation subsection): start from orthonormal
// trial vectors; form the matrix-vector products; project and diagonalise;
// Ritz vectors and residuals; precondition only the unconverged residuals with
// the diagonal; orthonormalise against the basis and append.  The subspace is
// capped (the paper derives the cap from free memory) and collapses onto the
// current best Ritz vectors when full.
//
// TDHF uses one orthonormal basis V for X+Y and X-Y: M+ = V^T (A+B) V and
// M- = V^T (A-B) V; with M- = L L^T, (L^T M+ L) z = w^2 z, t = L z / sqrt(w),
// u = M+ t / w, so that t^T u = 1 (X^T X - Y^T Y = 1).  Residuals:
// r_T = (A+B) T - w U, r_U = (A-B) U - w T.  New directions per unconverged
// root: (r_T + r_U)/(w - d) and (r_T - r_U)/(-w - d), d = eps_a - eps_i.
// Orthonormalisation: unit rows, classical Gram-Schmidt against V (a second
// pass when a row lost most of its norm), then symmetric (Loewdin)
// orthonormalisation inside the new block with near-dependent directions
// dropped.  (A+B)V and (A-B)V rows are stored interleaved so that one pass over
// the basis serves both projected matrices.  All subspace arithmetic is FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "davidson.hpp"
#include "gemm.hpp"
#include "sigma.hpp"

namespace seqx {

namespace {

__global__ void gap_kernel(int o, int v, const double* __restrict__ eps, double* __restrict__ d) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (x >= static_cast<long>(o) * v) return;
  const int i = static_cast<int>(x / v), a = static_cast<int>(x % v);
  d[x] = eps[o + a] - eps[i];
}

// smallest ng gaps (ties: lowest flat index i*v + a).  Any of them has i among
// the ng highest occupied and a among the ng lowest virtual orbitals.
__global__ void gap_guess_kernel(int o, int v, int ng, const double* __restrict__ eps, int* __restrict__ idx) {
  const int i0 = max(0, o - ng), ni = o - i0, na = min(v, ng);
  const int N = ni * na;
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    const int i = i0 + q / na, a = q % na;
    const double g = eps[o + a] - eps[i];
    const int f = i * v + a;
    int rank = 0;
    for (int q2 = 0; q2 < N; ++q2) {
      const int i2 = i0 + q2 / na, a2 = q2 % na;
      const double g2 = eps[o + a2] - eps[i2];
      const int f2 = i2 * v + a2;
      if (g2 < g || (g2 == g && f2 < f)) ++rank;
    }
    if (rank < ng) idx[rank] = f;
  }
}

template <class TV>
__global__ void unit_vectors_kernel(int ng, long nov, const int* __restrict__ idx, TV* __restrict__ V) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const int r = blockIdx.y;
  if (x >= nov) return;
  V[r * nov + x] = (x == idx[r]) ? TV(1) : TV(0);
}

// column-major M: new columns t in [S0, S1) are filled for rows [0, S1);
// mirror them into rows and symmetrise the new-new block
__global__ void sym_fill_kernel(double* M, int ld, int S0, int S1) {
  const int t = S0 + blockIdx.y;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S1; s += gridDim.x * blockDim.x) {
    if (s < S0) {
      M[static_cast<long>(s) * ld + t] = M[static_cast<long>(t) * ld + s];
    } else if (s < t) {
      const double a = 0.5 * (M[static_cast<long>(t) * ld + s] + M[static_cast<long>(s) * ld + t]);
      M[static_cast<long>(t) * ld + s] = a;
      M[static_cast<long>(s) * ld + t] = a;
    }
  }
}

// G (nr x S1, row r = product p = r % ps of new vector r / ps against V_0..V_S1-1)
// -> column S0 + r / ps of Mp (p = 0) or Mm (p = 1), column-major, ld ldm
__global__ void scatter_cols_kernel(const double* __restrict__ G, int S1, int ps, int S0, double* Mp, double* Mm,
                                    int ldm) {
  const int r = blockIdx.y;
  double* M = (r % ps == 0) ? Mp : Mm;
  const int t = S0 + r / ps;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S1; s += gridDim.x * blockDim.x)
    M[static_cast<long>(t) * ldm + s] = G[static_cast<long>(r) * S1 + s];
}

__global__ void omega_kernel(int K, const double* __restrict__ w2, double* __restrict__ om, int tdhf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < K) om[j] = tdhf ? sqrt(fmax(w2[j], 0.0)) : w2[j];
}

// C[:, j] *= om[j]^(-p) for j < K (column-major, nrows rows)
__global__ void scale_cols_kernel(double* C, int ld, int nrows, int K, const double* __restrict__ om, double p) {
  const int j = blockIdx.x;
  const double s = pow(om[j], -p);
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) C[static_cast<long>(j) * ld + r] *= s;
}

// residual norms^2, partial sums per block: TDHF r_T = PT - w U, r_U = MU - w T;
// CIS r = PT - w T
template <class TI>
__global__ void residual_norm_kernel(long nov, int tdhf, const double* __restrict__ om, const TI* __restrict__ Tv,
                                     const TI* __restrict__ Uv, const TI* __restrict__ PT,
                                     const TI* __restrict__ MU, double* __restrict__ part) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const double w = om[j];
  const long base = static_cast<long>(j) * nov;
  double s = 0.0;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < nov; x += 256L * gridDim.x) {
    if (tdhf) {
      const double rT = static_cast<double>(PT[base + x]) - w * static_cast<double>(Uv[base + x]);
      const double rU = static_cast<double>(MU[base + x]) - w * static_cast<double>(Tv[base + x]);
      s += rT * rT + rU * rU;
    } else {
      const double r = static_cast<double>(PT[base + x]) - w * static_cast<double>(Tv[base + x]);
      s += r * r;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[static_cast<long>(j) * gridDim.x + blockIdx.x] = red[0];
}

// the words the host checks after each iteration, beside the residual norms:
// lowest eigenvalue of the projected problem, eigh and potrf info
__global__ void check_words_kernel(const double* __restrict__ w2, const int* __restrict__ info, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = w2[0];
    out[1] = static_cast<double>(info[0]);
    out[2] = static_cast<double>(info[1]);
  }
}

__global__ void reduce_rows_kernel(int K, int nb, const double* __restrict__ part, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[static_cast<long>(j) * nb + b];
  out[j] = sqrt(s);
}

__device__ inline double guard(double x) {
  return fabs(x) < 1e-8 ? (x < 0 ? -1e-8 : 1e-8) : x;
}

template <class TI, class TW>
__global__ void precond_kernel(long nov, int tdhf, const int* __restrict__ sel, const double* __restrict__ om,
                               const double* __restrict__ d, const TI* __restrict__ Tv,
                               const TI* __restrict__ Uv, const TI* __restrict__ PT,
                               const TI* __restrict__ MU, TW* __restrict__ W) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (x >= nov) return;
  const int q = blockIdx.y;
  const int j = sel[q];
  const double w = om[j];
  const long b = static_cast<long>(j) * nov + x;
  if (tdhf) {
    const double rT = static_cast<double>(PT[b]) - w * static_cast<double>(Uv[b]);
    const double rU = static_cast<double>(MU[b]) - w * static_cast<double>(Tv[b]);
    W[(2L * q) * nov + x] = static_cast<TW>((rT + rU) / guard(w - d[x]));
    W[(2L * q + 1) * nov + x] = static_cast<TW>((rT - rU) / guard(-w - d[x]));
  } else {
    const double r = static_cast<double>(PT[b]) - w * static_cast<double>(Tv[b]);
    W[static_cast<long>(q) * nov + x] = static_cast<TW>(r / guard(w - d[x]));
  }
}

template <class TW>
__global__ void scale_rows_kernel(long nov, TW* __restrict__ W, const double* __restrict__ G, int ldg) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const int r = blockIdx.y;
  if (x >= nov) return;
  const double g = G[static_cast<long>(r) * ldg + r];
  W[r * nov + x] = static_cast<TW>(W[r * nov + x] * ((g > 0.0) ? 1.0 / sqrt(g) : 0.0));
}

// dst columns (ld) = src columns over rows [0, s0), zero over rows [s0, s1)
__global__ void pad_cols_kernel(int s0, int s1, const double* __restrict__ src, double* __restrict__ dst, int ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const long c = static_cast<long>(blockIdx.y) * ld;
  if (r < s1) dst[c + r] = r < s0 ? src[c + r] : 0.0;
}

__global__ void invsqrt_cols_kernel(double* Q, int ld, int nrows, int j0, const double* __restrict__ lam) {
  const int j = j0 + blockIdx.x;
  const double s = 1.0 / sqrt(lam[j]);
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) Q[static_cast<long>(j) * ld + r] *= s;
}

__global__ void finalize_kernel(long nov, int tdhf, const double* __restrict__ Tv, const double* __restrict__ Uv,
                                double* __restrict__ X, double* __restrict__ Y) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= nov) return;
  const long b = static_cast<long>(j) * nov + x;
  if (tdhf) {
    X[b] = 0.5 * (Tv[b] + Uv[b]);
    Y[b] = 0.5 * (Tv[b] - Uv[b]);
  } else {
    X[b] = Tv[b];
    Y[b] = 0.0;
  }
}

// flip root j so that its largest |X| element (lowest index on ties) is positive
__global__ void sign_fix_kernel(long nov, double* __restrict__ X, double* __restrict__ Y) {
  __shared__ double bv[256];
  __shared__ long bi[256];
  const int j = blockIdx.x;
  double* x = X + static_cast<long>(j) * nov;
  double best = -1.0;
  long bidx = 0;
  for (long t = threadIdx.x; t < nov; t += 256) {
    const double a = fabs(x[t]);
    if (a > best) {  // strided scan visits indices in increasing order
      best = a;
      bidx = t;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double a = bv[threadIdx.x + h];
      const long ia = bi[threadIdx.x + h];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ia < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ia;
      }
    }
    __syncthreads();
  }
  const bool flip = x[bi[0]] < 0.0;
  __syncthreads();
  if (flip) {
    double* y = Y + static_cast<long>(j) * nov;
    for (long t = threadIdx.x; t < nov; t += 256) {
      x[t] = -x[t];
      y[t] = -y[t];
    }
  }
}

// transition dipoles mu_j = sqrt(2) sum_mn T_mn <m|r|n> with the ZDO dipole
// (R_A on the diagonal, D1_A between s and p_k of one atom) and
// f_j = 2/3 w_j |mu_j|^2
__global__ void dipole_kernel(int natoms, int n, const double* __restrict__ T, const int* __restrict__ slot,
                              const int* __restrict__ ao_off, const double* __restrict__ xyz,
                              const Elem* __restrict__ elems, const double* __restrict__ om, double* __restrict__ mu,
                              double* __restrict__ f) {
  __shared__ double red[3][256];
  const int j = blockIdx.x;
  const double* Tj = T + static_cast<long>(j) * n * n;
  double s[3] = {0, 0, 0};
  for (int A = threadIdx.x; A < natoms; A += 256) {
    const Elem e = elems[slot[A]];
    const int o = ao_off[A];
    double tr = 0.0;
    for (int i = 0; i < e.nao; ++i) tr += Tj[static_cast<long>(o + i) * n + o + i];
    for (int c = 0; c < 3; ++c) {
      s[c] += tr * xyz[3 * A + c];
      if (e.nao == 4)
        s[c] += e.D1 * (Tj[static_cast<long>(o) * n + o + 1 + c] + Tj[static_cast<long>(o + 1 + c) * n + o]);
    }
  }
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double m2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double v = sqrt(2.0) * red[c][0];
      mu[3 * j + c] = v;
      m2 += v * v;
    }
    f[j] = 2.0 / 3.0 * om[j] * m2;
  }
}

template <class T>
void d2h(T* dst, const T* src, size_t n, hipStream_t st) {
  SEQX_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}

// per-iteration JSON lines on stderr when SEQX_LOG is set to a non-empty value other than 0
bool log_enabled() {
  static const bool on = [] {
    const char* s = std::getenv("SEQX_LOG");
    return s && *s && std::strcmp(s, "0") != 0;
  }();
  return on;
}

// Event marks on the stream; the time between consecutive marks is charged to
// the phase of the earlier mark.
class IterTimer {
 public:
  explicit IterTimer(hipStream_t st) : st_(st) {}
  ~IterTimer() {
    for (auto& m : marks_) (void)hipEventDestroy(m.second);
  }
  void mark(int phase) {
    hipEvent_t e;
    SEQX_HIP(hipEventCreate(&e));
    SEQX_HIP(hipEventRecord(e, st_));
    marks_.emplace_back(phase, e);
  }
  void accumulate(double* ms) {
    if (marks_.empty()) return;
    SEQX_HIP(hipEventSynchronize(marks_.back().second));
    for (size_t i = 0; i + 1 < marks_.size(); ++i) {
      float t = 0.f;
      SEQX_HIP(hipEventElapsedTime(&t, marks_[i].second, marks_[i + 1].second));
      ms[marks_[i].first] += t;
    }
  }

 private:
  hipStream_t st_;
  std::vector<std::pair<int, hipEvent_t>> marks_;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Basis operations for FP64 or FP32 basis rows (the FP32 basis of the
// low-precision phase): FP64 rows go through the general FP64 paths, FP32
// rows through the tall-skinny kernels that widen them on load.
template <class TB, class TC>
void comb(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const TB* B, long ldb,
          double beta, TC* C, long ldc) {
  if constexpr (std::is_same<TB, double>::value && std::is_same<TC, double>::value)
    dgemm(st, false, false, M, static_cast<int>(N), K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, nullptr);
  else
    combine_rows<TB, TC>(st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

template <class TX, class TY>
void dts(hipStream_t st, int ns, const TX* X, long ldx, int nt, const TY* Y, long ldy, long len, double* out, long ldo,
         double* ws) {
  if constexpr (std::is_same<TX, double>::value && std::is_same<TY, double>::value)
    dots(st, ns, X, ldx, nt, Y, ldy, len, out, ldo, ws);
  else
    dots_mixed<TX, TY>(st, ns, X, ldx, nt, Y, ldy, len, out, ldo, ws);
}

// Orthonormalise the nc rows of Wc against V[0:S] and among themselves, append
// the kept directions at V[S:]; returns how many were kept.  Wc: FP64 rows, or
// FP32 rows beside an FP32 basis (inner products and sums in FP64 either way).
template <class TV, class TW>
int orthonormalize_append(hipStream_t st, DenseSolver& ds, DavWork& w, long nov, int nc, TW* Wc, int S, TV* V,
                          int max_keep) {
  double* G = w.G.p;
  double* Cc = w.Q.p;  // nc x S coefficients, reused below for the Loewdin vectors
  dts(st, nc, Wc, nov, nc, Wc, nov, nov, G, nc, w.ws.p);
  hipLaunchKernelGGL(scale_rows_kernel<TW>, dim3(ceil_div(nov, 256), nc), dim3(256), 0, st, nov, Wc, G, nc);
  SEQX_LAUNCH_CHECK();
  // classical Gram-Schmidt against V; a second pass only when a unit row lost
  // more than three quarters of its norm ("twice is enough")
  for (int pass = 0; pass < 2 && S > 0; ++pass) {
    dts(st, nc, Wc, nov, S, V, nov, nov, Cc, S, w.ws.p);
    comb(st, nc, nov, S, -1.0, Cc, S, V, nov, 1.0, Wc, nov);
    dts(st, nc, Wc, nov, nc, Wc, nov, nov, G, nc, w.ws.p);
    if (pass == 1) break;
    std::vector<double> g(static_cast<size_t>(nc) * nc);
    d2h(g.data(), G, g.size(), st);
    SEQX_HIP(hipStreamSynchronize(st));
    bool again = false;
    for (int r = 0; r < nc; ++r) again = again || g[static_cast<size_t>(r) * nc + r] < 0.25;
    if (!again) break;
  }
  if (S == 0) dts(st, nc, Wc, nov, nc, Wc, nov, nov, G, nc, w.ws.p);
  ds.eigh(nc, G, nc, w.w2.p);
  std::vector<double> lam(nc);
  d2h(lam.data(), w.w2.p, nc, st);
  SEQX_HIP(hipStreamSynchronize(st));
  int j0 = 0;
  while (j0 < nc && !(lam[j0] > 1e-12)) ++j0;
  int kept = nc - j0;
  if (kept > max_keep) {
    j0 = nc - max_keep;
    kept = max_keep;
  }
  if (kept <= 0) return 0;
  hipLaunchKernelGGL(invsqrt_cols_kernel, dim3(kept), dim3(64), 0, st, G, nc, nc, j0, w.w2.p);
  SEQX_LAUNCH_CHECK();
  // V[S + r] = sum_c Q(c, j0 + r) W_c
  comb(st, kept, nov, nc, 1.0, G + static_cast<long>(j0) * nc, nc, Wc, nov, 0.0, V + static_cast<long>(S) * nov, nov);
  return kept;
}

}  // namespace

void finalize_roots(DeviceMolecule& m, int theory, int K, const double* om, const double* Tv, const double* Uv,
                    SigmaWork& sig, DBuf<double>& scratch, hipStream_t st) {
  const long nov = static_cast<long>(m.nocc) * m.nvirt;
  const bool tdhf = theory == 1;
  m.omega.ensure(K);
  m.X.ensure(static_cast<size_t>(K) * nov);
  m.Y.ensure(static_cast<size_t>(K) * nov);
  m.f.ensure(K);
  m.mu.ensure(3 * K);
  copy(st, m.omega.p, om, K);
  hipLaunchKernelGGL(finalize_kernel, dim3(ceil_div(nov, 256), K), dim3(256), 0, st, nov, tdhf ? 1 : 0, Tv, Uv,
                     m.X.p, m.Y.p);
  hipLaunchKernelGGL(sign_fix_kernel, dim3(K), dim3(256), 0, st, nov, m.X.p, m.Y.p);
  SEQX_LAUNCH_CHECK();
  // transition densities of X + Y (T for TDHF, X for CIS)
  const long nn = static_cast<long>(m.nao) * m.nao;
  scratch.ensure(static_cast<size_t>(K) * (nov + nn));
  double* T = scratch.p;
  double* TA = scratch.p + static_cast<long>(K) * nov;
  copy(st, T, m.X.p, K * nov);
  axpby(st, K * nov, 1.0, m.Y.p, 1.0, T);
  forward_transform(m, K, T, TA, sig, st);
  hipLaunchKernelGGL(dipole_kernel, dim3(K), dim3(256), 0, st, m.natoms, m.nao, TA, m.slot.p, m.ao_off.p, m.xyz.p,
                     m.elems, m.omega.p, m.mu.p, m.f.p);
  SEQX_LAUNCH_CHECK();
  SEQX_HIP(hipStreamSynchronize(st));
  m.nroots = K;
  m.theory = theory;
}

bool davidson_f32_basis(long nov, int precision) {
  return precision != kPrecFP64 && nov % 4 == 0 && nov >= 4096;
}

DavResult davidson(DeviceMolecule& m, const DavOptions& opt, DenseSolver& ds, DavWork& w, hipStream_t st) {
  const int o = m.nocc, v = m.nvirt, Kreq = opt.nroots;
  const long nov = static_cast<long>(o) * v;
  const bool tdhf = opt.theory == 1;
  if (Kreq < 1 || Kreq > nov) throw Error(kEArg, "nroots must be in [1, nocc*nvirt]");
  // K Ritz pairs are iterated: the Kreq wanted ones and the guard roots above them
  const int K = static_cast<int>(std::min<long>(nov, Kreq + std::max(0, opt.nguard)));
  int Smax = opt.max_sub > 0 ? opt.max_sub : 20 * K + 40;
  Smax = static_cast<int>(std::min<long>(Smax, nov));
  const int ncand_max = tdhf ? 2 * K : K;
  Smax = std::max(Smax, std::min<int>(static_cast<int>(nov), 2 * K + ncand_max));
  const int ng = opt.guess ? opt.nguess : static_cast<int>(std::min<long>(nov, 2L * K));
  if (opt.nlock > 0 && (!opt.lock_u || !(opt.shift > 0.0))) throw Error(kEArg, "locked roots need vectors and a shift");
  if (ng < 1 || ng > Smax) throw Error(kEArg, "guess size out of range");
  DavResult res;
  res.subspace_cap = Smax;
  const double t0 = now_s();

  w.V.ensure(static_cast<size_t>(Smax) * nov);
  // products of basis vector s: row ps*s holds (A+B)V_s (CIS: A V_s), row ps*s+1 holds (A-B)V_s
  const int ps = tdhf ? 2 : 1;
  const long ldp = ps * nov;
  w.SP.ensure(static_cast<size_t>(ps) * Smax * nov);
  w.Mp.ensure(static_cast<size_t>(Smax) * Smax);
  w.Mm.ensure(static_cast<size_t>(Smax) * Smax);
  w.Lm.ensure(static_cast<size_t>(Smax) * Smax);
  w.Tmp.ensure(static_cast<size_t>(Smax) * Smax);
  w.Hs.ensure(static_cast<size_t>(Smax) * Smax);
  w.w2.ensure(Smax);
  // Restarts keep, beside the current Ritz coefficients, those of the
  // previous iteration (padded with zeros for the rows added since): the
  // basis after a collapse spans both, as in a locally optimal block
  // iteration, which keeps most of the convergence rate of the unrestarted
  // iteration.  Two coefficient buffers alternate between iterations.
  const int q_ritz = 2 * K;                    // TDHF: t, u of K roots; CIS: 2K eigenvectors
  const int q_prev = opt.keep_prev ? (tdhf ? 2 * K : K) : 0;
  const bool use_prev = q_prev > 0 && q_ritz + q_prev + ncand_max <= Smax;
  const int q_max = q_ritz + (use_prev ? q_prev : 0);
  w.coef.ensure(static_cast<size_t>(Smax) * 4 * K);
  // Ritz rows: Tv holds [T; U] (U only for TDHF), PT holds [(A+B)T; (A-B)U] (CIS: A X)
  w.Tv.ensure(static_cast<size_t>(ps) * K * nov);
  w.PT.ensure(static_cast<size_t>(ps) * K * nov);
  double* Uv = w.Tv.p + static_cast<long>(K) * nov;
  double* MU = w.PT.p + static_cast<long>(K) * nov;
  // the low-precision phase keeps its Ritz vectors and products in FP32 (the
  // same storage holds them): they feed only residual norms and FP32 corrections
  float* Tv32 = reinterpret_cast<float*>(w.Tv.p);
  float* Uv32 = Tv32 + static_cast<long>(K) * nov;
  float* PT32 = reinterpret_cast<float*>(w.PT.p);
  float* MU32 = PT32 + static_cast<long>(K) * nov;
  w.W.ensure(static_cast<size_t>(std::max(ncand_max, opt.guess ? opt.nguess : 0)) * nov);
  w.scratch.ensure(static_cast<size_t>(ps) * q_max * nov);
  w.G.ensure(static_cast<size_t>(ps) * Smax * Smax);
  w.Q.ensure(static_cast<size_t>(std::max(ncand_max, q_max)) * Smax);
  // FP32 basis rows and products while the products are formed in low
  // precision (their own rounding is far coarser); FP64 after the switch
  bool lb = davidson_f32_basis(nov, opt.precision);
  if (lb) {
    w.V32.ensure(static_cast<size_t>(Smax) * nov);
    w.SP32.ensure(static_cast<size_t>(ps) * Smax * nov);
    w.scr32.ensure(static_cast<size_t>(ps) * q_max * nov);
  }
  w.ws.ensure(std::max<size_t>(dots_workspace(2 * Smax, std::max(Smax, opt.nlock), nov), 4096));
  w.d.ensure(nov);
  w.rn.ensure(2 * K + 3);  // residual norms, omega, then the check words (lowest eigenvalue, eigh / potrf info)
  const int nbres = static_cast<int>(std::min<long>(256, ceil_div(nov, 256)));
  w.part.ensure(static_cast<size_t>(K) * nbres);
  w.idx.ensure(std::max(ng, 1));
  w.sel.ensure(K);
  m.omega.ensure(K);
  m.X.ensure(static_cast<size_t>(K) * nov);
  m.Y.ensure(static_cast<size_t>(K) * nov);
  m.f.ensure(K);
  m.mu.ensure(3 * K);
  double* om = w.rn.p + K;  // omega of the current iteration (hartree)

  hipLaunchKernelGGL(gap_kernel, dim3(ceil_div(nov, 256)), dim3(256), 0, st, o, v, m.eps.p, w.d.p);
  int S = 0, knew = 0;
  if (opt.guess) {
    copy(st, w.W.p, opt.guess, static_cast<long>(opt.nguess) * nov);
    knew = lb ? orthonormalize_append(st, ds, w, nov, opt.nguess, w.W.p, 0, w.V32.p, Smax)
              : orthonormalize_append(st, ds, w, nov, opt.nguess, w.W.p, 0, w.V.p, Smax);
    if (knew == 0) throw Error(kEArg, "user guess vectors are linearly dependent or zero");
  } else {
    // with locked roots: unit vectors at the ng gaps that follow the nlock smallest
    const int skip = static_cast<int>(std::min<long>(opt.nlock, nov - ng));
    w.idx.ensure(skip + ng);
    hipLaunchKernelGGL(gap_guess_kernel, dim3(1), dim3(1024), 0, st, o, v, skip + ng, m.eps.p, w.idx.p);
    if (lb)
      hipLaunchKernelGGL(unit_vectors_kernel<float>, dim3(ceil_div(nov, 256), ng), dim3(256), 0, st, ng, nov,
                         w.idx.p + skip, w.V32.p);
    else
      hipLaunchKernelGGL(unit_vectors_kernel<double>, dim3(ceil_div(nov, 256), ng), dim3(256), 0, st, ng, nov,
                         w.idx.p + skip, w.V.p);
    SEQX_LAUNCH_CHECK();
    knew = ng;
  }
  // deflation of the locked roots: out_s += shift * sum_m U_m (U_m . V_s) for
  // the nv new vectors (their products nv rows of stride ldp from sp)
  auto deflate = [&](const auto* Vn, int nv, auto* sp) {
    if (opt.nlock <= 0 || nv <= 0) return;
    w.lc.ensure(static_cast<size_t>(nv) * opt.nlock);
    dts(st, nv, Vn, nov, opt.nlock, opt.lock_u, nov, nov, w.lc.p, opt.nlock, w.ws.p);
    comb(st, nv, nov, opt.nlock, opt.shift, w.lc.p, opt.nlock, opt.lock_u, nov, 1.0, sp, ldp);
  };

  std::vector<double> h_om(K), h_rn(K), h_chk(2 * K + 3);
  std::vector<int> sel;
  hipEvent_t e0, e1;
  IterTimer itimer(st);
  SEQX_HIP(hipEventCreate(&e0));
  SEQX_HIP(hipEventCreate(&e1));
  // Collapse the basis of size S onto the span of the best Ritz vectors
  // (TDHF: the 2K vectors t, u; CIS: the 2K lowest eigenvectors); V stays
  // orthonormal.  products: carry the products and projected matrices along
  // (else the caller recomputes them).  Returns the new basis size.
  // prev: the previous iteration's coefficients (rows [0, s_prev)) or null.
  // to64: the collapsed rows of an FP32 basis go to FP64 scratch (without products).
  auto collapse = [&](int S, bool products, const double* tco, const double* prev, int s_prev,
                      bool to64 = false) -> int {
    const int qr = tdhf ? 2 * K : std::min(2 * K, S);
    // coefficient block Cc (S x q0) = [t u] (TDHF) or the qr lowest eigenvectors
    // (CIS), then the previous coefficients
    double* Cc = w.Q.p;
    if (tdhf) {
      copy(st, Cc, tco, static_cast<long>(2 * K) * Smax);  // t and u are adjacent columns
    } else {
      copy(st, Cc, w.Hs.p, static_cast<long>(qr) * Smax);
    }
    // Orthonormal columns spanning C (S x nc, ld Smax), written to out (ld Smax):
    // C Z diag(lam^-1/2) over the eigenpairs of C^T C with lam > lmin; returns
    // their number.  lmin < 0: relative, -lmin times the largest eigenvalue.
    auto orth_cols = [&](const double* C, int nc, double lmin, double* out) -> int {
      dgemm_cm(st, true, false, nc, nc, S, 1.0, C, Smax, C, Smax, 0.0, w.G.p, nc);
      ds.eigh(nc, w.G.p, nc, w.w2.p);
      std::vector<double> lam(nc);
      d2h(lam.data(), w.w2.p, nc, st);
      SEQX_HIP(hipStreamSynchronize(st));
      const double lo = lmin < 0.0 ? -lmin * lam[nc - 1] : lmin;
      int j0 = 0;
      while (j0 < nc && !(lam[j0] > lo)) ++j0;
      const int kept = nc - j0;
      if (kept <= 0) return 0;
      hipLaunchKernelGGL(invsqrt_cols_kernel, dim3(kept), dim3(64), 0, st, w.G.p, nc, nc, j0, w.w2.p);
      dgemm_cm(st, false, false, S, kept, nc, 1.0, C, Smax, w.G.p + static_cast<long>(j0) * nc, nc, 0.0, out, Smax);
      return kept;
    };
    int q0 = qr;
    if (prev) {
      hipLaunchKernelGGL(pad_cols_kernel, dim3(ceil_div(S, 256), q_prev), dim3(256), 0, st, s_prev, S, prev,
                         Cc + static_cast<long>(qr) * Smax, Smax);
      SEQX_LAUNCH_CHECK();
      q0 += q_prev;
    }
    int q = orth_cols(Cc, q0, -1e-12, w.Lm.p);
    if (prev) {
      // the previous coefficients of converging roots nearly repeat the
      // current ones, so their directions come out of C^T C with a small lam
      // and rounding errors scaled by lam^-1/2; a second pass over the (nearly
      // orthonormal) result restores orthonormality to working precision
      copy(st, w.Hs.p, w.Lm.p, static_cast<long>(q) * Smax);
      q = orth_cols(w.Hs.p, q, -1e-12, w.Lm.p);
    }
    double* Qc = w.Lm.p;
    if (lb && to64) {
      // leaving the FP32 basis: the collapsed rows in FP64, in scratch (the
      // caller orthonormalises them into the FP64 basis)
      comb(st, q, nov, S, 1.0, Qc, Smax, w.V32.p, nov, 0.0, w.scratch.p, nov);
      return q;
    }
    if (lb) {
      comb(st, q, nov, S, 1.0, Qc, Smax, w.V32.p, nov, 0.0, w.scr32.p, nov);
      SEQX_HIP(hipMemcpyAsync(w.V32.p, w.scr32.p, static_cast<size_t>(q) * nov * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
      if (!products) return q;
      for (int p = 0; p < ps; ++p)
        comb(st, q, nov, S, 1.0, Qc, Smax, w.SP32.p + p * nov, ldp, 0.0, w.scr32.p + p * nov, ldp);
      SEQX_HIP(hipMemcpyAsync(w.SP32.p, w.scr32.p, static_cast<size_t>(q) * ldp * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
    } else {
      dgemm(st, false, false, q, static_cast<int>(nov), S, 1.0, Qc, Smax, 0, w.V.p, nov, 0, 0.0, w.scratch.p, nov, 0,
            1, nullptr);
      copy(st, w.V.p, w.scratch.p, static_cast<long>(q) * nov);
      if (!products) return q;
      for (int p = 0; p < ps; ++p)  // keep the interleaved product rows interleaved
        dgemm(st, false, false, q, static_cast<int>(nov), S, 1.0, Qc, Smax, 0, w.SP.p + p * nov, ldp, 0, 0.0,
              w.scratch.p + p * nov, ldp, 0, 1, nullptr);
      copy(st, w.SP.p, w.scratch.p, static_cast<long>(q) * ldp);
    }
    for (double* Mx : {w.Mp.p, tdhf ? w.Mm.p : nullptr}) {
      if (!Mx) continue;
      dgemm_cm(st, false, false, S, q, S, 1.0, Mx, Smax, Qc, Smax, 0.0, w.Tmp.p, Smax);
      dgemm_cm(st, true, false, q, q, S, 1.0, Qc, Smax, w.Tmp.p, Smax, 0.0, w.Hs.p, Smax);
      copy(st, Mx, w.Hs.p, static_cast<long>(q) * Smax);
    }
    return q;
  };

  int prec = opt.precision;
  double floor_low = 0.0, rbest = 1e300, dmax = 0.0;
  int stall = 0;
  // rounding floor of the low-precision products: sums over n terms carry a
  // relative error of about sqrt(n) u, on a scale set by the largest
  // orbital-energy gap; four times that.  FP32: u = 2^-24.  Split bfloat16:
  // one product may be off by 3 * 2^-16, but the operand splits round to
  // either side and their errors largely cancel in the sums; the residuals
  // of its phase level off about 16 times above those of the FP32 phase, so
  // u = 2^-20 there (a lower floor only lengthens that phase until the
  // stall rule ends it).
  auto rounding_floor = [&](int p) {
    const double u = std::ldexp(1.0, p == kPrecBF16x3 ? -20 : -24);
    return 4.0 * std::sqrt(static_cast<double>(m.nao)) * u * dmax;
  };
  if (prec != kPrecFP64) {
    max_abs(st, nov, w.d.p, w.rn.p, w.ws.p);
    d2h(&dmax, w.rn.p, 1, st);
    SEQX_HIP(hipStreamSynchronize(st));
    floor_low = rounding_floor(prec);
  }
  // coefficients of iteration it - 1 in the basis of iteration it, unless a
  // collapse in between rotated the basis
  int s_at[2] = {0, 0}, last_collapse = 0;
  auto prev_coef = [&](int it) -> const double* {
    if (!use_prev || it < 2 || last_collapse == it - 1) return nullptr;
    return w.coef.p + static_cast<long>((it - 1) & 1) * 2 * K * Smax;
  };
  bool converged = false;
  int it = 0;
  try {
    for (it = 1; it <= opt.max_iter; ++it) {
      // 1. products of the new vectors
      itimer.mark(kDavSigma);
      SEQX_HIP(hipEventRecord(e0, st));
      double* sp_new = w.SP.p + static_cast<long>(S) * ldp;
      float* sp_new32 = lb ? w.SP32.p + static_cast<long>(S) * ldp : nullptr;
      if (lb) {
        sigma_build_f32(m, opt.theory, knew, w.V32.p + S * nov, sp_new32, tdhf ? sp_new32 + nov : nullptr, w.sig, st,
                        opt.sigma_chunk, ldp, prec);
        deflate(w.V32.p + S * nov, knew, sp_new32);
      } else {
        sigma_build(m, opt.theory, knew, w.V.p + S * nov, sp_new, tdhf ? sp_new + nov : nullptr, w.sig, st,
                    opt.sigma_chunk, ldp, prec);
        deflate(w.V.p + S * nov, knew, sp_new);
      }
      SEQX_HIP(hipEventRecord(e1, st));
      itimer.mark(kDavProject);
      res.n_sigma += knew;
      if (prec == kPrecFP64) res.n_sigma_fp64 += knew;
      if (prec == kPrecBF16x3) res.n_sigma_bf16x3 += knew;
      const int S1 = S + knew;
      // 2. projected matrices, new columns (column-major, ld = Smax): one pass over
      // V for (A+B) and (A-B) together, since their rows are interleaved
      if (lb)
        dts(st, ps * knew, sp_new32, nov, S1, w.V32.p, nov, nov, w.G.p, S1, w.ws.p);
      else
        dots(st, ps * knew, sp_new, nov, S1, w.V.p, nov, nov, w.G.p, S1, w.ws.p);
      hipLaunchKernelGGL(scatter_cols_kernel, dim3(ceil_div(S1, 256), ps * knew), dim3(256), 0, st, w.G.p, S1, ps, S,
                         w.Mp.p, w.Mm.p, Smax);
      hipLaunchKernelGGL(sym_fill_kernel, dim3(ceil_div(S1, 256), knew), dim3(256), 0, st, w.Mp.p, Smax, S, S1);
      if (tdhf)
        hipLaunchKernelGGL(sym_fill_kernel, dim3(ceil_div(S1, 256), knew), dim3(256), 0, st, w.Mm.p, Smax, S, S1);
      SEQX_LAUNCH_CHECK();
      S = S1;
      res.max_subspace = std::max(res.max_subspace, S);
      // 3. subspace eigenproblem
      itimer.mark(kDavSmallEig);
      // t (TDHF) or x (CIS): S x K, ld Smax; u (TDHF) next to it
      double* tco = w.coef.p + static_cast<long>(it & 1) * 2 * K * Smax;
      double* uco = tco + static_cast<long>(K) * Smax;
      s_at[it & 1] = S;
      if (tdhf) {
        copy(st, w.Lm.p, w.Mm.p, static_cast<long>(S) * Smax);
        ds.potrf(S, w.Lm.p, Smax);
        zero_upper_cm(st, S, w.Lm.p, Smax);
        dgemm_cm(st, false, false, S, S, S, 1.0, w.Mp.p, Smax, w.Lm.p, Smax, 0.0, w.Tmp.p, Smax);  // M+ L
        dgemm_cm(st, true, false, S, S, S, 1.0, w.Lm.p, Smax, w.Tmp.p, Smax, 0.0, w.Hs.p, Smax);    // L^T M+ L
        ds.eigh_lowest(S, w.Hs.p, Smax, K, w.w2.p);  // only the K lowest pairs are used
        hipLaunchKernelGGL(omega_kernel, dim3(ceil_div(K, 64)), dim3(64), 0, st, K, w.w2.p, om, 1);
        dgemm_cm(st, false, false, S, K, S, 1.0, w.Lm.p, Smax, w.Hs.p, Smax, 0.0, tco, Smax);   // L z
        dgemm_cm(st, false, false, S, K, S, 1.0, w.Tmp.p, Smax, w.Hs.p, Smax, 0.0, uco, Smax);  // M+ L z
        hipLaunchKernelGGL(scale_cols_kernel, dim3(K), dim3(256), 0, st, tco, Smax, S, K, om, 0.5);
        hipLaunchKernelGGL(scale_cols_kernel, dim3(K), dim3(256), 0, st, uco, Smax, S, K, om, 1.5);
      } else {
        copy(st, w.Hs.p, w.Mp.p, static_cast<long>(S) * Smax);
        ds.eigh_lowest(S, w.Hs.p, Smax, std::min(2 * K, S), w.w2.p);  // K Ritz pairs, 2K for a collapse
        hipLaunchKernelGGL(omega_kernel, dim3(ceil_div(K, 64)), dim3(64), 0, st, K, w.w2.p, om, 0);
        copy(st, tco, w.Hs.p, static_cast<long>(K) * Smax);
      }
      SEQX_LAUNCH_CHECK();
      // 4. Ritz vectors and products: rows j of Tv = sum_s t(s, j) V_s, etc.
      itimer.mark(kDavRitz);
      // [T; U] in one pass over V (t and u are adjacent coefficient columns)
      if (lb) {
        comb(st, ps * K, nov, S, 1.0, tco, Smax, w.V32.p, nov, 0.0, Tv32, nov);
        comb(st, K, nov, S, 1.0, tco, Smax, w.SP32.p, ldp, 0.0, PT32, nov);
        if (tdhf) comb(st, K, nov, S, 1.0, uco, Smax, w.SP32.p + nov, ldp, 0.0, MU32, nov);
      } else {
        dgemm(st, false, false, ps * K, static_cast<int>(nov), S, 1.0, tco, Smax, 0, w.V.p, nov, 0, 0.0, w.Tv.p, nov,
              0, 1, nullptr);
        dgemm(st, false, false, K, static_cast<int>(nov), S, 1.0, tco, Smax, 0, w.SP.p, ldp, 0, 0.0, w.PT.p, nov, 0, 1,
              nullptr);
        if (tdhf)
          dgemm(st, false, false, K, static_cast<int>(nov), S, 1.0, uco, Smax, 0, w.SP.p + nov, ldp, 0, 0.0, MU, nov,
                0, 1, nullptr);
      }
      // 5. residual norms
      if (lb)
        hipLaunchKernelGGL(residual_norm_kernel<float>, dim3(nbres, K), dim3(256), 0, st, nov, tdhf ? 1 : 0, om, Tv32,
                           Uv32, PT32, MU32, w.part.p);
      else
        hipLaunchKernelGGL(residual_norm_kernel<double>, dim3(nbres, K), dim3(256), 0, st, nov, tdhf ? 1 : 0, om,
                           w.Tv.p, Uv, w.PT.p, MU, w.part.p);
      hipLaunchKernelGGL(reduce_rows_kernel, dim3(ceil_div(K, 64)), dim3(64), 0, st, K, nbres, w.part.p, w.rn.p);
      SEQX_LAUNCH_CHECK();
      itimer.mark(kDavCheck);
      // one copy to the host: residual norms, omega, the lowest eigenvalue of
      // the projected problem (TDHF: omega^2) and the eigh / potrf info words
      hipLaunchKernelGGL(check_words_kernel, dim3(1), dim3(64), 0, st, w.w2.p, ds.info_device(), w.rn.p + 2 * K);
      SEQX_LAUNCH_CHECK();
      d2h(h_chk.data(), w.rn.p, 2 * K + 3, st);
      SEQX_HIP(hipStreamSynchronize(st));
      std::copy(h_chk.begin(), h_chk.begin() + K, h_rn.begin());
      std::copy(h_chk.begin() + K, h_chk.begin() + 2 * K, h_om.begin());
      const double h_w2min = h_chk[2 * K];
      const int h_info[2] = {static_cast<int>(h_chk[2 * K + 1]), static_cast<int>(h_chk[2 * K + 2])};
      float ms = 0.f;
      SEQX_HIP(hipEventElapsedTime(&ms, e0, e1));
      res.t_sigma_ms += ms;
      if (tdhf && h_info[1] != 0)
        throw Error(kEUnstable, "A-B projected matrix not positive definite (unstable reference)");
      if (h_info[0] != 0) throw Error(kEDevice, "subspace eigensolver failed");
      // omega^2 <= 0: the projected A+B is not positive definite (L^T M+ L has
      // the inertia of M+), an imaginary or zero TDHF root
      if (tdhf && !(h_w2min > 0.0))
        throw Error(kEUnstable, "A+B projected matrix not positive definite (unstable reference)");
      res.t_iter.push_back(now_s() - t0);
      res.omega_iter.push_back(std::vector<double>(h_om.begin(), h_om.begin() + Kreq));
      if (log_enabled()) {
        double rmax = 0.0;
        for (double r : h_rn) rmax = std::max(rmax, r);
        std::fprintf(stderr,
                     "{\"davidson_iter\": %d, \"subspace\": %d, \"new\": %d, \"max_residual\": %.3e, "
                     "\"omega0_eV\": %.9f, \"omegaK_eV\": %.9f, \"t_s\": %.4f}\n",
                     it, S, knew, rmax, h_om[0] * kHartreeEV, h_om[K - 1] * kHartreeEV, res.t_iter.back());
      }
      sel.clear();
      double rmax = 0.0;  // over the wanted roots
      bool wanted_done = true;
      for (int j = 0; j < K; ++j) {
        if (!std::isfinite(h_rn[j]) || !std::isfinite(h_om[j])) throw Error(kEDavNoConv, "Davidson produced NaN");
        if (h_rn[j] > opt.tol) {
          sel.push_back(j);
          if (j < Kreq) wanted_done = false;
        }
        if (j < Kreq) rmax = std::max(rmax, h_rn[j]);
      }
      if (prec == kPrecFP64 && wanted_done) {
        converged = true;
        break;
      }
      if (it == opt.max_iter) break;
      if (prec != kPrecFP64) {
        // Mixed-precision phase: the residuals cannot fall much below the
        // rounding floor of the low-precision products.  Restart from the
        // Ritz vectors with products of the next precision (split bfloat16
        // -> FP32 -> FP64) once every root is below max(tol, floor), or once
        // the largest residual, within 4x of the floor, has not halved for
        // four iterations.
        if (rmax < 4.0 * floor_low) {
          stall = rmax < 0.5 * rbest ? 0 : stall + 1;
          rbest = std::min(rbest, rmax);
        }
        // the split-bfloat16 phase ends after max_iter / 3 iterations at the
        // latest, should its residuals level off above the stall window
        const bool bf_cap = prec == kPrecBF16x3 && it >= std::max(20, opt.max_iter / 3);
        if (rmax <= std::max(opt.tol, floor_low) || stall >= 4 || bf_cap) {
          const bool to_fp32 = prec == kPrecBF16x3 && rmax > opt.tol;
          if (log_enabled())
            std::fprintf(stderr, "{\"%s_after_iter\": %d, \"max_residual\": %.3e, \"floor\": %.3e}\n",
                         to_fp32 ? "fp32" : "refine", it, rmax, floor_low);
          itimer.mark(kDavCollapse);
          S = collapse(S, false, w.coef.p + static_cast<long>(it & 1) * 2 * K * Smax, prev_coef(it), s_at[(it - 1) & 1],
                       !to_fp32);
          last_collapse = it;
          if (to_fp32) {
            // same basis (FP32 rows, or FP64 rows for short vectors), products
            // formed again on the FP32 matrix cores
            knew = S;
            S = 0;
            prec = kPrecFP32;
            floor_low = rounding_floor(prec);
            rbest = 1e300;
            stall = 0;
            res.fp32_iter = it + 1;
            continue;
          }
          if (lb) {
            // FP32 rows are orthonormal to about 1e-7: orthonormalise them again in FP64
            itimer.mark(kDavOrtho);
            knew = orthonormalize_append(st, ds, w, nov, S, w.scratch.p, 0, w.V.p, Smax);
            lb = false;
          } else {
            knew = S;
          }
          S = 0;
          prec = kPrecFP64;
          res.refine_iter = it + 1;
          continue;
        }
      }
      // 6. preconditioned residuals of the unconverged roots
      itimer.mark(kDavPrecond);
      const int nsel = static_cast<int>(sel.size());
      SEQX_HIP(hipMemcpyAsync(w.sel.p, sel.data(), nsel * sizeof(int), hipMemcpyHostToDevice, st));
      // FP32 correction rows beside an FP32 basis (W's storage holds twice as many)
      float* W32 = reinterpret_cast<float*>(w.W.p);
      if (lb)
        hipLaunchKernelGGL((precond_kernel<float, float>), dim3(ceil_div(nov, 256), nsel), dim3(256), 0, st, nov,
                           tdhf ? 1 : 0, w.sel.p, om, w.d.p, Tv32, Uv32, PT32, MU32, W32);
      else
        hipLaunchKernelGGL((precond_kernel<double, double>), dim3(ceil_div(nov, 256), nsel), dim3(256), 0, st, nov,
                           tdhf ? 1 : 0, w.sel.p, om, w.d.p, w.Tv.p, Uv, w.PT.p, MU, w.W.p);
      SEQX_LAUNCH_CHECK();
      const int nc = tdhf ? 2 * nsel : nsel;
      // 7. collapse onto the best Ritz vectors when the basis would overflow
      itimer.mark(kDavCollapse);
      if (S + nc > Smax) {
        S = collapse(S, true, w.coef.p + static_cast<long>(it & 1) * 2 * K * Smax, prev_coef(it), s_at[(it - 1) & 1]);
        last_collapse = it;
        ++res.n_collapses;
      }
      // 8. orthonormalise and append
      itimer.mark(kDavOrtho);
      knew = lb ? orthonormalize_append(st, ds, w, nov, nc, W32, S, w.V32.p, Smax - S)
                : orthonormalize_append(st, ds, w, nov, nc, w.W.p, S, w.V.p, Smax - S);
      if (knew == 0) break;
    }
    itimer.mark(kDavSigma);
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  res.iterations = it;
  itimer.accumulate(res.phase_ms);
  if (!converged) throw Error(kEDavNoConv, "Davidson did not converge in " + std::to_string(opt.max_iter) + " iterations");

  // 9. amplitudes, sign convention, properties of the wanted roots
  finalize_roots(m, opt.theory, Kreq, om, w.Tv.p, Uv, w.sig, w.scratch, st);
  m.nroots = Kreq;
  m.theory = opt.theory;
  m.dav_iterations = it;
  m.n_sigma = res.n_sigma;
  return res;
}

__global__ void pair_rows_kernel(long nov, int K, const double* __restrict__ X, const double* __restrict__ Y,
                                 double* __restrict__ T, double* __restrict__ U) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= nov) return;
  const long b = static_cast<long>(j) * nov + x;
  T[b] = X[b] + Y[b];
  if (U) U[b] = X[b] - Y[b];
}

DavResult davidson_root_batches(DeviceMolecule& m, const DavOptions& opt, int batch, DenseSolver& ds, DavWork& w,
                                DBuf<double>& lock_t, DBuf<double>& lock_u, hipStream_t st) {
  const int K = opt.nroots, n = m.nao;
  const long nov = static_cast<long>(m.nocc) * m.nvirt;
  const bool tdhf = opt.theory == 1;
  if (batch < 1 || batch >= K) throw Error(kEArg, "root batch must be in [1, nroots)");
  if (opt.guess) throw Error(kEArg, "root batches start from the gap guess");
  lock_t.ensure(static_cast<size_t>(K) * nov);
  if (tdhf) lock_u.ensure(static_cast<size_t>(K) * nov);
  // spread of the orbital energies: every target root lies below it
  std::vector<double> eps(n);
  d2h(eps.data(), m.eps.p, n, st);
  SEQX_HIP(hipStreamSynchronize(st));
  const double D = eps[n - 1] - eps[0];
  DavResult total;
  std::vector<double> om_all;
  double t_off = 0.0;
  for (int k0 = 0; k0 < K; k0 += batch) {
    const int kb = std::min(batch, K - k0);
    DavOptions ob = opt;
    ob.nroots = kb;
    ob.nlock = k0;
    ob.lock_t = lock_t.p;
    ob.lock_u = tdhf ? lock_u.p : lock_t.p;
    // locked roots move to w + s (CIS) or sqrt(w (w + s)) (TDHF), at least 2 D either way
    const double wmin = k0 > 0 ? *std::min_element(om_all.begin(), om_all.end()) : 1.0;
    ob.shift = tdhf ? 4.0 * D * D / std::max(wmin, 1e-3) : 2.0 * D;
    DavResult r = davidson(m, ob, ds, w, st);
    hipLaunchKernelGGL(pair_rows_kernel, dim3(ceil_div(nov, 256), kb), dim3(256), 0, st, nov, kb, m.X.p, m.Y.p,
                       lock_t.p + static_cast<long>(k0) * nov, tdhf ? lock_u.p + static_cast<long>(k0) * nov : nullptr);
    SEQX_LAUNCH_CHECK();
    std::vector<double> om(kb);
    d2h(om.data(), m.omega.p, kb, st);
    SEQX_HIP(hipStreamSynchronize(st));
    // history: locked roots at their final values, this batch's Ritz values, NaN beyond
    for (size_t it = 0; it < r.t_iter.size(); ++it) {
      total.t_iter.push_back(t_off + r.t_iter[it]);
      std::vector<double> row(K, std::nan(""));
      for (int j = 0; j < k0; ++j) row[j] = om_all[j];
      for (int j = 0; j < kb; ++j) row[k0 + j] = r.omega_iter[it][j];
      total.omega_iter.push_back(row);
    }
    if (!r.t_iter.empty()) t_off += r.t_iter.back();
    om_all.insert(om_all.end(), om.begin(), om.end());
    for (int p = 0; p < kNumDavPhases; ++p) total.phase_ms[p] += r.phase_ms[p];
    total.iterations += r.iterations;
    total.n_sigma += r.n_sigma;
    total.n_sigma_fp64 += r.n_sigma_fp64;
    total.n_sigma_bf16x3 += r.n_sigma_bf16x3;
    total.fp32_iter = std::max(total.fp32_iter, r.fp32_iter);
    total.refine_iter = std::max(total.refine_iter, r.refine_iter);
    total.t_sigma_ms += r.t_sigma_ms;
    total.max_subspace = std::max(total.max_subspace, r.max_subspace);
    total.subspace_cap = std::max(total.subspace_cap, r.subspace_cap);
    total.n_collapses += r.n_collapses;
  }
  // all K roots in ascending order
  std::vector<int> perm(K);
  for (int j = 0; j < K; ++j) perm[j] = j;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return om_all[a] < om_all[b]; });
  std::vector<double> om_sorted(K);
  for (int j = 0; j < K; ++j) om_sorted[j] = om_all[perm[j]];
  DBuf<double> omd(K);
  SEQX_HIP(hipMemcpyAsync(omd.p, om_sorted.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
  bool ordered = true;
  for (int j = 0; j < K; ++j) ordered = ordered && perm[j] == j;
  const double* T = lock_t.p;
  const double* U = tdhf ? lock_u.p : lock_t.p;
  DBuf<double> Ts, Us;
  if (!ordered) {
    Ts.alloc(static_cast<size_t>(K) * nov);
    if (tdhf) Us.alloc(static_cast<size_t>(K) * nov);
    for (int j = 0; j < K; ++j) {
      copy(st, Ts.p + static_cast<long>(j) * nov, lock_t.p + static_cast<long>(perm[j]) * nov, nov);
      if (tdhf) copy(st, Us.p + static_cast<long>(j) * nov, lock_u.p + static_cast<long>(perm[j]) * nov, nov);
    }
    T = Ts.p;
    U = tdhf ? Us.p : Ts.p;
  }
  finalize_roots(m, opt.theory, K, omd.p, T, U, w.sig, w.scratch, st);
  m.dav_iterations = total.iterations;
  m.n_sigma = total.n_sigma;
  return total;
}

}  // namespace seqx
