// Closed-shell RHF SCF with Pulay DIIS, entirely on the device.
//
// Ground-state subsection of the paper: F C = C eps with the NDDO overlap
// replaced by the identity; the lowest nocc MOs are doubly occupied.
//   F = H + J(P) - K(P)/2,  P = 2 C_occ C_occ^T
// Guess: diagonal density (each atom's core charge spread evenly over its AOs),
// turned into the first idempotent density.  Converged when max |F P - P F| <=
// tol.  Inside the loop the aufbau density of the (DIIS-extrapolated) Fock
// matrix comes from SP2 purification (GEMMs only); the orbitals of the
// converged Fock matrix come from one dense eigensolve (rocSOLVER divide and
// conquer) at the end.  The host reads the commutator norm once per iteration
// and two traces per purification step.
#include <algorithm>

#include "gemm.hpp"
#include "scf.hpp"

namespace seqx {

namespace {

// P = 2 C_occ C_occ^T from MO-major eigenvectors CT (row p = MO p)
void density_from_CT(hipStream_t st, int n, int o, const double* CT, double* P) {
  dgemm(st, true, false, n, n, o, 2.0, CT, n, 0, CT, n, 0, 0.0, P, n, 0, 1, nullptr);
}

void fock(const DeviceMolecule& m, const double* P, double* G, double* F, GWork& gw, hipStream_t st) {
  const long nn = static_cast<long>(m.nao) * m.nao;
  build_G(m, 1, P, nn, G, nullptr, nn, kSymm, 1.0, -0.5, 0.0, gw, st);
  copy(st, F, m.H.p, nn);
  axpby(st, nn, 1.0, G, 1.0, F);
}

double read_scalar(const double* d, hipStream_t st) {
  double v = 0;
  SEQX_HIP(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st));
  SEQX_HIP(hipStreamSynchronize(st));
  return v;
}

// Gershgorin bounds of a symmetric matrix: per row lo = F_ii - sum_j!=i |F_ij|,
// hi = F_ii + sum_j!=i |F_ij|; one block per row
__global__ void gershgorin_rows_kernel(int n, const double* __restrict__ F, double* __restrict__ lohi) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const double* row = F + static_cast<long>(i) * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    if (j != i) s += fabs(row[j]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lohi[2 * i] = row[i] - red[0];
    lohi[2 * i + 1] = row[i] + red[0];
  }
}

// scal[0] = min lo, scal[1] = max hi
__global__ void bounds_reduce_kernel(int n, const double* __restrict__ lohi, double* __restrict__ scal) {
  __shared__ double lo[256], hi[256];
  double a = 1e300, b = -1e300;
  for (int i = threadIdx.x; i < n; i += 256) {
    a = fmin(a, lohi[2 * i]);
    b = fmax(b, lohi[2 * i + 1]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + h]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = lo[0];
    scal[1] = hi[0];
  }
}

// X = (hi I - F) / (hi - lo): spectrum mapped into [0, 1], occupied levels near 1
__global__ void sp2_init_kernel(int n, const double* __restrict__ F, const double* __restrict__ scal,
                                double* __restrict__ X) {
  const long idx = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<long>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  const double lo = scal[0], hi = scal[1];
  X[idx] = ((i == j ? hi : 0.0) - F[idx]) / (hi - lo);
}

// out[0] = tr X, out[1] = tr X2 (single block, fixed order, FP64 sums)
template <class T>
__global__ void traces_kernel(int n, const T* __restrict__ X, const T* __restrict__ X2, double* __restrict__ out) {
  __shared__ double a[256], b[256];
  double s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    s += static_cast<double>(X[static_cast<long>(i) * n + i]);
    t += static_cast<double>(X2[static_cast<long>(i) * n + i]);
  }
  a[threadIdx.x] = s;
  b[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      a[threadIdx.x] += a[threadIdx.x + h];
      b[threadIdx.x] += b[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = b[0];
  }
}

__global__ void axpby_f32_kernel(long n, float a, const float* __restrict__ x, float b, float* __restrict__ y) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void to_double_kernel(long n, const float* __restrict__ x, double* __restrict__ y) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = static_cast<double>(x[i]);
}

// SP2 with the decisions on the device (small n, where a host round trip per
// step costs more than the step): one block forms tr X and tr X^2 and takes
// the step's decision, exactly as the host loop below does; state[0] = done,
// state[1] = branch (0: X <- X^2, 1: X <- 2X - X^2), state[2..3] = the
// previous two values of sum lambda (1 - lambda).  Once done, the decision and
// update kernels leave X alone, so steps launched past convergence are no-ops.
__global__ void sp2_state_init_kernel(double* __restrict__ state) {
  state[0] = 0.0;
  state[1] = 0.0;
  state[2] = 1e300;
  state[3] = 1e300;
}

__global__ void sp2_decide_kernel(int n, int nocc, const double* __restrict__ X, const double* __restrict__ X2,
                                  double* __restrict__ state) {
  __shared__ double a[256], b[256];
  double s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    s += X[static_cast<long>(i) * n + i];
    t += X2[static_cast<long>(i) * n + i];
  }
  a[threadIdx.x] = s;
  b[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      a[threadIdx.x] += a[threadIdx.x + h];
      b[threadIdx.x] += b[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0 || state[0] != 0.0) return;
  const double tx = a[0], tx2 = b[0], e = tx - tx2;
  if (e <= 1e-13 * n || (e < 1e-6 && e >= state[2])) {
    state[0] = 1.0;
    return;
  }
  state[2] = state[3];
  state[3] = e;
  state[1] = fabs(tx2 - nocc) < fabs(2.0 * tx - tx2 - nocc) ? 0.0 : 1.0;
}

__global__ void sp2_update_kernel(long nn, double* __restrict__ X, const double* __restrict__ X2,
                                  const double* __restrict__ state) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i >= nn || state[0] != 0.0) return;
  X[i] = state[1] == 0.0 ? X2[i] : -X2[i] + 2.0 * X[i];
}

// below this size the SP2 decisions stay on the device and the host checks
// for convergence once every kSp2Group steps
constexpr int kSp2DeviceMaxN = 512;
constexpr int kSp2Group = 4;

// FP32 purification steps go on below this sum lambda (1 - lambda) only while
// it keeps falling quadratically, down to kSp2Fp32Floor; the FP64 steps that
// follow converge quadratically from there
constexpr double kSp2Switch = 1e-2;
constexpr double kSp2Fp32Floor = 1e-4;
// FP32 steps are used for n >= kSp2MixedMinN (where the products dominate)
// while max |F P - P F| > kSp2MixedMaxErr, far above the ~1e-7 they leave
constexpr int kSp2MixedMinN = 512;
constexpr double kSp2MixedMaxErr = 1e-5;

// Second-order spectral projection (SP2, Niklasson): starting from F mapped into
// [0, 1], repeatedly apply X^2 or 2X - X^2, whichever keeps the trace closer to
// the number of occupied orbitals, until X is idempotent.  P = 2 X is the
// aufbau density of F (lowest `nocc` levels), the same as diagonalising F and
// occupying its lowest orbitals, without the eigensolver.  With fp32_first the
// steps run in FP32 (FP32 matrix-core products) until X is close to
// idempotent and finish in FP64; the result then carries FP32 rounding
// (about 1e-7 relative), which only the early SCF cycles can afford.
void sp2_density(hipStream_t st, int n, int nocc, const double* F, double* P, ScfWork& w, bool fp32_first) {
  const long nn = static_cast<long>(n) * n;
  w.X2.ensure(nn);
  double* X = w.FP.p;  // free during purification
  double* X2 = w.X2.p;
  hipLaunchKernelGGL(gershgorin_rows_kernel, dim3(n), dim3(256), 0, st, n, F, w.red.p);
  hipLaunchKernelGGL(bounds_reduce_kernel, dim3(1), dim3(256), 0, st, n, w.red.p, w.scal.p);
  hipLaunchKernelGGL(sp2_init_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, n, F, w.scal.p, X);
  SEQX_LAUNCH_CHECK();
  if (fp32_first) {
    w.X32.ensure(nn);
    w.X2_32.ensure(nn);
    float* Xs = w.X32.p;
    float* X2s = w.X2_32.p;
    to_float(st, nn, X, Xs);
    double e_prev = 1e300;
    for (int it = 0; it < 200; ++it) {
      sgemm(st, false, false, n, n, n, 1.0, Xs, n, 0, Xs, n, 0, 0.0, X2s, n, 0, 1);
      hipLaunchKernelGGL(traces_kernel<float>, dim3(1), dim3(256), 0, st, n, Xs, X2s, w.scal.p + 2);
      double tr[2];
      SEQX_HIP(hipMemcpyAsync(tr, w.scal.p + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      SEQX_HIP(hipStreamSynchronize(st));
      const double e = tr[0] - tr[1];
      // below kSp2Switch the steps converge quadratically until FP32 rounding
      // stops them: leave once e is small or no longer falls fourfold a step
      if (e < kSp2Fp32Floor || (e < kSp2Switch && e > 0.25 * e_prev)) break;
      e_prev = e;
      if (std::fabs(tr[1] - nocc) < std::fabs(2.0 * tr[0] - tr[1] - nocc)) {
        std::swap(Xs, X2s);  // X <- X^2
      } else {
        hipLaunchKernelGGL(axpby_f32_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, nn, -1.0f, X2s, 2.0f, Xs);
      }
    }
    hipLaunchKernelGGL(to_double_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, nn, Xs, X);
    SEQX_LAUNCH_CHECK();
  }
  if (!fp32_first && n < kSp2DeviceMaxN) {
    double* state = w.scal.p + 4;
    hipLaunchKernelGGL(sp2_state_init_kernel, dim3(1), dim3(1), 0, st, state);
    for (int it = 0; it < 200; it += kSp2Group) {
      for (int g = 0; g < kSp2Group; ++g) {
        dgemm(st, false, false, n, n, n, 1.0, X, n, 0, X, n, 0, 0.0, X2, n, 0, 1, nullptr);
        hipLaunchKernelGGL(sp2_decide_kernel, dim3(1), dim3(256), 0, st, n, nocc, X, X2, state);
        hipLaunchKernelGGL(sp2_update_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, nn, X, X2, state);
      }
      SEQX_LAUNCH_CHECK();
      double done = 0.0;
      SEQX_HIP(hipMemcpyAsync(&done, state, sizeof(double), hipMemcpyDeviceToHost, st));
      SEQX_HIP(hipStreamSynchronize(st));
      if (done != 0.0) break;
    }
    copy(st, P, X, nn);
    axpby(st, nn, 0.0, X, 2.0, P);
    return;
  }
  double e_prev[2] = {1e300, 1e300};
  for (int it = 0; it < 200; ++it) {
    dgemm(st, false, false, n, n, n, 1.0, X, n, 0, X, n, 0, 0.0, X2, n, 0, 1, nullptr);
    hipLaunchKernelGGL(traces_kernel<double>, dim3(1), dim3(256), 0, st, n, X, X2, w.scal.p + 2);
    double tr[2];
    SEQX_HIP(hipMemcpyAsync(tr, w.scal.p + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    SEQX_HIP(hipStreamSynchronize(st));
    const double e = tr[0] - tr[1];  // sum of lambda (1 - lambda) >= 0
    if (e <= 1e-13 * n || (e < 1e-6 && e >= e_prev[0])) break;
    e_prev[0] = e_prev[1];
    e_prev[1] = e;
    if (std::fabs(tr[1] - nocc) < std::fabs(2.0 * tr[0] - tr[1] - nocc)) {
      std::swap(X, X2);                                  // X <- X^2
    } else {
      axpby(st, nn, -1.0, X2, 2.0, X);                   // X <- 2X - X^2
    }
  }
  // the converged X and X^2 agree to rounding; keep X
  copy(st, P, X, nn);
  axpby(st, nn, 0.0, X, 2.0, P);
}

}  // namespace

void run_scf(DeviceMolecule& m, const ScfOptions& opt, DenseSolver& ds, GWork& gw, ScfWork& w, hipStream_t st) {
  const int n = m.nao, o = m.nocc;
  const long nn = static_cast<long>(n) * n;
  const int nd = std::max(1, std::min(opt.ndiis, 16));
  w.G.ensure(nn);
  w.F.ensure(nn);
  w.FP.ensure(nn);
  w.E.ensure(nn);
  w.CT.ensure(nn);
  w.Fhist.ensure(nd * nn);
  w.Ehist.ensure(nd * nn);
  w.B.ensure(nd * nd);
  w.c.ensure(nd);
  w.scal.ensure(8);
  w.red.ensure(std::max<size_t>(std::max<size_t>(1024, 2 * static_cast<size_t>(n)), dots_workspace(nd, nd, nn)));
  m.C.ensure(nn);
  m.P.ensure(nn);
  m.eps.ensure(n);

  // first density from the diagonal guess
  guess_density(st, n, m.atom_of_ao.p, m.slot.p, m.elems, m.P.p);
  fock(m, m.P.p, w.G.p, w.F.p, gw, st);
  if (opt.purify) {
    sp2_density(st, n, o, w.F.p, m.P.p, w, n >= kSp2MixedMinN);
  } else {
    copy(st, w.CT.p, w.F.p, nn);
    ds.eigh(n, w.CT.p, n, m.eps.p);
    density_from_CT(st, n, o, w.CT.p, m.P.p);
  }

  double err = 1e300;
  int it = 0, count = 0;
  for (it = 1; it <= opt.max_iter; ++it) {
    fock(m, m.P.p, w.G.p, w.F.p, gw, st);
    // commutator F P - P F = X - X^T with X = F P (F, P symmetric)
    dgemm(st, false, false, n, n, n, 1.0, w.F.p, n, 0, m.P.p, n, 0, 0.0, w.FP.p, n, 0, 1, nullptr);
    antisym(st, n, w.FP.p, w.E.p);
    max_abs(st, nn, w.E.p, w.scal.p, w.red.p);
    err = read_scalar(w.scal.p, st);
    if (!(err == err)) throw Error(kEScfNoConv, "SCF produced NaN");
    if (err <= opt.tol) break;
    const double* Fx = w.F.p;
    if (nd > 1) {
      const int slot = count % nd;
      ++count;
      copy(st, w.Fhist.p + slot * nn, w.F.p, nn);
      copy(st, w.Ehist.p + slot * nn, w.E.p, nn);
      const int mh = std::min(count, nd);
      if (mh >= 2) {
        dots(st, mh, w.Ehist.p, nn, mh, w.Ehist.p, nn, nn, w.B.p, mh, w.red.p);
        diis_coefficients(st, mh, w.B.p, mh, w.c.p);
        // F_diis (1 x nn) = c^T (1 x mh) * Fhist (mh x nn)
        dgemm(st, false, false, 1, static_cast<int>(nn), mh, 1.0, w.c.p, mh, 0, w.Fhist.p, nn, 0, 0.0, w.FP.p, nn, 0,
              1, nullptr);
        Fx = w.FP.p;
      }
    }
    if (opt.purify) {
      // FP32 purification steps while the commutator is far above their rounding
      sp2_density(st, n, o, Fx, m.P.p, w, n >= kSp2MixedMinN && err > kSp2MixedMaxErr);
    } else {
      copy(st, w.CT.p, Fx, nn);
      ds.eigh(n, w.CT.p, n, m.eps.p);
      density_from_CT(st, n, o, w.CT.p, m.P.p);
    }
  }
  m.commutator = err;
  m.scf_iterations = it;
  if (err > opt.tol) throw Error(kEScfNoConv, "SCF did not converge: max|FP-PF| = " + std::to_string(err));
  // final orbitals of the converged Fock matrix
  copy(st, w.CT.p, w.F.p, nn);
  ds.eigh(n, w.CT.p, n, m.eps.p);
  if (ds.info_eigh() != 0) throw Error(kEDevice, "dense eigensolver failed in SCF");
  transpose(st, n, n, w.CT.p, n, m.C.p, n);  // C[mu][p] = CT[p][mu]
  m.C32.ensure(nn);
  to_float(st, nn, m.C.p, m.C32.p);
  density_from_CT(st, n, o, w.CT.p, m.P.p);
}

}  // namespace seqx
