// Derivatives of the excitation energies with respect to the NDDO parameters:
// the paper's machine-learning interface re-optimises the semiempirical
// parameters by gradient descent and extends this to excited states
// (overview and conclusion).
//
// With T = X + Y and U = X - Y of one root (CIS: T = U = X), carried to the
// AO basis and split into the symmetric part Ts of T and the antisymmetric
// part Ua of U, the excitation energy is
//   omega = tr(D F) + <Ts, 2 J(Ts) - K(Ts)> - <Ua, K(Ua)>,
//   D = (Cv (T^T T + U^T U) Cv^T - Co (T T^T + U U^T) Co^T) / 2,
// stationary in the amplitudes.  Its dependence on the orbitals enters through
// one linear system with the SCF Hessian, (A+B) Z = -L (orbital response,
// Z-vector), with the orbital gradient
//   L = 4 Co^T G(D) Cv + 2 (T Qt_vv - Qt_oo T + U Qu_vv - Qu_oo U),
//   G(D) = J(D) - K(D)/2, Qt = 2 J(Ts) - K(Ts), Qu = K(Ua), Q_xy = Cx^T Q Cy.
// Then, with Drel = D + sym(Co Z Cv^T) and the ground-state density P,
//   d omega / d theta = sum Drel dH/dtheta + sum (mn|ls)' Gamma_mnls,
//   Gamma = Drel_mn P_ls - Drel_ml P_ns / 2 + 2 Ts_mn Ts_ls - Ts_ml Ts_ns - Ua_ml Ua_ns.
// The orbital basis is orthonormal whatever the parameters (S = I in the
// secular equation), so there is no overlap-derivative term.  The derivative
// tables dH/dtheta and d(mn|ls)/dtheta come from central differences of the
// library's own integral builder at theta +- h (h = 1e-5 |theta|): the
// integrals are cheap next to a solve and smooth in every parameter; the
// response above is analytic.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gemm.hpp"
#include "gradient.hpp"
#include "integrals.hpp"
#include "model.hpp"

namespace seqx {

namespace {

__global__ void pair_rows_kernel(long nov, const double* __restrict__ X, const double* __restrict__ Y,
                                 double* __restrict__ T, double* __restrict__ U) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  const long b = static_cast<long>(blockIdx.y) * nov + x;
  if (x >= nov) return;
  T[b] = X[b] + Y[b];
  U[b] = X[b] - Y[b];
}

// in place: A <- (A + A^T)/2 (sign +1) or (A - A^T)/2 (sign -1), k matrices n x n
__global__ void sym_part_kernel(int n, double* __restrict__ A, double sign) {
  const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n || j < i) return;
  double* M = A + static_cast<long>(blockIdx.z) * n * n;
  const double a = M[static_cast<long>(i) * n + j], b = M[static_cast<long>(j) * n + i];
  M[static_cast<long>(i) * n + j] = 0.5 * (a + sign * b);
  M[static_cast<long>(j) * n + i] = 0.5 * (b + sign * a);
}

// Drel = D + (Z + Z^T)/2, k matrices n x n
__global__ void add_sym_kernel(int n, const double* __restrict__ Z, double* __restrict__ D) {
  const long base = static_cast<long>(blockIdx.z) * n * n;
  const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n) return;
  D[base + static_cast<long>(i) * n + j] +=
      0.5 * (Z[base + static_cast<long>(i) * n + j] + Z[base + static_cast<long>(j) * n + i]);
}

// Gamma[k][P][Q] summed over the orderings of the AO pairs P = (m n), Q = (l s)
__global__ void __launch_bounds__(256) gamma_kernel(int np, int n, const int* __restrict__ pi_mu,
                                                    const int* __restrict__ pi_nu, const double* __restrict__ Dr,
                                                    const double* __restrict__ Pd, const double* __restrict__ Ts,
                                                    const double* __restrict__ Ua, double* __restrict__ G) {
  const int Q = blockIdx.x * 256 + threadIdx.x;
  const int P = blockIdx.y;
  if (Q >= np) return;
  const long nn = static_cast<long>(n) * n;
  const double* dr = Dr + blockIdx.z * nn;
  const double* ts = Ts + blockIdx.z * nn;
  const double* ua = Ua + blockIdx.z * nn;
  const int a = pi_mu[P], b = pi_nu[P], c = pi_mu[Q], d = pi_nu[Q];
  const int np_ = a == b ? 1 : 2, nq = c == d ? 1 : 2;
  double g = 0.0;
  for (int x = 0; x < np_; ++x) {
    const long m = x ? b : a, nu = x ? a : b;
    for (int y = 0; y < nq; ++y) {
      const long l = y ? d : c, s = y ? c : d;
      g += dr[m * n + nu] * Pd[l * n + s] - 0.5 * dr[m * n + l] * Pd[nu * n + s] +
           2.0 * ts[m * n + nu] * ts[l * n + s] - ts[m * n + l] * ts[nu * n + s] - ua[m * n + l] * ua[nu * n + s];
    }
  }
  G[blockIdx.z * static_cast<long>(np) * np + static_cast<long>(P) * np + Q] = g;
}

// preconditioner of the response: z = r / (eps_a - eps_i), k rows
__global__ void precond_rows_kernel(long nov, int v, int o, const double* __restrict__ eps,
                                    const double* __restrict__ r, double* __restrict__ z) {
  const long x = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (x >= nov) return;
  const long b = static_cast<long>(blockIdx.y) * nov + x;
  const int i = static_cast<int>(x / v), a = static_cast<int>(x % v);
  z[b] = r[b] / (eps[o + a] - eps[i]);
}

// x += alpha_j p, r -= alpha_j q for row j
__global__ void cg_step_kernel(long nov, const double* __restrict__ alpha, const double* __restrict__ p,
                               const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r) {
  const long t = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (t >= nov) return;
  const long b = static_cast<long>(blockIdx.y) * nov + t;
  const double a = alpha[blockIdx.y];
  x[b] += a * p[b];
  r[b] -= a * q[b];
}

// p = z + beta_j p for row j
__global__ void cg_dir_kernel(long nov, const double* __restrict__ beta, const double* __restrict__ z,
                              double* __restrict__ p) {
  const long t = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (t >= nov) return;
  const long b = static_cast<long>(blockIdx.y) * nov + t;
  p[b] = z[b] + beta[blockIdx.y] * p[b];
}

// diagonal of the k x k inner products of the rows of X and Y, to the host
std::vector<double> row_dots(hipStream_t st, int k, const double* X, const double* Y, long len, double* kk,
                             double* ws) {
  dots(st, k, X, len, k, Y, len, len, kk, k, ws);
  std::vector<double> h(static_cast<size_t>(k) * k), out(k);
  SEQX_HIP(hipMemcpyAsync(h.data(), kk, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SEQX_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < k; ++j) out[j] = h[static_cast<size_t>(j) * k + j];
  return out;
}

}  // namespace

GradientResult param_gradient(DeviceMolecule& m, int theory, const Elem* elems_host,
                              const double (*raw)[kNumElemParams], SigmaWork& sig, GWork& gw, hipStream_t st,
                              double* grad) {
  (void)theory;  // CIS amplitudes have Y = 0, so T = U = X and the same expressions apply
  const int K = m.nroots, n = m.nao, o = m.nocc, v = m.nvirt, np = m.np;
  const long nov = static_cast<long>(o) * v, nn = static_cast<long>(n) * n, npp = static_cast<long>(np) * np;
  const long nv = static_cast<long>(n) * v, no = static_cast<long>(n) * o;
  if (K < 1) throw Error(kEState, "no roots: call seqx_solve first");
  GradientResult res;
  std::fill(grad, grad + static_cast<size_t>(K) * kNumSlots * kNumElemParams, 0.0);
  const double* C = m.C.p;
  const double* Cv = m.C.p + o;
  // roots per group: the AO matrices and Gamma of a group stay below about 4 GB
  const double per_root = 8.0 * (10.0 * nn + npp + 8.0 * nov + 2.0 * nv + no + v * static_cast<double>(v) +
                                 o * static_cast<double>(o));
  const int kg_max = static_cast<int>(std::max(1.0, std::min<double>(16.0, 4e9 / per_root)));
  // parameter perturbations: which (slot, parameter) pairs apply
  std::vector<int> present(kNumSlots, 0);
  for (int s : m.L.slot) present[s] = 1;
  DBuf<Elem> dtab(2 * kNumSlots);
  DBuf<double> Wp(2 * npp), Hp(2 * nn);  // tables at theta + h and theta - h
  for (int k0 = 0; k0 < K; k0 += kg_max) {
    const int kg = std::min(kg_max, K - k0);
    DBuf<double> T(kg * nov), U(kg * nov), L(kg * nov), Z(kg * nov), R(kg * nov), Pz(kg * nov), Q(kg * nov),
        Q2(kg * nov), Zr(kg * nov);
    DBuf<double> Tao(kg * nn), Uao(kg * nn), Dm(kg * nn), GD(kg * nn), Qt(kg * nn), Qu(kg * nn), Fj(kg * nn);
    DBuf<double> Mvv(static_cast<size_t>(kg) * v * v), Moo(static_cast<size_t>(kg) * o * o), Tnv(kg * nv),
        Tno(kg * no);
    DBuf<double> kk(static_cast<size_t>(kg) * kg), coef(2 * kg), ws;
    ws.alloc(std::max<size_t>(std::max(dots_workspace(kg, kg, nov), dots_workspace(kg, 1, std::max(npp, nn))), 1024));
    const double* X = m.X.p + k0 * nov;
    const double* Y = m.Y.p + k0 * nov;
    const dim3 rows(ceil_div(nov, 256), kg);
    hipLaunchKernelGGL(pair_rows_kernel, rows, dim3(256), 0, st, nov, X, Y, T.p, U.p);
    SEQX_LAUNCH_CHECK();
    // D = (Cv (T^T T + U^T U) Cv^T - Co (T T^T + U U^T) Co^T) / 2
    dgemm(st, true, false, v, v, o, 1.0, T.p, v, nov, T.p, v, nov, 0.0, Mvv.p, v, static_cast<long>(v) * v, kg);
    dgemm(st, true, false, v, v, o, 1.0, U.p, v, nov, U.p, v, nov, 1.0, Mvv.p, v, static_cast<long>(v) * v, kg);
    dgemm(st, false, true, o, o, v, 1.0, T.p, v, nov, T.p, v, nov, 0.0, Moo.p, o, static_cast<long>(o) * o, kg);
    dgemm(st, false, true, o, o, v, 1.0, U.p, v, nov, U.p, v, nov, 1.0, Moo.p, o, static_cast<long>(o) * o, kg);
    dgemm(st, false, false, n, v, v, 1.0, Cv, n, 0, Mvv.p, v, static_cast<long>(v) * v, 0.0, Tnv.p, v, nv, kg);
    dgemm(st, false, true, n, n, v, 0.5, Tnv.p, v, nv, Cv, n, 0, 0.0, Dm.p, n, nn, kg);
    dgemm(st, false, false, n, o, o, 1.0, C, n, 0, Moo.p, o, static_cast<long>(o) * o, 0.0, Tno.p, o, no, kg);
    dgemm(st, false, true, n, n, o, -0.5, Tno.p, o, no, C, n, 0, 1.0, Dm.p, n, nn, kg);
    // AO amplitudes and their symmetric / antisymmetric parts
    forward_transform(m, kg, T.p, Tao.p, sig, st);
    forward_transform(m, kg, U.p, Uao.p, sig, st);
    const dim3 sq(ceil_div(n, 16), ceil_div(n, 16), kg);
    hipLaunchKernelGGL(sym_part_kernel, sq, dim3(16, 16), 0, st, n, Tao.p, 1.0);
    hipLaunchKernelGGL(sym_part_kernel, sq, dim3(16, 16), 0, st, n, Uao.p, -1.0);
    SEQX_LAUNCH_CHECK();
    double* Ts = Tao.p;
    double* Ua = Uao.p;
    // G(D), Qt = 2 J(Ts) - K(Ts), Qu = K(Ua)
    build_G(m, kg, Dm.p, nn, GD.p, static_cast<double*>(nullptr), nn, kSymm, 1.0, -0.5, 0.0, gw, st);
    build_G(m, kg, Ts, nn, Qt.p, static_cast<double*>(nullptr), nn, kSymm, 2.0, -1.0, 0.0, gw, st);
    build_G(m, kg, Ua, nn, Fj.p, Qu.p, nn, kTwo, 0.0, 0.0, 1.0, gw, st);
    // L = 4 Co^T G(D) Cv + 2 (T Qt_vv - Qt_oo T + U Qu_vv - Qu_oo U)
    dgemm(st, false, false, n, v, n, 1.0, GD.p, n, nn, Cv, n, 0, 0.0, Tnv.p, v, nv, kg);
    dgemm(st, true, false, o, v, n, 4.0, C, n, 0, Tnv.p, v, nv, 0.0, L.p, v, nov, kg);
    for (int w = 0; w < 2; ++w) {
      const double* Qm = w ? Qu.p : Qt.p;
      const double* A = w ? U.p : T.p;
      dgemm(st, false, false, n, v, n, 1.0, Qm, n, nn, Cv, n, 0, 0.0, Tnv.p, v, nv, kg);
      dgemm(st, true, false, v, v, n, 1.0, Cv, n, 0, Tnv.p, v, nv, 0.0, Mvv.p, v, static_cast<long>(v) * v, kg);
      dgemm(st, false, false, o, v, v, 2.0, A, v, nov, Mvv.p, v, static_cast<long>(v) * v, 1.0, L.p, v, nov, kg);
      dgemm(st, false, false, n, o, n, 1.0, Qm, n, nn, C, n, 0, 0.0, Tno.p, o, no, kg);
      dgemm(st, true, false, o, o, n, 1.0, C, n, 0, Tno.p, o, no, 0.0, Moo.p, o, static_cast<long>(o) * o, kg);
      dgemm(st, false, false, o, v, o, -2.0, Moo.p, o, static_cast<long>(o) * o, A, v, nov, 1.0, L.p, v, nov, kg);
    }
    // orbital response: (A+B) Z = -L by conjugate gradients, preconditioned with the gaps
    fill(st, Z.p, kg * nov, 0.0);
    copy(st, R.p, L.p, kg * nov);
    axpby(st, kg * nov, 0.0, L.p, -1.0, R.p);  // R = -L
    const std::vector<double> bnorm2 = row_dots(st, kg, R.p, R.p, nov, kk.p, ws.p);
    hipLaunchKernelGGL(precond_rows_kernel, rows, dim3(256), 0, st, nov, v, o, m.eps.p, R.p, Zr.p);
    copy(st, Pz.p, Zr.p, kg * nov);
    std::vector<double> rz = row_dots(st, kg, R.p, Zr.p, nov, kk.p, ws.p);
    std::vector<double> hc(kg);
    const double rtol = 1e-11;
    int it = 0;
    double worst = 0.0;
    for (it = 1; it <= 300; ++it) {
      sigma_build(m, 1, kg, Pz.p, Q.p, Q2.p, sig, st);  // Q = (A+B) P
      const std::vector<double> pq = row_dots(st, kg, Pz.p, Q.p, nov, kk.p, ws.p);
      for (int j = 0; j < kg; ++j) hc[j] = pq[j] > 0.0 ? rz[j] / pq[j] : 0.0;
      SEQX_HIP(hipMemcpyAsync(coef.p, hc.data(), kg * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(cg_step_kernel, rows, dim3(256), 0, st, nov, coef.p, Pz.p, Q.p, Z.p, R.p);
      const std::vector<double> rr = row_dots(st, kg, R.p, R.p, nov, kk.p, ws.p);
      worst = 0.0;
      for (int j = 0; j < kg; ++j)
        worst = std::max(worst, bnorm2[j] > 0.0 ? std::sqrt(rr[j] / bnorm2[j]) : 0.0);
      if (!std::isfinite(worst)) throw Error(kEUnstable, "orbital response diverged (A+B not positive definite)");
      if (worst <= rtol) break;
      hipLaunchKernelGGL(precond_rows_kernel, rows, dim3(256), 0, st, nov, v, o, m.eps.p, R.p, Zr.p);
      const std::vector<double> rz2 = row_dots(st, kg, R.p, Zr.p, nov, kk.p, ws.p);
      for (int j = 0; j < kg; ++j) {
        hc[j] = rz[j] > 0.0 ? rz2[j] / rz[j] : 0.0;
        rz[j] = rz2[j];
      }
      SEQX_HIP(hipMemcpyAsync(coef.p + kg, hc.data(), kg * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(cg_dir_kernel, rows, dim3(256), 0, st, nov, coef.p + kg, Zr.p, Pz.p);
      SEQX_LAUNCH_CHECK();
    }
    if (worst > 1e-8) throw Error(kEDavNoConv, "orbital response did not converge");
    res.zvector_iterations = std::max(res.zvector_iterations, std::min(it, 300));
    res.zvector_residual = std::max(res.zvector_residual, worst);
    // Drel = D + sym(Co Z Cv^T)
    forward_transform(m, kg, Z.p, Fj.p, sig, st);
    hipLaunchKernelGGL(add_sym_kernel, sq, dim3(16, 16), 0, st, n, Fj.p, Dm.p);
    SEQX_LAUNCH_CHECK();
    // Gamma of every root of the group (reuses GD, Qt, Qu storage only if large enough: own buffer)
    DBuf<double> Gam(static_cast<size_t>(kg) * npp);
    hipLaunchKernelGGL(gamma_kernel, dim3(ceil_div(np, 256), np, kg), dim3(256), 0, st, np, n, m.pi_mu.p,
                       m.pi_nu.p, Dm.p, m.P.p, Ts, Ua, Gam.p);
    SEQX_LAUNCH_CHECK();
    // derivative tables by central differences of the integral builder, contracted per parameter
    std::vector<double> hg(kg), hh(kg);
    for (int s = 0; s < kNumSlots; ++s) {
      if (!present[s]) continue;
      const int Zs = elems_host[s].Z;
      for (int p = 0; p < kNumElemParams; ++p) {
        if (Zs == 1 && !(p == 0 || p == 2 || p == 4 || p == 6)) continue;  // H: zeta_s, U_ss, beta_s, g_ss
        const double h = 1e-5 * std::max(std::fabs(raw[s][p]), 1e-2);
        Elem tab[2 * kNumSlots];
        for (int sg = 0; sg < 2; ++sg) {
          double rv[kNumElemParams];
          for (int q = 0; q < kNumElemParams; ++q) rv[q] = raw[s][q];
          rv[p] += sg == 0 ? h : -h;
          for (int t = 0; t < kNumSlots; ++t) tab[sg * kNumSlots + t] = elems_host[t];
          tab[sg * kNumSlots + s] = make_elem(Zs, rv);
        }
        SEQX_HIP(hipMemcpyAsync(dtab.p, tab, sizeof(tab), hipMemcpyHostToDevice, st));
        build_integrals(m, dtab.p, Wp.p, Hp.p, st);
        build_integrals(m, dtab.p + kNumSlots, Wp.p + npp, Hp.p + nn, st);
        axpby(st, npp, -1.0, Wp.p + npp, 1.0, Wp.p);  // W+ - W-
        axpby(st, nn, -1.0, Hp.p + nn, 1.0, Hp.p);
        dots(st, kg, Gam.p, npp, 1, Wp.p, npp, npp, kk.p, 1, ws.p);
        dots(st, kg, Dm.p, nn, 1, Hp.p, nn, nn, kk.p + kg, 1, ws.p);
        SEQX_HIP(hipMemcpyAsync(hg.data(), kk.p, kg * sizeof(double), hipMemcpyDeviceToHost, st));
        SEQX_HIP(hipMemcpyAsync(hh.data(), kk.p + kg, kg * sizeof(double), hipMemcpyDeviceToHost, st));
        SEQX_HIP(hipStreamSynchronize(st));  // also keeps `tab` alive until its copy is done
        for (int j = 0; j < kg; ++j)
          grad[(static_cast<size_t>(k0 + j) * kNumSlots + s) * kNumElemParams + p] =
              kHartreeEV * (hg[j] + hh[j]) / (2.0 * h);
      }
    }
  }
  return res;
}

}  // namespace seqx
