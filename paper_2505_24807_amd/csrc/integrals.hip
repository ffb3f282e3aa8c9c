// NDDO integral tables on the device: two-centre ERIs (point multipoles in the
// diatomic frame, rotated to the molecular frame), one-centre blocks, Slater
// overlaps in closed form, and the core Hamiltonian.
//
// Model (ground-state subsection of the paper; MNDO-family multipole scheme):
// each same-atom orbital product becomes point charges -- ss a unit monopole,
// s p_k a dipole of +-1/2 at +-D1 along k, p_k p_k a unit monopole plus a linear
// quadrupole (+1/4 at +-2 D2 along k, -1/2 at the centre), p_k p_l a square
// quadrupole (+-1/4 at D2 (+-e_k +-e_l)).  Charges q, q' interact as
// q q' / sqrt(d^2 + (rho + rho')^2) with the additive terms of their multipoles.
// (px py|px py) is set to ((px px|px px) - (px px|py py)) / 2 so that the set is
// invariant under rotation about the bond.
#include "integrals.hpp"

namespace seqx {

namespace {

struct Charges {
  int n;
  double q[4];
  double x[4], y[4], z[4];
  double rho[4];
};

__device__ inline void add_charge(Charges& c, double q, double x, double y, double z, double rho) {
  c.q[c.n] = q; c.x[c.n] = x; c.y[c.n] = y; c.z[c.n] = z; c.rho[c.n] = rho; ++c.n;
}

// point charges of the local-frame product of AOs i <= j (0=s, 1=x', 2=y', 3=z')
__device__ Charges local_charges(const Elem& e, int i, int j) {
  Charges c;
  c.n = 0;
  double ek[3] = {0, 0, 0}, el[3] = {0, 0, 0};
  if (i == 0 && j == 0) {
    add_charge(c, 1.0, 0, 0, 0, e.rho0);
  } else if (i == 0) {
    ek[j - 1] = e.D1;
    add_charge(c, 0.5, ek[0], ek[1], ek[2], e.rho1);
    add_charge(c, -0.5, -ek[0], -ek[1], -ek[2], e.rho1);
  } else if (i == j) {
    ek[i - 1] = 2.0 * e.D2;
    add_charge(c, 1.0, 0, 0, 0, e.rho0);
    add_charge(c, 0.25, ek[0], ek[1], ek[2], e.rho2);
    add_charge(c, 0.25, -ek[0], -ek[1], -ek[2], e.rho2);
    add_charge(c, -0.5, 0, 0, 0, e.rho2);
  } else {
    ek[i - 1] = e.D2;
    el[j - 1] = e.D2;
    add_charge(c, 0.25, ek[0] + el[0], ek[1] + el[1], ek[2] + el[2], e.rho2);
    add_charge(c, 0.25, -ek[0] - el[0], -ek[1] - el[1], -ek[2] - el[2], e.rho2);
    add_charge(c, -0.25, ek[0] - el[0], ek[1] - el[1], ek[2] - el[2], e.rho2);
    add_charge(c, -0.25, el[0] - ek[0], el[1] - ek[1], el[2] - ek[2], e.rho2);
  }
  return c;
}

// interaction of charge sets a (at the origin) and b (centred at (0, 0, R))
__device__ double charge_interaction(const Charges& a, const Charges& b, double R) {
  double s = 0.0;
  for (int k = 0; k < a.n; ++k)
    for (int l = 0; l < b.n; ++l) {
      const double dx = b.x[l] - a.x[k], dy = b.y[l] - a.y[k], dz = R + b.z[l] - a.z[k];
      const double rr = a.rho[k] + b.rho[l];
      s += a.q[k] * b.q[l] / sqrt(dx * dx + dy * dy + dz * dz + rr * rr);
    }
  return s;
}

// frame rows x', y', z' with z' along A->B; returns R
__device__ double local_frame(const double* xa, const double* xb, double f[3][3]) {
  double d[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
  const double R = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double z[3] = {d[0] / R, d[1] / R, d[2] / R};
  int k = 0;
  if (fabs(z[1]) < fabs(z[k])) k = 1;
  if (fabs(z[2]) < fabs(z[k])) k = 2;
  double x[3] = {0, 0, 0};
  x[k] = 1.0;
  const double dot = z[k];
  for (int c = 0; c < 3; ++c) x[c] -= dot * z[c];
  const double nx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  for (int c = 0; c < 3; ++c) x[c] /= nx;
  double y[3] = {z[1] * x[2] - z[2] * x[1], z[2] * x[0] - z[0] * x[2], z[0] * x[1] - z[1] * x[0]};
  for (int c = 0; c < 3; ++c) {
    f[0][c] = x[c];
    f[1][c] = y[c];
    f[2][c] = z[c];
  }
  return R;
}

// U[alpha][mu]: local AO alpha = sum_mu U[alpha][mu] molecular AO mu
__device__ inline double rot(const double f[3][3], int alpha, int mu) {
  if (alpha == 0 || mu == 0) return (alpha == 0 && mu == 0) ? 1.0 : 0.0;
  return f[alpha - 1][mu - 1];
}

// pair rotation: Ut[P][Pl] = U[a][m] U[b][n] + (a != b) U[b][m] U[a][n],
// P = (m <= n) molecular, Pl = (a <= b) local
template <int NP>
__device__ inline void pair_rotation(const double f[3][3], double Ut[NP][NP]) {
  for (int P = 0; P < NP; ++P) {
    const int m = NP == 1 ? 0 : pair_first(P), n = NP == 1 ? 0 : pair_second(P);
    for (int Q = 0; Q < NP; ++Q) {
      const int a = NP == 1 ? 0 : pair_first(Q), b = NP == 1 ? 0 : pair_second(Q);
      double v = rot(f, a, m) * rot(f, b, n);
      if (a != b) v += rot(f, b, m) * rot(f, a, n);
      Ut[P][Q] = v;
    }
  }
}

template <int NPA, int NPB>
__global__ void __launch_bounds__(128) two_centre_kernel(int npairs, const int2* __restrict__ pairs,
                                                         const int* __restrict__ slot, const double* __restrict__ xyz,
                                                         const int* __restrict__ pi_off, const Elem* __restrict__ elems,
                                                         double* __restrict__ W, int ldw) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int A = pairs[p].x, B = pairs[p].y;
  const Elem ea = elems[slot[A]], eb = elems[slot[B]];
  double f[3][3];
  const double R = local_frame(xyz + 3 * A, xyz + 3 * B, f);
  double L[NPA][NPB];
  for (int P = 0; P < NPA; ++P) {
    const Charges ca = local_charges(ea, NPA == 1 ? 0 : pair_first(P), NPA == 1 ? 0 : pair_second(P));
    for (int Q = 0; Q < NPB; ++Q) {
      const Charges cb = local_charges(eb, NPB == 1 ? 0 : pair_first(Q), NPB == 1 ? 0 : pair_second(Q));
      L[P][Q] = charge_interaction(ca, cb, R);
    }
  }
  if constexpr (NPA == 10 && NPB == 10) {
    // (x'y'|x'y') from the rotation-invariance relation
    L[5][5] = 0.5 * (L[4][4] - L[4][7]);
  }
  double UA[NPA][NPA], UB[NPB][NPB];
  pair_rotation<NPA>(f, UA);
  pair_rotation<NPB>(f, UB);
  // Wm = UA L UB^T
  double T[NPA][NPB];
  for (int P = 0; P < NPA; ++P)
    for (int Q = 0; Q < NPB; ++Q) {
      double s = 0;
      for (int k = 0; k < NPA; ++k) s += UA[P][k] * L[k][Q];
      T[P][Q] = s;
    }
  const int oa = pi_off[A], ob = pi_off[B];
  for (int P = 0; P < NPA; ++P)
    for (int Q = 0; Q < NPB; ++Q) {
      double s = 0;
      for (int k = 0; k < NPB; ++k) s += T[P][k] * UB[Q][k];
      W[static_cast<size_t>(oa + P) * ldw + ob + Q] = s;
      W[static_cast<size_t>(ob + Q) * ldw + oa + P] = s;
    }
}

// one-centre blocks of W: (mm|nn) = gss, gsp, gpp, gp2; (mn|mn) = hsp, hpp
__global__ void one_centre_kernel(int natoms, const int* __restrict__ slot, const int* __restrict__ pi_off,
                                  const Elem* __restrict__ elems, double* __restrict__ W, int ldw) {
  const int A = blockIdx.x;
  if (A >= natoms) return;
  const Elem e = elems[slot[A]];
  const int o = pi_off[A];
  const int np = e.nao == 4 ? 10 : 1;
  for (int t = threadIdx.x; t < np * np; t += blockDim.x) {
    const int P = t / np, Q = t % np;
    double v = 0.0;
    if (np == 1) {
      v = e.gss;
    } else {
      const int m = pair_first(P), n = pair_second(P), l = pair_first(Q), s = pair_second(Q);
      if (m == n && l == s) {
        if (m == 0 && l == 0) v = e.gss;
        else if (m == 0 || l == 0) v = e.gsp;
        else v = (m == l) ? e.gpp : e.gp2;
      } else if (m != n && P == Q) {
        v = (m == 0) ? e.hsp : e.hpp;
      }
    }
    W[static_cast<size_t>(o + P) * ldw + o + Q] = v;
  }
}

// ---------------------------------------------------------------- overlaps
// Closed forms in prolate spheroidal coordinates: with h = R/2, r_A = h(l+m),
// r_B = h(l-m), z_A = h(1+lm), z_B = h(lm-1), rho^2 = h^2 (l^2-1)(1-m^2),
// dV = h^3 (l^2 - m^2) dl dm dphi, every overlap is a polynomial in (l, m)
// times exp(-p l - t m) and integrates to sums of A_i(p) B_j(t).

struct Poly {  // c[i][j] multiplies l^i m^j
  double c[5][5];
};

__device__ inline void poly_zero(Poly& a) {
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) a.c[i][j] = 0.0;
}

__device__ inline Poly poly_mul(const Poly& a, const Poly& b) {
  Poly r;
  poly_zero(r);
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      if (a.c[i][j] == 0.0) continue;
      for (int k = 0; k + i < 5; ++k)
        for (int l = 0; l + j < 5; ++l) r.c[i + k][j + l] += a.c[i][j] * b.c[k][l];
    }
  return r;
}

__device__ void aux_A(double p, double* A) {  // A_k = int_1^inf x^k e^{-px} dx, k = 0..4
  const double e = exp(-p);
  A[0] = e / p;
  for (int k = 1; k < 5; ++k) A[k] = (k * A[k - 1] + e) / p;
}

__device__ void aux_B(double t, double* B) {  // B_k = int_{-1}^{1} y^k e^{-ty} dy, k = 0..4
  if (fabs(t) < 10.0) {
    for (int k = 0; k < 5; ++k) {
      double s = 0.0, term = 1.0;  // (-t)^m / m!
      for (int m = 0; m < 90; ++m) {
        if (((k + m) & 1) == 0) s += term * 2.0 / (k + m + 1);
        term *= -t / (m + 1);
        if (fabs(term) < 1e-18 * fabs(s) && m > k + 4) break;
      }
      B[k] = s;
    }
  } else {
    const double ep = exp(t), em = exp(-t);
    B[0] = (ep - em) / t;
    for (int k = 1; k < 5; ++k) B[k] = (((k & 1) ? -ep : ep) - em + k * B[k - 1]) / t;
  }
}

// polynomial of one orbital factor: kind 0 = s, 1 = p_sigma (z'); atom 0 = A, 1 = B
__device__ Poly orbital_poly(int n, int kind, int atom, double h) {
  Poly r;
  poly_zero(r);
  if (kind == 0) {
    if (n == 1) {
      r.c[0][0] = 1.0;
    } else {  // r_A = h(l + m), r_B = h(l - m)
      r.c[1][0] = h;
      r.c[0][1] = atom == 0 ? h : -h;
    }
  } else {  // z_A = h(1 + l m), z_B = h(l m - 1)
    r.c[1][1] = h;
    r.c[0][0] = atom == 0 ? h : -h;
  }
  return r;
}

__device__ inline double sto_norm(int n, double z) {
  const double fact2n = (n == 1) ? 2.0 : 24.0;
  return pow(2.0 * z, n + 0.5) / sqrt(fact2n);
}

// local overlap between AO a on A (0=s, 1=x', 2=y', 3=z') and AO b on B
__device__ double local_overlap(const Elem& ea, int a, const Elem& eb, int b, double R) {
  const bool pa = a > 0, pb = b > 0;
  const bool pia = (a == 1 || a == 2), pib = (b == 1 || b == 2);
  if (pia || pib) {
    if (!(pia && pib && a == b)) return 0.0;
  }
  const double h = 0.5 * R;
  const double za = pa ? ea.zp : ea.zs, zb = pb ? eb.zp : eb.zs;
  const double p = h * (za + zb), t = h * (za - zb);
  Poly jac;
  poly_zero(jac);
  jac.c[2][0] = 1.0;
  jac.c[0][2] = -1.0;
  Poly f;
  double ang, phi;
  if (pia) {  // (l^2 - 1)(1 - m^2) h^2 times the Jacobian
    Poly s2;
    poly_zero(s2);
    s2.c[2][0] = h * h;
    s2.c[0][0] = -h * h;
    s2.c[2][2] = -h * h;
    s2.c[0][2] = h * h;
    f = poly_mul(s2, jac);
    ang = 3.0 / (4.0 * M_PI);
    phi = M_PI;
  } else {
    f = poly_mul(poly_mul(orbital_poly(ea.n, a == 3 ? 1 : 0, 0, h), orbital_poly(eb.n, b == 3 ? 1 : 0, 1, h)), jac);
    ang = (a == 3 ? sqrt(3.0 / (4.0 * M_PI)) : 1.0 / sqrt(4.0 * M_PI)) *
          (b == 3 ? sqrt(3.0 / (4.0 * M_PI)) : 1.0 / sqrt(4.0 * M_PI));
    phi = 2.0 * M_PI;
  }
  double Av[5], Bv[5];
  aux_A(p, Av);
  aux_B(t, Bv);
  double s = 0.0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j)
      if (f.c[i][j] != 0.0) s += f.c[i][j] * Av[i] * Bv[j];
  return sto_norm(ea.n, za) * sto_norm(eb.n, zb) * ang * phi * h * h * h * s;
}

template <int NA, int NB>
__global__ void __launch_bounds__(128) resonance_kernel(int npairs, const int2* __restrict__ pairs,
                                                        const int* __restrict__ slot, const double* __restrict__ xyz,
                                                        const int* __restrict__ ao_off, const Elem* __restrict__ elems,
                                                        double* __restrict__ H, int ldh) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int A = pairs[p].x, B = pairs[p].y;
  const Elem ea = elems[slot[A]], eb = elems[slot[B]];
  double f[3][3];
  const double R = local_frame(xyz + 3 * A, xyz + 3 * B, f);
  double Sl[NA][NB];
  for (int a = 0; a < NA; ++a)
    for (int b = 0; b < NB; ++b) Sl[a][b] = local_overlap(ea, a, eb, b, R);
  const int oa = ao_off[A], ob = ao_off[B];
  for (int m = 0; m < NA; ++m)
    for (int n = 0; n < NB; ++n) {
      double s = 0.0;
      for (int a = 0; a < NA; ++a)
        for (int b = 0; b < NB; ++b) s += rot(f, a, m) * Sl[a][b] * rot(f, b, n);
      const double bm = m == 0 ? ea.bs : ea.bp, bn = n == 0 ? eb.bs : eb.bp;
      const double v = 0.5 * (bm + bn) * s;
      H[static_cast<size_t>(oa + m) * ldh + ob + n] = v;
      H[static_cast<size_t>(ob + n) * ldh + oa + m] = v;
    }
}

// atom-diagonal blocks of H: U on the diagonal minus sum_{B != A} Z'_B (mn|s_B s_B)
__global__ void core_diag_kernel(int natoms, const int* __restrict__ slot, const int* __restrict__ ao_off,
                                 const int* __restrict__ pi_off, const Elem* __restrict__ elems,
                                 const double* __restrict__ W, int ldw, double* __restrict__ H, int ldh) {
  const int A = blockIdx.x;
  const Elem e = elems[slot[A]];
  const int np = e.nao == 4 ? 10 : 1;
  __shared__ double part[10][64];
  const int P = threadIdx.x / 64, lane = threadIdx.x % 64;  // blockDim = 640
  double s = 0.0;
  if (P < np) {
    const double* row = W + static_cast<size_t>(pi_off[A] + P) * ldw;
    for (int B = lane; B < natoms; B += 64) {
      if (B == A) continue;
      s += elems[slot[B]].core * row[pi_off[B]];
    }
  }
  part[P][lane] = s;
  __syncthreads();
  if (threadIdx.x < np) {
    const int Pp = threadIdx.x;
    double v = 0.0;
    for (int l = 0; l < 64; ++l) v += part[Pp][l];  // fixed order: deterministic
    const int m = np == 1 ? 0 : pair_first(Pp), n = np == 1 ? 0 : pair_second(Pp);
    double h = -v;
    if (m == n) h += (m == 0) ? e.Uss : e.Upp;
    const int o = ao_off[A];
    H[static_cast<size_t>(o + m) * ldh + o + n] = h;
    H[static_cast<size_t>(o + n) * ldh + o + m] = h;
  }
}

}  // namespace

void build_integrals(const DeviceMolecule& m, const Elem* elems, double* W, double* H, hipStream_t st) {
  const int ldw = m.np;
  // two-centre blocks, one launch per pair type (heavy-heavy, heavy-H, H-H)
  if (m.npairs[0])
    hipLaunchKernelGGL((two_centre_kernel<10, 10>), dim3(ceil_div(m.npairs[0], 128)), dim3(128), 0, st, m.npairs[0],
                       m.pairs[0].p, m.slot.p, m.xyz.p, m.pi_off.p, elems, W, ldw);
  if (m.npairs[1])
    hipLaunchKernelGGL((two_centre_kernel<10, 1>), dim3(ceil_div(m.npairs[1], 128)), dim3(128), 0, st, m.npairs[1],
                       m.pairs[1].p, m.slot.p, m.xyz.p, m.pi_off.p, elems, W, ldw);
  if (m.npairs[2])
    hipLaunchKernelGGL((two_centre_kernel<1, 1>), dim3(ceil_div(m.npairs[2], 128)), dim3(128), 0, st, m.npairs[2],
                       m.pairs[2].p, m.slot.p, m.xyz.p, m.pi_off.p, elems, W, ldw);
  hipLaunchKernelGGL(one_centre_kernel, dim3(m.natoms), dim3(128), 0, st, m.natoms, m.slot.p, m.pi_off.p, elems,
                     W, ldw);
  SEQX_LAUNCH_CHECK();
  // core Hamiltonian: off-atom resonance blocks, then atom-diagonal blocks
  const int ldh = m.nao;
  if (m.npairs[0])
    hipLaunchKernelGGL((resonance_kernel<4, 4>), dim3(ceil_div(m.npairs[0], 128)), dim3(128), 0, st, m.npairs[0],
                       m.pairs[0].p, m.slot.p, m.xyz.p, m.ao_off.p, elems, H, ldh);
  if (m.npairs[1])
    hipLaunchKernelGGL((resonance_kernel<4, 1>), dim3(ceil_div(m.npairs[1], 128)), dim3(128), 0, st, m.npairs[1],
                       m.pairs[1].p, m.slot.p, m.xyz.p, m.ao_off.p, elems, H, ldh);
  if (m.npairs[2])
    hipLaunchKernelGGL((resonance_kernel<1, 1>), dim3(ceil_div(m.npairs[2], 128)), dim3(128), 0, st, m.npairs[2],
                       m.pairs[2].p, m.slot.p, m.xyz.p, m.ao_off.p, elems, H, ldh);
  hipLaunchKernelGGL(core_diag_kernel, dim3(m.natoms), dim3(640), 0, st, m.natoms, m.slot.p, m.ao_off.p, m.pi_off.p,
                     elems, W, ldw, H, ldh);
  SEQX_LAUNCH_CHECK();
}

void build_integrals(const DeviceMolecule& m, hipStream_t st) { build_integrals(m, m.elems, m.W.p, m.H.p, st); }

}  // namespace seqx
