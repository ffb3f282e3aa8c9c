// Element constants and molecule layout (host code).
#include "model.hpp"

#include <cmath>
#include <sstream>

namespace seqx {

int element_slot(int Z) {
  switch (Z) {
    case 1: return 0;
    case 6: return 1;
    case 8: return 2;
    default: return -1;
  }
}

namespace {

// Solve f(rho) = target for a function that falls strictly from +inf at
// rho -> 0 to 0 at rho -> inf, by bisection to full double precision.
template <class F>
double solve_falling(F f, double target) {
  double lo = 1e-10, hi = 1.0;
  while (f(hi) > target) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (f(mid) > target) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

Elem make_elem(int Z, const double* v) {
  // v: zeta_s, zeta_p, U_ss, U_pp, beta_s, beta_p, g_ss, g_sp, g_pp, g_p2, h_sp
  const double ev = 1.0 / kHartreeEV;
  Elem e;
  std::memset(&e, 0, sizeof(e));
  e.Z = Z;
  e.nao = (Z == 1) ? 1 : 4;
  e.n = (Z == 1) ? 1 : 2;
  e.core = (Z == 1) ? 1.0 : (Z == 6 ? 4.0 : 6.0);
  e.zs = v[0];
  e.Uss = v[2] * ev;
  e.bs = v[4] * ev;
  e.gss = v[6] * ev;
  e.rho0 = 0.5 / e.gss;  // monopole self-interaction at R = 0 equals gss
  if (e.nao == 4) {
    e.zp = v[1];
    e.Upp = v[3] * ev;
    e.bp = v[5] * ev;
    e.gsp = v[7] * ev;
    e.gpp = v[8] * ev;
    e.gp2 = v[9] * ev;
    e.hsp = v[10] * ev;
    e.hpp = 0.5 * (e.gpp - e.gp2);
    const double n = e.n, zs = e.zs, zp = e.zp;
    // <s|z|pz> for ns, np Slater functions, and D2 with D2^2 = <r^2>_p / 5
    e.D1 = (2 * n + 1) * std::pow(4 * zs * zp, n + 0.5) / (std::pow(zs + zp, 2 * n + 2) * std::sqrt(3.0));
    e.D2 = std::sqrt((4 * n * n + 6 * n + 2) / 20.0) / zp;
    const double D1 = e.D1, D2 = e.D2;
    // dipole self-interaction equals hsp; square-quadrupole self-interaction equals hpp
    e.rho1 = solve_falling([&](double r) { return 0.25 / r - 0.25 / std::sqrt(D1 * D1 + r * r); }, e.hsp);
    e.rho2 = solve_falling(
        [&](double r) {
          return 0.125 / r - 0.25 / std::sqrt(D2 * D2 + r * r) + 0.125 / std::sqrt(2 * D2 * D2 + r * r);
        },
        e.hpp);
  }
  return e;
}

void validate_molecules(int nmol, const int32_t* natoms, const int32_t* Z, const double* xyz) {
  if (nmol <= 0 || !natoms || !Z || !xyz) throw Error(kEArg, "nmol must be > 0 and arrays non-null");
  size_t off = 0;
  for (int m = 0; m < nmol; ++m) {
    const int na = natoms[m];
    if (na <= 0) {
      std::ostringstream os;
      os << "molecule " << m << ": natoms must be > 0";
      throw Error(kEArg, os.str());
    }
    long nel = 0;
    for (int a = 0; a < na; ++a) {
      const int z = Z[off + a];
      if (element_slot(z) < 0) {
        std::ostringstream os;
        os << "molecule " << m << " atom " << a << ": unsupported element Z=" << z;
        throw Error(kEElement, os.str());
      }
      nel += (z == 1) ? 1 : (z == 6 ? 4 : 6);
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(xyz[3 * (off + a) + c])) {
          std::ostringstream os;
          os << "molecule " << m << " atom " << a << ": non-finite coordinate";
          throw Error(kEGeometry, os.str());
        }
    }
    if (nel % 2) {
      std::ostringstream os;
      os << "molecule " << m << ": odd electron count " << nel << " (closed shell required)";
      throw Error(kEOpenShell, os.str());
    }
    long nao = 0;
    for (int a = 0; a < na; ++a) nao += (Z[off + a] == 1) ? 1 : 4;
    if (nel / 2 >= nao) {
      std::ostringstream os;
      os << "molecule " << m << ": no virtual orbitals";
      throw Error(kEArg, os.str());
    }
    for (int a = 0; a < na; ++a)
      for (int b = a + 1; b < na; ++b) {
        double d2 = 0;
        for (int c = 0; c < 3; ++c) {
          const double d = xyz[3 * (off + a) + c] - xyz[3 * (off + b) + c];
          d2 += d * d;
        }
        if (d2 < 0.01) {
          std::ostringstream os;
          os << "molecule " << m << ": atoms " << a << " and " << b << " closer than 0.1 Angstrom";
          throw Error(kEGeometry, os.str());
        }
      }
    off += na;
  }
}

Layout make_layout(int natoms, const int32_t* Z, const double* xyz, const Elem* elems) {
  Layout L;
  L.natoms = natoms;
  for (int a = 0; a < natoms; ++a)
    if (Z[a] != 1) L.perm.push_back(a);
  L.nheavy = static_cast<int>(L.perm.size());
  for (int a = 0; a < natoms; ++a)
    if (Z[a] == 1) L.perm.push_back(a);
  L.slot.resize(natoms);
  L.ao_off.assign(natoms + 1, 0);
  L.pi_off.assign(natoms + 1, 0);
  L.xyz.resize(3 * natoms);
  long nel = 0;
  for (int k = 0; k < natoms; ++k) {
    const int a = L.perm[k];
    L.slot[k] = element_slot(Z[a]);
    const Elem& e = elems[L.slot[k]];
    L.ao_off[k + 1] = L.ao_off[k] + e.nao;
    L.pi_off[k + 1] = L.pi_off[k] + (e.nao == 4 ? 10 : 1);
    for (int c = 0; c < 3; ++c) L.xyz[3 * k + c] = xyz[3 * a + c] / kBohrAng;
    nel += static_cast<long>(e.core);
  }
  L.nao = L.ao_off[natoms];
  L.np = L.pi_off[natoms];
  L.nocc = static_cast<int>(nel / 2);
  L.nvirt = L.nao - L.nocc;
  // input-order offsets
  std::vector<int> ao_in(natoms + 1, 0), pi_in(natoms + 1, 0);
  for (int a = 0; a < natoms; ++a) {
    ao_in[a + 1] = ao_in[a] + (Z[a] == 1 ? 1 : 4);
    pi_in[a + 1] = pi_in[a] + (Z[a] == 1 ? 1 : 10);
  }
  L.ao_user.resize(L.nao);
  L.pi_user.resize(L.np);
  for (int k = 0; k < natoms; ++k) {
    const int a = L.perm[k];
    for (int i = 0; i < L.ao_off[k + 1] - L.ao_off[k]; ++i) L.ao_user[L.ao_off[k] + i] = ao_in[a] + i;
    for (int i = 0; i < L.pi_off[k + 1] - L.pi_off[k]; ++i) L.pi_user[L.pi_off[k] + i] = pi_in[a] + i;
  }
  return L;
}

}  // namespace seqx
