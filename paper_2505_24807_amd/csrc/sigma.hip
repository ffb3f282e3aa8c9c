// Matrix-free products of Eqs. 8-9 (paper, GPU-implementation subsection).
//
//   R_I   = C_o V_I C_v^T                     two MFMA GEMMs (n x o x v, n x v x n)
//   F_I   = G(R_I)                            NDDO contraction (fock.hip)
//   out_I = C_o^T F_I C_v + de o V_I          two MFMA GEMMs, de added in the epilogue
// Singlet CIS:  F = 2 J(R) - K(R).  TDHF:  (A+B) <-> 4 J(S) - 2 K(S) and
// (A-B) <-> -2 K(D) with S, D the symmetric / antisymmetric parts of R: A V
// pairs with K(R) and B V with K(R^T), which gives exactly these combinations.
#include "gemm.hpp"
#include "linalg.hpp"
#include "sigma.hpp"

namespace seqx {

void PhaseTimer::reset() {
  resolve();
  for (int p = 0; p < kNumPhases; ++p) {
    ms[p] = flops[p] = bytes[p] = 0.0;
    launches[p] = 0;
  }
}

void PhaseTimer::resolve() {
  for (size_t c = 0; c < pending.size(); ++c) {
    auto& ev = pending[c];
    SEQX_HIP(hipEventSynchronize(ev[kNumPhases]));
    for (int p = 0; p < kNumPhases; ++p) {
      float t = 0.f;
      SEQX_HIP(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
      ms[p] += t;
      flops[p] += pending_flops[c][p];
      bytes[p] += pending_bytes[c][p];
      launches[p] += pending_launches[c][p];
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  pending.clear();
  pending_flops.clear();
  pending_bytes.clear();
  pending_launches.clear();
}

PhaseTimer::~PhaseTimer() {
  for (auto& ev : pending)
    for (auto& e : ev) (void)hipEventDestroy(e);
}

void forward_transform(const DeviceMolecule& m, int k, const double* X, double* T, SigmaWork& w, hipStream_t st) {
  const int n = m.nao, o = m.nocc, v = m.nvirt;
  w.T1.ensure(static_cast<size_t>(k) * n * v);
  // T1_I (n x v) = C[:, :o] (n x o, ld n) * X_I (o x v)
  dgemm(st, false, false, n, v, o, 1.0, m.C.p, n, 0, X, v, static_cast<long>(o) * v, 0.0, w.T1.p, v,
        static_cast<long>(n) * v, k);
  // T_I (n x n) = T1_I * C[:, o:]^T, one GEMM over the stacked T1_I
  dgemm(st, false, true, k * n, n, v, 1.0, w.T1.p, v, 0, m.C.p + o, n, 0, 0.0, T, n, 0, 1);
}

void sigma_build(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                 SigmaWork& w, hipStream_t st, int chunk, long out_stride, int precision) {
  const int n = m.nao, o = m.nocc, v = m.nvirt;
  const long nn = static_cast<long>(n) * n, nv = static_cast<long>(n) * v, ov = static_cast<long>(o) * v;
  const long os = out_stride > 0 ? out_stride : ov;
  const bool tdhf = theory == 1;
  const bool f32 = precision == kPrecFP32;
  if (precision != kPrecFP64 && precision != kPrecFP32) throw Error(kEArg, "unsupported transform precision");
  if (f32 && m.C32.n < static_cast<size_t>(nn)) throw Error(kEState, "FP32 MO coefficients missing");
  for (int c0 = 0; c0 < k; c0 += chunk) {
    const int kc = std::min(chunk, k - c0);
    const int nb = tdhf ? 2 * kc : kc;
    const double* Vc = V + c0 * ov;
    if (f32) {
      w.V32.ensure(static_cast<size_t>(kc) * ov);
      w.Rs.ensure(static_cast<size_t>(kc) * nn);
      w.Fs.ensure(static_cast<size_t>(nb) * nn);
      w.Zs.ensure(static_cast<size_t>(nb) * nv);
      w.T1s.ensure(static_cast<size_t>(kc) * nv);
    } else {
      w.R.ensure(static_cast<size_t>(kc) * nn);
      w.F.ensure(static_cast<size_t>(nb) * nn);
      w.Z.ensure(static_cast<size_t>(nb) * nv);
      w.T1.ensure(static_cast<size_t>(kc) * nv);
    }
    std::array<hipEvent_t, kNumPhases + 1> ev;
    for (auto& e : ev) SEQX_HIP(hipEventCreate(&e));
    SEQX_HIP(hipEventRecord(ev[0], st));
    SigmaEpilogue ep;
    ep.eps = m.eps.p;
    ep.nocc = o;
    ep.V = Vc;
    ep.strideV = ov;
    ep.kv = kc;
    // Outputs interleaved by vector ((A+B)V_I and (A-B)V_I half a row stride
    // apart, as the Davidson basis keeps them): F+ and F- are built
    // interleaved too, so the last product is one launch over all 2 kc
    // matrices (twice the workgroups of a launch per half).
    const bool merged = tdhf && os % 2 == 0 && out2 == out1 + os / 2;
    const long sF = merged ? 2 * nn : nn;
    const long f2off = merged ? nn : kc * nn;
    if (merged) ep.vdiv = 2;
    if (!f32) {
      // T1_I (n x v) = C[:, :o] V_I
      dgemm(st, false, false, n, v, o, 1.0, m.C.p, n, 0, Vc, v, ov, 0.0, w.T1.p, v, nv, kc);
      SEQX_HIP(hipEventRecord(ev[1], st));
      // R_I (n x n) = T1_I C[:, o:]^T: the T1_I are stacked rows, so one GEMM with M = kc n
      dgemm(st, false, true, kc * n, n, v, 1.0, w.T1.p, v, 0, m.C.p + o, n, 0, 0.0, w.R.p, n, 0, 1);
      SEQX_HIP(hipEventRecord(ev[2], st));
      if (tdhf)
        build_G(m, kc, w.R.p, nn, w.F.p, w.F.p + f2off, sF, kTwo, 4.0, -2.0, -2.0, w.g, st);
      else
        build_G(m, kc, w.R.p, nn, w.F.p, static_cast<double*>(nullptr), nn, kSum, 2.0, -1.0, -1.0, w.g, st);
      SEQX_HIP(hipEventRecord(ev[3], st));
      // Z_b (n x v) = F_b (n x n) * C[:, o:], all nb at once (M = nb n)
      dgemm(st, false, false, nb * n, v, n, 1.0, w.F.p, n, 0, m.C.p + o, n, 0, 0.0, w.Z.p, v, 0, 1);
      SEQX_HIP(hipEventRecord(ev[4], st));
      // out_b (o x v) = C[:, :o]^T * Z_b + de o V_b
      if (merged) {
        dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, w.Z.p, v, nv, 0.0, out1 + c0 * os, v, os / 2, nb, &ep);
      } else {
        dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, w.Z.p, v, nv, 0.0, out1 + c0 * os, v, os, kc, &ep);
        if (tdhf)
          dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, w.Z.p + kc * nv, v, nv, 0.0, out2 + c0 * os, v, os, kc,
                &ep);
      }
    } else {
      const float* C32 = m.C32.p;
      to_float(st, kc * ov, Vc, w.V32.p);
      sgemm(st, false, false, n, v, o, 1.0, C32, n, 0, w.V32.p, v, ov, 0.0, w.T1s.p, v, nv, kc);
      SEQX_HIP(hipEventRecord(ev[1], st));
      sgemm(st, false, true, kc * n, n, v, 1.0, w.T1s.p, v, 0, C32 + o, n, 0, 0.0, w.Rs.p, n, 0, 1);
      SEQX_HIP(hipEventRecord(ev[2], st));
      if (tdhf)
        build_G(m, kc, w.Rs.p, nn, w.Fs.p, w.Fs.p + f2off, sF, kTwo, 4.0, -2.0, -2.0, w.g, st);
      else
        build_G(m, kc, w.Rs.p, nn, w.Fs.p, static_cast<float*>(nullptr), nn, kSum, 2.0, -1.0, -1.0, w.g, st);
      SEQX_HIP(hipEventRecord(ev[3], st));
      sgemm(st, false, false, nb * n, v, n, 1.0, w.Fs.p, n, 0, C32 + o, n, 0, 0.0, w.Zs.p, v, 0, 1);
      SEQX_HIP(hipEventRecord(ev[4], st));
      if (merged) {
        sgemm_out64(st, true, false, o, v, n, 1.0, C32, n, 0, w.Zs.p, v, nv, 0.0, out1 + c0 * os, v, os / 2, nb, &ep);
      } else {
        sgemm_out64(st, true, false, o, v, n, 1.0, C32, n, 0, w.Zs.p, v, nv, 0.0, out1 + c0 * os, v, os, kc, &ep);
        if (tdhf)
          sgemm_out64(st, true, false, o, v, n, 1.0, C32, n, 0, w.Zs.p + kc * nv, v, nv, 0.0, out2 + c0 * os, v,
                      os, kc, &ep);
      }
    }
    SEQX_HIP(hipEventRecord(ev[5], st));
    // algorithmic work of this chunk; d = bytes per stored element of the transforms
    const double d = f32 ? 4.0 : 8.0;
    std::array<double, kNumPhases> fl{}, by{};
    std::array<long, kNumPhases> la{};
    fl[kPhaseFwd1] = 2.0 * n * o * v * kc;
    by[kPhaseFwd1] = d * (static_cast<double>(n) * o + (ov + nv) * static_cast<double>(kc));
    fl[kPhaseFwd2] = 2.0 * n * static_cast<double>(n) * v * kc;
    by[kPhaseFwd2] = d * (static_cast<double>(n) * v + (nv + nn) * static_cast<double>(kc));
    // contraction: read R, write every F, read the packed ERIs (FP64) once
    by[kPhaseG] = d * (static_cast<double>(kc) * nn + static_cast<double>(nb) * nn) +
                  8.0 * static_cast<double>(m.np) * m.np;
    fl[kPhaseG] = 0.0;
    fl[kPhaseBwd1] = 2.0 * n * static_cast<double>(n) * v * nb;
    by[kPhaseBwd1] = d * (static_cast<double>(n) * v + (nn + nv) * static_cast<double>(nb));
    fl[kPhaseBwd2] = 2.0 * o * static_cast<double>(n) * v * nb;
    by[kPhaseBwd2] = d * (static_cast<double>(n) * o + nv * static_cast<double>(nb)) + 8.0 * 2.0 * ov * nb;
    la[kPhaseFwd1] = f32 ? 2 : 1;
    la[kPhaseFwd2] = 1;
    la[kPhaseG] = 1;
    la[kPhaseBwd1] = 1;
    la[kPhaseBwd2] = tdhf && !merged ? 2 : 1;
    w.timer.pending.push_back(ev);
    w.timer.pending_flops.push_back(fl);
    w.timer.pending_bytes.push_back(by);
    w.timer.pending_launches.push_back(la);
  }
}

}  // namespace seqx
