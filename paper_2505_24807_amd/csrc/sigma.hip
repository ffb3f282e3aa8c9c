// Matrix-free products of Eqs. 8-9 (paper, GPU-implementation subsection).
//
//   R_I   = C_o V_I C_v^T                     two MFMA GEMMs (n x o x v, n x v x n)
//   F_I   = G(R_I)                            NDDO contraction (fock.hip)
//   out_I = C_o^T F_I C_v + de o V_I          two MFMA GEMMs, de added in the epilogue
// Singlet CIS:  F = 2 J(R) - K(R).  TDHF:  (A+B) <-> 4 J(S) - 2 K(S) and
// (A-B) <-> -2 K(D) with S, D the symmetric / antisymmetric parts of R: A V
// pairs with K(R) and B V with K(R^T), which gives exactly these combinations.
#include <mutex>

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

namespace {

// Intermediates of one chunk of kc trial vectors: the FP64 set (T1, R, F, Z)
// or the FP32 set (V32, T1s, Rs, Fs, Zs), and the contraction's work arrays.
struct ChunkBufs {
  double *T1 = nullptr, *R = nullptr, *F = nullptr, *Z = nullptr;
  float *V32 = nullptr, *T1s = nullptr, *Rs = nullptr, *Fs = nullptr, *Zs = nullptr;
  double *gr = nullptr, *gJ = nullptr, *gws = nullptr;
};

// FP32 trial vectors in and FP32 products out (low-precision modes only), in
// place of the FP64 ones
struct F32Io {
  const float* V = nullptr;
  float* out1 = nullptr;
  float* out2 = nullptr;
};

// One chunk of the product: kc vectors Vc -> out1c (and out2c), outputs os
// elements apart.  ev (optional) receives the phase boundaries.
void sigma_chunk(const DeviceMolecule& m, int theory, int kc, const double* Vc, double* out1c, double* out2c, long os,
                 int precision, const ChunkBufs& b, hipStream_t st, std::array<hipEvent_t, kNumPhases + 1>* ev,
                 const F32Io* io = nullptr) {
  const int n = m.nao, o = m.nocc, v = m.nvirt;
  const long nn = static_cast<long>(n) * n, nv = static_cast<long>(n) * v, ov = static_cast<long>(o) * v;
  const bool tdhf = theory == 1;
  const int nb = tdhf ? 2 * kc : kc;
  auto mark = [&](int p) {
    if (ev) SEQX_HIP(hipEventRecord((*ev)[p], st));
  };
  mark(0);
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
  const bool merged = tdhf && os % 2 == 0 && (io ? io->out2 == io->out1 + os / 2 : out2c == out1c + os / 2);
  const long sF = merged ? 2 * nn : nn;
  const long f2off = merged ? nn : kc * nn;
  if (merged) ep.vdiv = 2;
  if (precision == kPrecFP64) {
    // T1_I (n x v) = C[:, :o] V_I
    dgemm(st, false, false, n, v, o, 1.0, m.C.p, n, 0, Vc, v, ov, 0.0, b.T1, v, nv, kc);
    mark(1);
    // R_I (n x n) = T1_I C[:, o:]^T: the T1_I are stacked rows, so one GEMM with M = kc n
    dgemm(st, false, true, kc * n, n, v, 1.0, b.T1, v, 0, m.C.p + o, n, 0, 0.0, b.R, n, 0, 1);
    mark(2);
    if (tdhf)
      build_G(m, kc, b.R, nn, b.F, b.F + f2off, sF, kTwo, 4.0, -2.0, -2.0, b.gr, b.gJ, b.gws, st);
    else
      build_G(m, kc, b.R, nn, b.F, static_cast<double*>(nullptr), nn, kSum, 2.0, -1.0, -1.0, b.gr, b.gJ, b.gws, st);
    mark(3);
    // Z_b (n x v) = F_b (n x n) * C[:, o:], all nb at once (M = nb n)
    dgemm(st, false, false, nb * n, v, n, 1.0, b.F, n, 0, m.C.p + o, n, 0, 0.0, b.Z, v, 0, 1);
    mark(4);
    // out_b (o x v) = C[:, :o]^T * Z_b + de o V_b
    if (merged) {
      dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, b.Z, v, nv, 0.0, out1c, v, os / 2, nb, &ep);
    } else {
      dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, b.Z, v, nv, 0.0, out1c, v, os, kc, &ep);
      if (tdhf) dgemm(st, true, false, o, v, n, 1.0, m.C.p, n, 0, b.Z + kc * nv, v, nv, 0.0, out2c, v, os, kc, &ep);
    }
  } else {
    // FP32 storage; products on the FP32 matrix cores or as split bfloat16 (BF16x3)
    const bool x3 = precision == kPrecBF16x3;
    auto mm = x3 ? sgemm3 : sgemm;
    auto mm64 = x3 ? sgemm3_out64 : sgemm_out64;
    const float* C32 = m.C32.p;
    const float* Vs = b.V32;
    if (io) {
      Vs = io->V;
      ep.V = nullptr;
      ep.Vf = io->V;
    } else {
      to_float(st, kc * ov, Vc, b.V32);
    }
    mm(st, false, false, n, v, o, 1.0, C32, n, 0, Vs, v, ov, 0.0, b.T1s, v, nv, kc, nullptr);
    mark(1);
    mm(st, false, true, kc * n, n, v, 1.0, b.T1s, v, 0, C32 + o, n, 0, 0.0, b.Rs, n, 0, 1, nullptr);
    mark(2);
    if (tdhf)
      build_G(m, kc, b.Rs, nn, b.Fs, b.Fs + f2off, sF, kTwo, 4.0, -2.0, -2.0, b.gr, b.gJ, b.gws, st);
    else
      build_G(m, kc, b.Rs, nn, b.Fs, static_cast<float*>(nullptr), nn, kSum, 2.0, -1.0, -1.0, b.gr, b.gJ, b.gws, st);
    mark(3);
    mm(st, false, false, nb * n, v, n, 1.0, b.Fs, n, 0, C32 + o, n, 0, 0.0, b.Zs, v, 0, 1, nullptr);
    mark(4);
    if (io) {
      if (merged) {
        mm(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs, v, nv, 0.0, io->out1, v, os / 2, nb, &ep);
      } else {
        mm(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs, v, nv, 0.0, io->out1, v, os, kc, &ep);
        if (tdhf) mm(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs + kc * nv, v, nv, 0.0, io->out2, v, os, kc, &ep);
      }
    } else if (merged) {
      mm64(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs, v, nv, 0.0, out1c, v, os / 2, nb, &ep);
    } else {
      mm64(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs, v, nv, 0.0, out1c, v, os, kc, &ep);
      if (tdhf) mm64(st, true, false, o, v, n, 1.0, C32, n, 0, b.Zs + kc * nv, v, nv, 0.0, out2c, v, os, kc, &ep);
    }
  }
  mark(5);
}

void check_sigma_args(const DeviceMolecule& m, int precision) {
  if (precision != kPrecFP64 && precision != kPrecFP32 && precision != kPrecBF16x3)
    throw Error(kEArg, "unsupported transform precision");
  if (precision != kPrecFP64 && m.C32.n < static_cast<size_t>(m.nao) * m.nao)
    throw Error(kEState, "FP32 MO coefficients missing");
}

// Pieces of one chunk's intermediates laid out in a single workspace, each
// starting on a 256-byte boundary; returns the bytes used.  base == nullptr
// only measures.
size_t carve_chunk(const DeviceMolecule& m, int theory, int kc, int precision, unsigned char* base, ChunkBufs* b) {
  const size_t n = m.nao, v = m.nvirt, ov = static_cast<size_t>(m.nocc) * m.nvirt;
  const size_t nn = n * n, nv = n * v, nb = theory == 1 ? 2 * static_cast<size_t>(kc) : kc;
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    unsigned char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  ChunkBufs c;
  if (precision == kPrecFP64) {
    c.T1 = reinterpret_cast<double*>(take(kc * nv * sizeof(double)));
    c.R = reinterpret_cast<double*>(take(kc * nn * sizeof(double)));
    c.F = reinterpret_cast<double*>(take(nb * nn * sizeof(double)));
    c.Z = reinterpret_cast<double*>(take(nb * nv * sizeof(double)));
  } else {
    c.V32 = reinterpret_cast<float*>(take(kc * ov * sizeof(float)));
    c.T1s = reinterpret_cast<float*>(take(kc * nv * sizeof(float)));
    c.Rs = reinterpret_cast<float*>(take(kc * nn * sizeof(float)));
    c.Fs = reinterpret_cast<float*>(take(nb * nn * sizeof(float)));
    c.Zs = reinterpret_cast<float*>(take(nb * nv * sizeof(float)));
  }
  const size_t kp = static_cast<size_t>(kc) * m.np;
  c.gr = reinterpret_cast<double*>(take(kp * sizeof(double)));
  c.gJ = reinterpret_cast<double*>(take(kp * sizeof(double)));
  c.gws = reinterpret_cast<double*>(take((g_work_doubles(kc, m.np) - 2 * kp) * sizeof(double)));
  if (b) *b = c;
  return off;
}

// Algorithmic work of one chunk (flops, bytes, launches per phase); d = bytes
// per stored element of the transforms.
void chunk_work(const DeviceMolecule& m, int theory, int kc, int precision, bool merged,
                std::array<double, kNumPhases>& fl, std::array<double, kNumPhases>& by,
                std::array<long, kNumPhases>& la) {
  const int n = m.nao, o = m.nocc, v = m.nvirt;
  const long nn = static_cast<long>(n) * n, nv = static_cast<long>(n) * v, ov = static_cast<long>(o) * v;
  const bool tdhf = theory == 1, f32 = precision != kPrecFP64;
  const int nb = tdhf ? 2 * kc : kc;
  const double d = f32 ? 4.0 : 8.0;
  fl = {};
  by = {};
  la = {};
  fl[kPhaseFwd1] = 2.0 * n * o * v * kc;
  by[kPhaseFwd1] = d * (static_cast<double>(n) * o + (ov + nv) * static_cast<double>(kc));
  fl[kPhaseFwd2] = 2.0 * n * static_cast<double>(n) * v * kc;
  by[kPhaseFwd2] = d * (static_cast<double>(n) * v + (nv + nn) * static_cast<double>(kc));
  // contraction: read R, write every F, read the packed ERIs (FP64) once
  by[kPhaseG] = d * (static_cast<double>(kc) * nn + static_cast<double>(nb) * nn) + 8.0 * static_cast<double>(m.np) * m.np;
  fl[kPhaseBwd1] = 2.0 * n * static_cast<double>(n) * v * nb;
  by[kPhaseBwd1] = d * (static_cast<double>(n) * v + (nn + nv) * static_cast<double>(nb));
  fl[kPhaseBwd2] = 2.0 * o * static_cast<double>(n) * v * nb;
  by[kPhaseBwd2] = d * (static_cast<double>(n) * o + nv * static_cast<double>(nb)) + 8.0 * 2.0 * ov * nb;
  la[kPhaseFwd1] = f32 ? 2 : 1;
  la[kPhaseFwd2] = 1;
  la[kPhaseG] = 1;
  la[kPhaseBwd1] = 1;
  la[kPhaseBwd2] = tdhf && !merged ? 2 : 1;
}

}  // namespace

namespace {

// FP64 vectors and products (V, out1, out2), or FP32 ones (Vf, out1f, out2f)
void sigma_build_any(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                     const float* Vf, float* out1f, float* out2f, SigmaWork& w, hipStream_t st, int chunk,
                     long out_stride, int precision) {
  const int n = m.nao, o = m.nocc, v = m.nvirt;
  const long nn = static_cast<long>(n) * n, nv = static_cast<long>(n) * v, ov = static_cast<long>(o) * v;
  const long os = out_stride > 0 ? out_stride : ov;
  const bool tdhf = theory == 1;
  const bool f32io = Vf != nullptr;
  check_sigma_args(m, precision);
  if (f32io && precision == kPrecFP64) throw Error(kEArg, "FP32 vectors need a low-precision transform mode");
  for (int c0 = 0; c0 < k; c0 += chunk) {
    const int kc = std::min(chunk, k - c0);
    const int nb = tdhf ? 2 * kc : kc;
    ChunkBufs b;
    if (precision != kPrecFP64) {
      w.V32.ensure(static_cast<size_t>(kc) * ov);
      w.Rs.ensure(static_cast<size_t>(kc) * nn);
      w.Fs.ensure(static_cast<size_t>(nb) * nn);
      w.Zs.ensure(static_cast<size_t>(nb) * nv);
      w.T1s.ensure(static_cast<size_t>(kc) * nv);
      b.V32 = w.V32.p;
      b.Rs = w.Rs.p;
      b.Fs = w.Fs.p;
      b.Zs = w.Zs.p;
      b.T1s = w.T1s.p;
    } else {
      w.R.ensure(static_cast<size_t>(kc) * nn);
      w.F.ensure(static_cast<size_t>(nb) * nn);
      w.Z.ensure(static_cast<size_t>(nb) * nv);
      w.T1.ensure(static_cast<size_t>(kc) * nv);
      b.R = w.R.p;
      b.F = w.F.p;
      b.Z = w.Z.p;
      b.T1 = w.T1.p;
    }
    w.g.r.ensure(static_cast<size_t>(kc) * m.np);
    w.g.J.ensure(static_cast<size_t>(kc) * m.np);
    w.g.ws.ensure(dots_workspace(kc, m.np, m.np));
    b.gr = w.g.r.p;
    b.gJ = w.g.J.p;
    b.gws = w.g.ws.p;
    std::array<hipEvent_t, kNumPhases + 1> ev;
    for (auto& e : ev) SEQX_HIP(hipEventCreate(&e));
    bool merged;
    if (f32io) {
      F32Io io;
      io.V = Vf + c0 * ov;
      io.out1 = out1f + c0 * os;
      io.out2 = out2f ? out2f + c0 * os : nullptr;
      sigma_chunk(m, theory, kc, nullptr, nullptr, nullptr, os, precision, b, st, &ev, &io);
      merged = tdhf && os % 2 == 0 && io.out2 == io.out1 + os / 2;
    } else {
      double* o1 = out1 + c0 * os;
      double* o2 = out2 ? out2 + c0 * os : nullptr;
      sigma_chunk(m, theory, kc, V + c0 * ov, o1, o2, os, precision, b, st, &ev);
      merged = tdhf && os % 2 == 0 && o2 == o1 + os / 2;
    }
    std::array<double, kNumPhases> fl, by;
    std::array<long, kNumPhases> la;
    chunk_work(m, theory, kc, precision, merged, fl, by, la);
    w.timer.pending.push_back(ev);
    w.timer.pending_flops.push_back(fl);
    w.timer.pending_bytes.push_back(by);
    w.timer.pending_launches.push_back(la);
  }
}

}  // namespace

void sigma_build(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                 SigmaWork& w, hipStream_t st, int chunk, long out_stride, int precision) {
  sigma_build_any(m, theory, k, V, out1, out2, nullptr, nullptr, nullptr, w, st, chunk, out_stride, precision);
}

void sigma_build_f32(const DeviceMolecule& m, int theory, int k, const float* V, float* out1, float* out2,
                     SigmaWork& w, hipStream_t st, int chunk, long out_stride, int precision) {
  sigma_build_any(m, theory, k, nullptr, nullptr, nullptr, V, out1, out2, w, st, chunk, out_stride, precision);
}

// ---- no-allocation variant --------------------------------------------------
// One fixed workspace per GPU: a file-scope device array.  Its name is only a
// host-side stand-in for the symbol; the device address of each GPU's copy
// comes from hipGetSymbolAddress (sigma_scratch_setup) and only that address
// is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kSigmaScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

void sigma_scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) throw Error(kEDevice, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error(kEDevice, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
}

int sigma_scratch_max_chunk(const DeviceMolecule& m, int theory, int precision) {
  int kc = 32;
  while (kc > 0 && carve_chunk(m, theory, kc, precision, nullptr, nullptr) > kSigmaScratchBytes) --kc;
  return kc;
}

void sigma_build_noalloc(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                         hipStream_t st, int precision) {
  check_sigma_args(m, precision);
  int device = 0;
  SEQX_HIP(hipGetDevice(&device));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device >= 0 && device < kMaxScratchDevices) base = g_scratch_ptr[device];
  }
  if (!base) {
    sigma_scratch_setup(device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[device];
  }
  const int chunk = sigma_scratch_max_chunk(m, theory, precision);
  if (chunk < 1)
    throw Error(kEBufSize, "one trial vector needs " +
                               std::to_string(carve_chunk(m, theory, 1, precision, nullptr, nullptr)) +
                               " bytes of intermediates; the fixed workspace holds " +
                               std::to_string(kSigmaScratchBytes));
  const long ov = static_cast<long>(m.nocc) * m.nvirt;
  for (int c0 = 0; c0 < k; c0 += chunk) {
    const int kc = std::min(chunk, k - c0);
    ChunkBufs b;
    carve_chunk(m, theory, kc, precision, static_cast<unsigned char*>(base), &b);
    sigma_chunk(m, theory, kc, V + c0 * ov, out1 + c0 * ov, out2 ? out2 + c0 * ov : nullptr, ov, precision, b, st,
                nullptr);
  }
}

}  // namespace seqx
