// C ABI of libseqx (declared in include/seqx.h): context and job lifecycle,
// host validation, argument marshalling and the error model.  No exception
// crosses the boundary; every entry point returns a status code.
#include <cctype>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <deque>
#include <fstream>
#include <map>
#include <atomic>
#include <exception>
#include <thread>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/seqx.h"
#include "batch.hpp"
#include "davidson.hpp"
#include "gradient.hpp"
#include "integrals.hpp"
#include "linalg.hpp"
#include "mlp.hpp"
#include "model.hpp"
#include "molecule.hpp"
#include "scf.hpp"
#include "sigma.hpp"
#include "spectrum.hpp"

namespace seqx {
thread_local const DeviceAllocator* g_device_allocator = nullptr;
static_assert(SEQX_SIGMA_SCRATCH_BYTES == kSigmaScratchBytes, "workspace size of the header and the library differ");
}  // namespace seqx

using namespace seqx;

struct seqx_ctx {
  // caller allocators, never modified once added (buffers keep a pointer to
  // theirs).  Declared first so that they are destroyed last, after every
  // buffer of the context has been handed back.
  std::deque<DeviceAllocator> allocators;
  const DeviceAllocator* allocator = nullptr;  // current one; nullptr: hipMalloc / hipFree
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  Elem elems[kNumSlots];
  double raw[kNumSlots][SEQX_NPARAM] = {};  // the parameter values behind elems (eV, 1/bohr)
  bool have[kNumSlots] = {false, false, false};
  DBuf<Elem> d_elems;
  std::unique_ptr<DenseSolver> ds;
  TileTuning tune;
  Mlp mlp;
  MlpWork mw;
};

struct seqx_job {
  seqx_ctx* ctx = nullptr;
  std::vector<std::unique_ptr<DeviceMolecule>> mols;
  GWork gw;
  ScfWork sw;
  DavWork dw;
  BatchWork bw;
  DBuf<double> guess_v;
  DBuf<double> lock_t, lock_u;  // locked roots of a root-batch solve
  seqx_stats stats{};
  bool solved = false;
};

namespace {

thread_local std::string g_noctx_err;

// makes the context's allocator current for the duration of one ABI call
struct AllocatorScope {
  const DeviceAllocator* saved;
  explicit AllocatorScope(const seqx_ctx* ctx) : saved(g_device_allocator) {
    g_device_allocator = ctx ? ctx->allocator : nullptr;
  }
  ~AllocatorScope() { g_device_allocator = saved; }
};

template <class F>
seqx_status guarded(seqx_ctx* ctx, F&& f) {
  AllocatorScope scope(ctx);
  try {
    if (ctx) SEQX_HIP(hipSetDevice(ctx->device));
    f();
    if (ctx) ctx->err.clear();
    return SEQX_OK;
  } catch (const Error& e) {
    (ctx ? ctx->err : g_noctx_err) = e.what();
    return static_cast<seqx_status>(e.status);
  } catch (const std::bad_alloc&) {
    (ctx ? ctx->err : g_noctx_err) = "host allocation failed";
    return SEQX_E_NOMEM;
  } catch (const std::exception& e) {
    (ctx ? ctx->err : g_noctx_err) = e.what();
    return SEQX_E_DEVICE;
  }
}

template <class T>
void h2d(DBuf<T>& d, const std::vector<T>& h, hipStream_t st) {
  d.alloc(h.size());
  if (!h.empty()) SEQX_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

template <class T>
void d2h(T* dst, const T* src, size_t n, hipStream_t st) {
  if (n) SEQX_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}

DeviceMolecule& mol_of(const seqx_job* job, int32_t mol) {
  if (!job) throw Error(kEArg, "job is NULL");
  if (mol < 0 || mol >= static_cast<int>(job->mols.size())) throw Error(kEArg, "molecule index out of range");
  return *job->mols[mol];
}

DeviceMolecule& scf_mol_of(const seqx_job* job, int32_t mol) {
  DeviceMolecule& m = mol_of(job, mol);
  if (!m.scf_done) throw Error(kEState, "job was prepared with integrals_only: no ground state");
  return m;
}

void setup_molecule(seqx_ctx* ctx, DeviceMolecule& m, int natoms, const int32_t* Z, const double* xyz,
                    hipStream_t st) {
  m.L = make_layout(natoms, Z, xyz, ctx->elems);
  const Layout& L = m.L;
  m.natoms = L.natoms;
  m.nheavy = L.nheavy;
  m.nao = L.nao;
  m.nocc = L.nocc;
  m.nvirt = L.nvirt;
  m.np = L.np;
  m.elems = ctx->d_elems.p;
  h2d(m.slot, L.slot, st);
  h2d(m.ao_off, L.ao_off, st);
  h2d(m.pi_off, L.pi_off, st);
  h2d(m.xyz, L.xyz, st);
  std::vector<int2> pr[3];
  for (int A = 0; A < natoms; ++A)
    for (int B = A + 1; B < natoms; ++B) {
      const int g = (B < L.nheavy) ? 0 : (A < L.nheavy ? 1 : 2);
      pr[g].push_back(make_int2(A, B));
    }
  for (int g = 0; g < 3; ++g) {
    m.npairs[g] = static_cast<int>(pr[g].size());
    h2d(m.pairs[g], pr[g], st);
  }
  std::vector<int> pmu(L.np), pnu(L.np), aoa(L.nao);
  for (int A = 0; A < natoms; ++A) {
    const int o = L.ao_off[A], na = L.ao_off[A + 1] - o, po = L.pi_off[A];
    for (int i = 0; i < na; ++i) aoa[o + i] = A;
    if (na == 1) {
      pmu[po] = o;
      pnu[po] = o;
    } else {
      for (int P = 0; P < 10; ++P) {
        pmu[po + P] = o + pair_first(P);
        pnu[po + P] = o + pair_second(P);
      }
    }
  }
  h2d(m.pi_mu, pmu, st);
  h2d(m.pi_nu, pnu, st);
  h2d(m.atom_of_ao, aoa, st);
  m.W.alloc(static_cast<size_t>(L.np) * L.np);
  m.H.alloc(static_cast<size_t>(L.nao) * L.nao);
}

// permute a square internal-order matrix into input order
void unpermute_square(const std::vector<double>& in, int n, const std::vector<int>& map, double* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[static_cast<size_t>(map[i]) * n + map[j]] = in[static_cast<size_t>(i) * n + j];
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  SEQX_HIP(hipEventElapsedTime(&ms, a, b));
  return ms;
}

// Molecules of a batch are independent.  One molecule's launches are small and
// its SCF waits on the host every few purification steps, so a single stream
// leaves the GPU mostly idle: from kPrepareParallelMin molecules on, a few
// host threads, each with its own stream, dense solver and work buffers, take
// molecules in turn.  Every molecule gets exactly the computation of the
// sequential path.  Buffers come from hipMalloc here (with a caller allocator
// the sequential path runs, so its callbacks are only entered from the calling
// thread).  Times are summed over molecules.
constexpr int kPrepareParallelMin = 4;
constexpr int kPrepareThreads = 8;

// Worker threads of a batched preparation: SEQX_PREPARE_THREADS (1 .. 64) when
// set, else kPrepareThreads; 1 keeps the preparation on the calling thread.
int prepare_threads() {
  static const int n = [] {
    const char* s = std::getenv("SEQX_PREPARE_THREADS");
    if (!s || !*s) return kPrepareThreads;
    const int v = std::atoi(s);
    return v >= 1 && v <= 64 ? v : kPrepareThreads;
  }();
  return n;
}

void prepare_parallel(seqx_ctx* ctx, seqx_job* job, int nmol, const int32_t* natoms, const int32_t* Z,
                      const double* xyz, const ScfOptions& so, bool integrals_only) {
  std::vector<size_t> offs(nmol, 0);
  for (int m = 1; m < nmol; ++m) offs[m] = offs[m - 1] + natoms[m - 1];
  std::vector<std::unique_ptr<DeviceMolecule>> mols(nmol);
  std::vector<double> t_int(nmol, 0.0), t_scf(nmol, 0.0);
  std::atomic<int> next{0};
  const int nw = std::min(nmol, prepare_threads());
  std::vector<std::exception_ptr> errs(nw);
  SEQX_HIP(hipStreamSynchronize(ctx->stream));  // element data uploaded on the context stream
  std::vector<std::thread> pool;
  // joins the started workers however this function is left (a thread that
  // cannot be started stops the others after their current molecule)
  struct Joiner {
    std::vector<std::thread>& p;
    std::atomic<int>& next;
    int nmol;
    ~Joiner() {
      if (std::uncaught_exceptions() > 0) next.store(nmol);
      for (auto& t : p)
        if (t.joinable()) t.join();
    }
  } joiner{pool, next, nmol};
  for (int wk = 0; wk < nw; ++wk)
    pool.emplace_back([&, wk] {
      try {
        SEQX_HIP(hipSetDevice(ctx->device));
        hipStream_t ws = nullptr;
        SEQX_HIP(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
        struct StreamGuard {
          hipStream_t s;
          ~StreamGuard() {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
          }
        } guard{ws};
        hipEvent_t e[3] = {nullptr, nullptr, nullptr};
        struct EventGuard {
          hipEvent_t* e;
          ~EventGuard() {
            for (int i = 0; i < 3; ++i)
              if (e[i]) (void)hipEventDestroy(e[i]);
          }
        } eguard{e};
        for (auto& ev : e) SEQX_HIP(hipEventCreate(&ev));
        DenseSolver ds(ws);
        GWork gw;
        ScfWork sw;
        for (int m = next.fetch_add(1); m < nmol; m = next.fetch_add(1)) {
          std::unique_ptr<DeviceMolecule> dm(new DeviceMolecule());
          setup_molecule(ctx, *dm, natoms[m], Z + offs[m], xyz + 3 * offs[m], ws);
          SEQX_HIP(hipEventRecord(e[0], ws));
          build_integrals(*dm, ws);
          SEQX_HIP(hipEventRecord(e[1], ws));
          if (!integrals_only) run_scf(*dm, so, ds, gw, sw, ws);
          dm->scf_done = !integrals_only;
          SEQX_HIP(hipEventRecord(e[2], ws));
          SEQX_HIP(hipStreamSynchronize(ws));
          t_int[m] = elapsed_ms(e[0], e[1]);
          t_scf[m] = elapsed_ms(e[1], e[2]);
          mols[m] = std::move(dm);
        }
      } catch (...) {
        errs[wk] = std::current_exception();
        next.store(nmol);  // the others stop after their current molecule
      }
    });
  for (auto& t : pool) t.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  double ti = 0.0, ts = 0.0;
  for (int m = 0; m < nmol; ++m) {
    ti += t_int[m];
    ts += t_scf[m];
    job->stats.scf_iterations += mols[m]->scf_iterations;
    job->stats.commutator = std::max(job->stats.commutator, mols[m]->commutator);
    job->mols.push_back(std::move(mols[m]));
  }
  job->stats.t_integrals_s = ti * 1e-3;
  job->stats.t_scf_s = ts * 1e-3;
}

}  // namespace

extern "C" {

int seqx_abi_version(void) { return SEQX_ABI_VERSION; }

seqx_status seqx_validate(int32_t nmol, const int32_t* natoms, const int32_t* Z, const double* xyz, char* msg,
                          size_t msglen) {
  try {
    validate_molecules(nmol, natoms, Z, xyz);
    if (msg && msglen) msg[0] = 0;
    return SEQX_OK;
  } catch (const Error& e) {
    if (msg && msglen) {
      std::strncpy(msg, e.what(), msglen - 1);
      msg[msglen - 1] = 0;
    }
    return static_cast<seqx_status>(e.status);
  }
}

seqx_status seqx_create(int device, void* hip_stream, seqx_ctx** out) {
  if (!out) return SEQX_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    g_noctx_err = "no HIP device available";
    return SEQX_E_DEVICE;
  }
  if (device < 0 || device >= count) {
    g_noctx_err = "device index out of range";
    return SEQX_E_ARG;
  }
  std::unique_ptr<seqx_ctx> ctx(new seqx_ctx());
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  const seqx_status s = guarded(ctx.get(), [&] {
    ctx->d_elems.alloc(kNumSlots);
    ctx->ds.reset(new DenseSolver(ctx->stream));
    // device address of this GPU's fixed sigma workspace (no-allocation entry point)
    sigma_scratch_setup(device);
  });
  if (s != SEQX_OK) {
    g_noctx_err = ctx->err;
    return s;
  }
  *out = ctx.release();
  return SEQX_OK;
}

void seqx_destroy(seqx_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

const char* seqx_last_error(const seqx_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

namespace {

// Minimal JSON reader for parameter files: objects, arrays, strings, numbers,
// true / false / null.  Parse errors raise SEQX_E_ARG.
struct Json {
  enum Kind { kNull, kNum, kStr, kObj, kArr, kBool } kind = kNull;
  double num = 0.0;
  std::string str;
  std::map<std::string, Json> obj;
  std::vector<Json> arr;
};

struct JsonParser {
  const std::string& t;
  size_t i = 0;
  explicit JsonParser(const std::string& text) : t(text) {}
  [[noreturn]] void fail(const char* what) {
    throw Error(kEArg, std::string("parameter file: ") + what + " at offset " + std::to_string(i));
  }
  void ws() { while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i; }
  std::string string() {
    if (t[i] != '"') fail("string expected");
    std::string out;
    for (++i; i < t.size() && t[i] != '"'; ++i) {
      if (t[i] == '\\') {
        if (++i >= t.size()) fail("bad escape");
        const char c = t[i];
        out += c == 'n' ? '\n' : c == 't' ? '\t' : c;
      } else {
        out += t[i];
      }
    }
    if (i >= t.size()) fail("unterminated string");
    ++i;
    return out;
  }
  Json value() {
    ws();
    if (i >= t.size()) fail("value expected");
    Json v;
    const char c = t[i];
    if (c == '{') {
      v.kind = Json::kObj;
      ++i;
      ws();
      if (i < t.size() && t[i] == '}') { ++i; return v; }
      for (;;) {
        ws();
        const std::string key = string();
        ws();
        if (i >= t.size() || t[i] != ':') fail("':' expected");
        ++i;
        v.obj[key] = value();
        ws();
        if (i < t.size() && t[i] == ',') { ++i; continue; }
        if (i < t.size() && t[i] == '}') { ++i; return v; }
        fail("',' or '}' expected");
      }
    }
    if (c == '[') {
      v.kind = Json::kArr;
      ++i;
      ws();
      if (i < t.size() && t[i] == ']') { ++i; return v; }
      for (;;) {
        v.arr.push_back(value());
        ws();
        if (i < t.size() && t[i] == ',') { ++i; continue; }
        if (i < t.size() && t[i] == ']') { ++i; return v; }
        fail("',' or ']' expected");
      }
    }
    if (c == '"') {
      v.kind = Json::kStr;
      v.str = string();
      return v;
    }
    if (t.compare(i, 4, "true") == 0 || t.compare(i, 5, "false") == 0) {
      v.kind = Json::kBool;
      v.num = t[i] == 't' ? 1.0 : 0.0;
      i += t[i] == 't' ? 4 : 5;
      return v;
    }
    if (t.compare(i, 4, "null") == 0) {
      i += 4;
      return v;
    }
    const char* b = t.c_str() + i;
    char* e = nullptr;
    v.num = std::strtod(b, &e);
    if (e == b) fail("number expected");
    v.kind = Json::kNum;
    i += static_cast<size_t>(e - b);
    return v;
  }
};

void set_params_impl(seqx_ctx* ctx, int32_t nelem, const int32_t* Z, const double* values) {
    if (nelem <= 0 || !Z || !values) throw Error(kEArg, "nelem must be > 0 and arrays non-null");
    for (int i = 0; i < nelem; ++i) {
      const int s = element_slot(Z[i]);
      if (s < 0) throw Error(kEElement, "unsupported element Z=" + std::to_string(Z[i]));
      const double* v = values + static_cast<size_t>(i) * SEQX_NPARAM;
      const int need = Z[i] == 1 ? 1 : SEQX_NPARAM;
      for (int k = 0; k < need; ++k)
        if (!std::isfinite(v[k])) throw Error(kEArg, "non-finite parameter");
      if (v[0] <= 0 || (Z[i] != 1 && v[1] <= 0)) throw Error(kEArg, "orbital exponents must be positive");
      if (v[6] <= 0 || (Z[i] != 1 && (v[10] <= 0 || v[8] <= v[9])))
        throw Error(kEArg, "one-centre parameters need g_ss > 0, h_sp > 0 and g_pp > g_p2");
      ctx->elems[s] = make_elem(Z[i], v);
      for (int k = 0; k < SEQX_NPARAM; ++k) ctx->raw[s][k] = v[k];
      ctx->have[s] = true;
    }
    SEQX_HIP(hipMemcpyAsync(ctx->d_elems.p, ctx->elems, sizeof(ctx->elems), hipMemcpyHostToDevice, ctx->stream));
    SEQX_HIP(hipStreamSynchronize(ctx->stream));
}

}  // namespace

seqx_status seqx_set_params(seqx_ctx* ctx, int32_t nelem, const int32_t* Z, const double* values) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] { set_params_impl(ctx, nelem, Z, values); });
}

seqx_status seqx_load_params(seqx_ctx* ctx, seqx_method method, const char* path) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    if (method != SEQX_PARAMS_FILE)
      throw Error(kEArg, "published MNDO/AM1/PM3 tables are not bundled; load a parameter file (SEQX_PARAMS_FILE)");
    if (!path) throw Error(kEArg, "parameter file path is null");
    std::ifstream f(path);
    if (!f) throw Error(kEArg, std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    JsonParser jp(text);
    const Json doc = jp.value();
    auto it = doc.obj.find("elements");
    if (doc.kind != Json::kObj || it == doc.obj.end() || it->second.kind != Json::kObj)
      throw Error(kEArg, "parameter file has no \"elements\" object");
    static const char* const names[SEQX_NPARAM] = {"zeta_s", "zeta_p", "U_ss", "U_pp", "beta_s", "beta_p",
                                                   "g_ss", "g_sp", "g_pp", "g_p2", "h_sp"};
    std::vector<int32_t> zs;
    std::vector<double> vals;
    for (const auto& kv : it->second.obj) {
      char* e = nullptr;
      const long z = std::strtol(kv.first.c_str(), &e, 10);
      if (e == kv.first.c_str() || *e != '\0') throw Error(kEArg, "element key is not an atomic number: " + kv.first);
      if (kv.second.kind != Json::kObj) throw Error(kEArg, "element entry is not an object: " + kv.first);
      zs.push_back(static_cast<int32_t>(z));
      for (const char* nm : names) {
        auto p = kv.second.obj.find(nm);
        if (p != kv.second.obj.end() && p->second.kind != Json::kNum)
          throw Error(kEArg, std::string("parameter ") + nm + " of Z=" + kv.first + " is not a number");
        vals.push_back(p == kv.second.obj.end() ? 0.0 : p->second.num);  // absent (p terms of H): 0
      }
    }
    set_params_impl(ctx, static_cast<int32_t>(zs.size()), zs.data(), vals.data());
  });
}

seqx_status seqx_set_allocator(seqx_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                               void (*release)(void* ptr, void* user), void* user) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    if (!alloc != !release) throw Error(kEArg, "alloc and release must both be set or both be null");
    if (!alloc) {
      ctx->allocator = nullptr;
      return;
    }
    DeviceAllocator a;
    a.alloc = alloc;
    a.release = release;
    a.user = user;
    ctx->allocators.push_back(a);
    ctx->allocator = &ctx->allocators.back();
  });
}

seqx_status seqx_prepare(seqx_ctx* ctx, int32_t nmol, const int32_t* natoms, const int32_t* Z, const double* xyz,
                         const seqx_scf_opts* opts, seqx_job** out) {
  if (!ctx || !out) return SEQX_E_ARG;
  *out = nullptr;
  std::unique_ptr<seqx_job> job(new seqx_job());
  job->ctx = ctx;
  const seqx_status s = guarded(ctx, [&] {
    validate_molecules(nmol, natoms, Z, xyz);
    size_t off = 0;
    for (int m = 0; m < nmol; ++m) {
      for (int a = 0; a < natoms[m]; ++a)
        if (!ctx->have[element_slot(Z[off + a])])
          throw Error(kEElement, "no parameters loaded for Z=" + std::to_string(Z[off + a]));
      off += natoms[m];
    }
    ScfOptions so;
    bool integrals_only = false;
    if (opts) {
      if (opts->tol > 0) so.tol = opts->tol;
      if (opts->max_iter > 0) so.max_iter = opts->max_iter;
      if (opts->ndiis > 0) so.ndiis = opts->ndiis;
      integrals_only = opts->integrals_only != 0;
    }
    hipStream_t st = ctx->stream;
    if (nmol >= kPrepareParallelMin && !ctx->allocator && prepare_threads() > 1) {
      prepare_parallel(ctx, job.get(), nmol, natoms, Z, xyz, so, integrals_only);
      return;
    }
    hipEvent_t e[3];
    for (auto& ev : e) SEQX_HIP(hipEventCreate(&ev));
    off = 0;
    double t_int = 0, t_scf = 0;
    try {
      for (int m = 0; m < nmol; ++m) {
        std::unique_ptr<DeviceMolecule> dm(new DeviceMolecule());
        setup_molecule(ctx, *dm, natoms[m], Z + off, xyz + 3 * off, st);
        SEQX_HIP(hipEventRecord(e[0], st));
        build_integrals(*dm, st);
        SEQX_HIP(hipEventRecord(e[1], st));
        if (!integrals_only) run_scf(*dm, so, *ctx->ds, job->gw, job->sw, st);
        dm->scf_done = !integrals_only;
        SEQX_HIP(hipEventRecord(e[2], st));
        SEQX_HIP(hipStreamSynchronize(st));
        t_int += elapsed_ms(e[0], e[1]);
        t_scf += elapsed_ms(e[1], e[2]);
        job->stats.scf_iterations += dm->scf_iterations;
        job->stats.commutator = std::max(job->stats.commutator, dm->commutator);
        job->mols.push_back(std::move(dm));
        off += natoms[m];
      }
    } catch (...) {
      for (auto& ev : e) (void)hipEventDestroy(ev);
      throw;
    }
    for (auto& ev : e) (void)hipEventDestroy(ev);
    job->stats.t_integrals_s = t_int * 1e-3;
    job->stats.t_scf_s = t_scf * 1e-3;
  });
  if (s != SEQX_OK) return s;
  *out = job.release();
  return SEQX_OK;
}

void seqx_job_free(seqx_job* job) {
  if (!job) return;
  (void)hipSetDevice(job->ctx->device);
  (void)hipStreamSynchronize(job->ctx->stream);
  delete job;
}

seqx_status seqx_dims(const seqx_job* job, int32_t mol, int32_t* nao, int32_t* nocc, int32_t* nvirt) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    if (nao) *nao = m.nao;
    if (nocc) *nocc = m.nocc;
    if (nvirt) *nvirt = m.nvirt;
  });
}

seqx_status seqx_scf_results(const seqx_job* job, int32_t mol, double* eps_eV, double* C, double* P) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = scf_mol_of(job, mol);
    hipStream_t st = job->ctx->stream;
    const int n = m.nao;
    std::vector<double> e(n), c, p;
    d2h(e.data(), m.eps.p, n, st);
    if (C) {
      c.resize(static_cast<size_t>(n) * n);
      d2h(c.data(), m.C.p, c.size(), st);
    }
    if (P) {
      p.resize(static_cast<size_t>(n) * n);
      d2h(p.data(), m.P.p, p.size(), st);
    }
    SEQX_HIP(hipStreamSynchronize(st));
    if (eps_eV)
      for (int i = 0; i < n; ++i) eps_eV[i] = e[i] * kHartreeEV;
    if (C)  // rows are AOs (permute), columns are MOs (unchanged)
      for (int mu = 0; mu < n; ++mu)
        for (int q = 0; q < n; ++q) C[static_cast<size_t>(m.L.ao_user[mu]) * n + q] = c[static_cast<size_t>(mu) * n + q];
    if (P) unpermute_square(p, n, m.L.ao_user, P);
  });
}

seqx_status seqx_core_hamiltonian(const seqx_job* job, int32_t mol, double* H) {
  if (!job || !H) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    const int n = m.nao;
    std::vector<double> h(static_cast<size_t>(n) * n);
    d2h(h.data(), m.H.p, h.size(), job->ctx->stream);
    SEQX_HIP(hipStreamSynchronize(job->ctx->stream));
    unpermute_square(h, n, m.L.ao_user, H);
  });
}

seqx_status seqx_integrals(const seqx_job* job, int32_t mol, double* out, size_t cap, size_t* needed) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    const size_t need = static_cast<size_t>(m.np) * m.np;
    if (needed) *needed = need;
    if (!out) return;
    if (cap < need) throw Error(kEBufSize, "integral buffer too small");
    std::vector<double> w(need);
    d2h(w.data(), m.W.p, need, job->ctx->stream);
    SEQX_HIP(hipStreamSynchronize(job->ctx->stream));
    unpermute_square(w, m.np, m.L.pi_user, out);
  });
}

namespace {
void check_precision(int32_t precision) {
  if (precision == SEQX_FP64 || precision == SEQX_FP32 || precision == SEQX_BF16X3) return;
  if (precision == SEQX_BF16) throw Error(kEArg, "single-bfloat16 transforms are not available (use SEQX_BF16X3)");
  throw Error(kEArg, "unknown precision");
}
}  // namespace

seqx_status seqx_sigma_device(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* dV, double* dout1,
                              double* dout2, int32_t precision) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    DeviceMolecule& m = scf_mol_of(job, mol);
    if (theory != SEQX_CIS && theory != SEQX_TDHF) throw Error(kEArg, "theory must be CIS or TDHF");
    if (k <= 0 || !dV || !dout1 || (theory == SEQX_TDHF && !dout2)) throw Error(kEArg, "bad sigma arguments");
    check_precision(precision);
    sigma_build(m, theory, k, dV, dout1, dout2, job->dw.sig, job->ctx->stream, 32, 0, precision);
  });
}

seqx_status seqx_sigma_device_noalloc(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* dV,
                                      double* dout1, double* dout2, int32_t precision) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    DeviceMolecule& m = scf_mol_of(job, mol);
    if (theory != SEQX_CIS && theory != SEQX_TDHF) throw Error(kEArg, "theory must be CIS or TDHF");
    if (k <= 0 || !dV || !dout1 || (theory == SEQX_TDHF && !dout2)) throw Error(kEArg, "bad sigma arguments");
    check_precision(precision);
    sigma_build_noalloc(m, theory, k, dV, dout1, dout2, job->ctx->stream, precision);
  });
}

seqx_status seqx_sigma(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* V, double* out1,
                       double* out2, int32_t precision) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    DeviceMolecule& m = scf_mol_of(job, mol);
    if (theory != SEQX_CIS && theory != SEQX_TDHF) throw Error(kEArg, "theory must be CIS or TDHF");
    if (k <= 0 || !V || !out1 || (theory == SEQX_TDHF && !out2)) throw Error(kEArg, "bad sigma arguments");
    check_precision(precision);
    hipStream_t st = job->ctx->stream;
    const size_t n = static_cast<size_t>(k) * m.nocc * m.nvirt;
    DBuf<double> dV(n), d1(n), d2(theory == SEQX_TDHF ? n : 0);
    SEQX_HIP(hipMemcpyAsync(dV.p, V, n * sizeof(double), hipMemcpyHostToDevice, st));
    sigma_build(m, theory, k, dV.p, d1.p, d2.p, job->dw.sig, st, 32, 0, precision);
    d2h(out1, d1.p, n, st);
    if (theory == SEQX_TDHF) d2h(out2, d2.p, n, st);
    SEQX_HIP(hipStreamSynchronize(st));
  });
}

seqx_status seqx_solve(seqx_job* job, const seqx_solve_opts* opts) {
  if (!job || !opts) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    if (opts->theory != SEQX_CIS && opts->theory != SEQX_TDHF) throw Error(kEArg, "theory must be CIS or TDHF");
    check_precision(opts->precision);
    if (opts->guess < SEQX_GUESS_GAP || opts->guess > SEQX_GUESS_GAP_PSPACE) throw Error(kEArg, "unknown guess");
    if (opts->guess == SEQX_GUESS_LEARNED && !job->ctx->mlp.ready)
      throw Error(kEState, "learned guess needs network parameters (seqx_mlp_load, _set_params or _train)");
    hipStream_t st = job->ctx->stream;
    DavOptions d;
    d.theory = opts->theory;
    d.nroots = opts->nroots;
    d.tol = opts->tol > 0 ? opts->tol : 1e-6;
    d.max_iter = opts->max_iter > 0 ? opts->max_iter : 100;
    d.max_sub = opts->max_subspace;
    d.precision = opts->precision;
    if (opts->nguard < 0 || opts->nguard > 64) throw Error(kEArg, "nguard must be in [0, 64]");
    d.nguard = opts->nguard;
    DBuf<double> guess;
    job->solved = false;
    job->stats.n_sigma = 0;
    job->stats.n_sigma_fp64 = 0;
    job->stats.refine_iteration = 0;
    job->stats.fp32_iteration = 0;
    job->stats.n_sigma_bf16x3 = 0;
    for (double& x : job->stats.dav_phase_ms) x = 0.0;
    job->dw.sig.timer.reset();
    job->stats.dav_iterations = 0;
    job->stats.t_sigma_s = 0;
    job->stats.n_history = 0;
    job->stats.t_autotune_s = 0.0;
    job->stats.batched_graph = 0;
    job->stats.batched_sigma_flops = 0.0;
    job->stats.max_subspace_used = 0;
    job->stats.subspace_cap = 0;
    job->stats.n_collapses = 0;
    for (int32_t& x : job->stats.tile_variant) x = 0;
    const bool root_batches = opts->root_batch > 0 && opts->root_batch < opts->nroots;
    if (opts->root_batch < 0) throw Error(kEArg, "root_batch must be >= 0");
    if (root_batches && (opts->batched || opts->guess != SEQX_GUESS_GAP))
      throw Error(kEArg, "root batches run the single-molecule solver from the gap guess");
    if (opts->batched) {
      if (opts->theory != SEQX_CIS) throw Error(kEArg, "batched solve supports CIS only");
      if (opts->guess != SEQX_GUESS_GAP) throw Error(kEArg, "batched solve uses the gap guess");
      if (opts->nguard != 0) throw Error(kEArg, "guard roots need the single-molecule solver");
      std::vector<DeviceMolecule*> ms;
      for (size_t mi = 0; mi < job->mols.size(); ++mi) ms.push_back(&scf_mol_of(job, static_cast<int32_t>(mi)));
      BatchOptions bo;
      bo.nroots = opts->nroots;
      bo.tol = d.tol;
      bo.max_iter = d.max_iter;
      bo.max_sub = opts->max_subspace;
      bo.precision = opts->precision;
      const auto tb = std::chrono::steady_clock::now();
      BatchResult r = batched_cis(ms, bo, job->bw, job->ctx->tune, job->dw.sig, st);
      const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
      for (DeviceMolecule* m : ms) {
        m->hist_t.clear();
        m->hist_omega.clear();
      }
      job->stats.n_sigma = r.n_sigma;
      job->stats.n_sigma_fp64 = opts->precision == SEQX_FP64 ? r.n_sigma : 0;
      job->stats.dav_iterations = r.iterations;
      job->stats.t_sigma_s = r.t_sigma_ms * 1e-3;
      job->stats.t_autotune_s = r.t_autotune_ms * 1e-3;
      job->stats.t_davidson_s = wall - job->stats.t_autotune_s;
      job->stats.batched_graph = r.used_graph ? 1 : 0;
      job->stats.batched_sigma_flops = r.sigma_flops;
      for (int b = 0; b < kNumSizeBuckets; ++b) job->stats.tile_variant[b] = r.variant_of_bucket[b];
      job->solved = true;
      return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (size_t mi = 0; mi < job->mols.size(); ++mi) {
      DeviceMolecule& m = scf_mol_of(job, static_cast<int32_t>(mi));
      const long nov = static_cast<long>(m.nocc) * m.nvirt;
      if (opts->nroots < 1 || opts->nroots > nov) throw Error(kEArg, "nroots must be in [1, nocc*nvirt]");
      if (opts->guess == SEQX_GUESS_LEARNED || opts->guess == SEQX_GUESS_GAP_PSPACE) {
        const int M = static_cast<int>(std::min<long>(nov, opts->pspace > 0 ? opts->pspace : 4L * opts->nroots));
        job->guess_v.ensure(static_cast<size_t>(M) * nov);
        pspace_guess(&job->ctx->mlp, m, M, opts->guess == SEQX_GUESS_LEARNED, job->guess_v.p, job->ctx->mw, st);
        d.guess = job->guess_v.p;
        d.nguess = M;
      } else if (opts->guess == SEQX_GUESS_USER && mi == 0) {
        if (!opts->user_guess || opts->n_user_guess < 1) throw Error(kEArg, "user guess missing");
        guess.alloc(static_cast<size_t>(opts->n_user_guess) * nov);
        SEQX_HIP(hipMemcpyAsync(guess.p, opts->user_guess, guess.n * sizeof(double), hipMemcpyHostToDevice, st));
        d.guess = guess.p;
        d.nguess = opts->n_user_guess;
      } else {
        d.guess = nullptr;
        d.nguess = 0;
      }
      // subspace cap from the memory budget, per molecule: V, (A+B)V, (A-B)V rows of nov doubles
      DavOptions dm = d;
      if (dm.max_sub <= 0) {
        size_t budget = opts->mem_budget_bytes;
        if (budget == 0) {
          size_t fr = 0, tot = 0;
          SEQX_HIP(hipMemGetInfo(&fr, &tot));
          budget = fr * 2 / 5;
        }
        // bytes per basis row: the row and its products in FP64, plus their FP32
        // copies where the low-precision phase keeps an FP32 basis
        const size_t per = static_cast<size_t>(opts->theory == SEQX_TDHF ? 3 : 2) * nov *
                           (sizeof(double) + (davidson_f32_basis(nov, opts->precision) ? sizeof(float) : 0));
        // root batches keep K locked rows (T, and U for TDHF) beside the batch's subspace
        const size_t locked = root_batches ? static_cast<size_t>(opts->theory == SEQX_TDHF ? 2 : 1) *
                                                 opts->nroots * nov * sizeof(double)
                                           : 0;
        const long cap_mem = static_cast<long>((budget > locked ? budget - locked : 0) / std::max<size_t>(per, 1));
        const long kcap = (root_batches ? opts->root_batch : opts->nroots) + opts->nguard;
        dm.max_sub = static_cast<int>(std::max<long>(std::min<long>(cap_mem, 20L * kcap + 40), 1));
      }
      DavResult r = root_batches ? davidson_root_batches(m, dm, opts->root_batch, *job->ctx->ds, job->dw,
                                                         job->lock_t, job->lock_u, st)
                                 : davidson(m, dm, *job->ctx->ds, job->dw, st);
      m.hist_t = r.t_iter;
      m.hist_omega.clear();
      for (const auto& w : r.omega_iter) m.hist_omega.insert(m.hist_omega.end(), w.begin(), w.end());
      job->stats.n_sigma += r.n_sigma;
      job->stats.n_sigma_fp64 += r.n_sigma_fp64;
      job->stats.refine_iteration = std::max(job->stats.refine_iteration, r.refine_iter);
      job->stats.fp32_iteration = std::max(job->stats.fp32_iteration, r.fp32_iter);
      job->stats.n_sigma_bf16x3 += r.n_sigma_bf16x3;
      for (int p = 0; p < kNumDavPhases; ++p) job->stats.dav_phase_ms[p] += r.phase_ms[p];
      job->stats.dav_iterations = std::max(job->stats.dav_iterations, r.iterations);
      job->stats.max_subspace_used = std::max(job->stats.max_subspace_used, r.max_subspace);
      job->stats.subspace_cap = std::max(job->stats.subspace_cap, r.subspace_cap);
      job->stats.n_collapses += r.n_collapses;
      job->stats.t_sigma_s += r.t_sigma_ms * 1e-3;
      if (mi == 0) {
        const int nh = std::min<int>(static_cast<int>(r.t_iter.size()), 64);
        job->stats.n_history = nh;
        for (int i = 0; i < nh; ++i) job->stats.time_to_roots_s[i] = r.t_iter[i];
      }
    }
    job->stats.t_davidson_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    job->solved = true;
  });
}

seqx_status seqx_results(const seqx_job* job, int32_t mol, double* omega_eV, double* X, double* Y, double* f,
                         double* mu) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    if (!job->solved || m.nroots == 0) throw Error(kEState, "no results: call seqx_solve first");
    hipStream_t st = job->ctx->stream;
    const int K = m.nroots;
    const size_t nx = static_cast<size_t>(K) * m.nocc * m.nvirt;
    std::vector<double> om(K);
    d2h(om.data(), m.omega.p, K, st);
    if (X) d2h(X, m.X.p, nx, st);
    if (Y) d2h(Y, m.Y.p, nx, st);
    if (f) d2h(f, m.f.p, K, st);
    if (mu) d2h(mu, m.mu.p, 3 * static_cast<size_t>(K), st);
    SEQX_HIP(hipStreamSynchronize(st));
    if (omega_eV)
      for (int j = 0; j < K; ++j) omega_eV[j] = om[j] * kHartreeEV;
  });
}

namespace {
void check_grid(double sigma_eV, double de_eV, int32_t npts, const double* out) {
  if (!(sigma_eV > 0.0) || !std::isfinite(sigma_eV)) throw Error(kEArg, "sigma must be positive and finite");
  if (!(de_eV > 0.0) || !std::isfinite(de_eV)) throw Error(kEArg, "grid step must be positive and finite");
  if (npts <= 0 || !out) throw Error(kEArg, "bad spectrum grid");
}
}  // namespace

seqx_status seqx_spectrum(const seqx_job* job, int32_t mol, double sigma_eV, double e0_eV, double de_eV,
                          int32_t npts, double* out) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    if (!job->solved || m.nroots == 0) throw Error(kEState, "no roots: call seqx_solve first");
    check_grid(sigma_eV, de_eV, npts, out);
    hipStream_t st = job->ctx->stream;
    DBuf<double> d(static_cast<size_t>(npts));
    broaden(st, m.nroots, m.omega.p, kHartreeEV, m.f.p, sigma_eV, e0_eV, de_eV, npts, d.p);
    d2h(out, d.p, static_cast<size_t>(npts), st);
    SEQX_HIP(hipStreamSynchronize(st));
  });
}

seqx_status seqx_broaden(seqx_ctx* ctx, int32_t K, const double* omega_eV, const double* f, double sigma_eV,
                         double e0_eV, double de_eV, int32_t npts, double* out) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    if (K < 0 || (K > 0 && (!omega_eV || !f))) throw Error(kEArg, "bad line list");
    check_grid(sigma_eV, de_eV, npts, out);
    hipStream_t st = ctx->stream;
    DBuf<double> d(static_cast<size_t>(npts) + 2 * static_cast<size_t>(K));
    double* dw = d.p + npts;
    double* df = dw + K;
    if (K > 0) {
      SEQX_HIP(hipMemcpyAsync(dw, omega_eV, K * sizeof(double), hipMemcpyHostToDevice, st));
      SEQX_HIP(hipMemcpyAsync(df, f, K * sizeof(double), hipMemcpyHostToDevice, st));
    }
    broaden(st, K, dw, 1.0, df, sigma_eV, e0_eV, de_eV, npts, d.p);
    d2h(out, d.p, static_cast<size_t>(npts), st);
    SEQX_HIP(hipStreamSynchronize(st));
  });
}

seqx_status seqx_param_gradient(seqx_job* job, int32_t mol, double* grad, size_t cap, int32_t* zvector_iterations) {
  if (!job) return SEQX_E_ARG;
  static_assert(SEQX_NPARAM == kNumElemParams, "parameter count of the header and the library differ");
  return guarded(job->ctx, [&] {
    DeviceMolecule& m = scf_mol_of(job, mol);
    if (!job->solved || m.nroots == 0) throw Error(kEState, "no roots: call seqx_solve first");
    const size_t need = static_cast<size_t>(m.nroots) * kNumSlots * SEQX_NPARAM;
    if (!grad) throw Error(kEArg, "grad is NULL");
    if (cap < need) throw Error(kEBufSize, "grad holds fewer than nroots * 3 * SEQX_NPARAM values");
    std::vector<double> g(need);
    GradientResult r = param_gradient(m, m.theory, job->ctx->elems, job->ctx->raw, job->dw.sig, job->gw,
                                      job->ctx->stream, g.data());
    std::copy(g.begin(), g.end(), grad);
    if (zvector_iterations) *zvector_iterations = r.zvector_iterations;
  });
}

seqx_status seqx_history(const seqx_job* job, int32_t mol, int32_t cap, int32_t* n_iter, double* t_s,
                         double* omega_eV) {
  if (!job || !n_iter) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = mol_of(job, mol);
    if (!job->solved || m.nroots == 0) throw Error(kEState, "no history: call seqx_solve first");
    const int n = static_cast<int>(m.hist_t.size());
    *n_iter = n;
    if (!t_s && !omega_eV) return;
    if (n > cap) throw Error(kEBufSize, "history longer than cap");
    for (int i = 0; i < n; ++i) {
      if (t_s) t_s[i] = m.hist_t[i];
      if (omega_eV)
        for (int j = 0; j < m.nroots; ++j)
          omega_eV[static_cast<size_t>(i) * m.nroots + j] = m.hist_omega[static_cast<size_t>(i) * m.nroots + j] * kHartreeEV;
    }
  });
}

seqx_status seqx_get_stats(const seqx_job* job, seqx_stats* out) {
  if (!job || !out) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    // fold in sigma builds still pending on the stream (waits for them)
    PhaseTimer& t = const_cast<seqx_job*>(job)->dw.sig.timer;
    t.resolve();
    *out = job->stats;
    for (int p = 0; p < kNumPhases; ++p) {
      out->phase_ms[p] = t.ms[p];
      out->phase_launches[p] = t.launches[p];
      out->phase_flops[p] = t.flops[p];
      out->phase_bytes[p] = t.bytes[p];
    }
  });
}

}  // extern "C"

// ---------------------------------------------------------------- learned starting space

seqx_status seqx_mlp_set_params(seqx_ctx* ctx, const float* params, size_t n) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    if (!params || n != static_cast<size_t>(kNumParams)) throw Error(kEArg, "expected SEQX_MLP_NPARAMS floats");
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(params[i])) throw Error(kEArg, "non-finite network parameter");
    for (int f = 0; f < kNumFeatures; ++f)
      if (!(params[kOffSd + f] > 0.0f)) throw Error(kEArg, "feature scales must be positive");
    ctx->mlp.set(params, ctx->stream);
  });
}

seqx_status seqx_mlp_get_params(const seqx_ctx* ctx, float* out, size_t cap, size_t* needed) {
  if (!ctx) return SEQX_E_ARG;
  seqx_ctx* c = const_cast<seqx_ctx*>(ctx);
  return guarded(c, [&] {
    if (needed) *needed = kNumParams;
    if (!out) return;
    if (cap < static_cast<size_t>(kNumParams)) throw Error(kEBufSize, "parameter buffer too small");
    c->mlp.get(out, c->stream);
  });
}

seqx_status seqx_mlp_save(const seqx_ctx* ctx, const char* path) {
  if (!ctx || !path) return SEQX_E_ARG;
  seqx_ctx* c = const_cast<seqx_ctx*>(ctx);
  return guarded(c, [&] {
    std::vector<float> p(kNumParams);
    c->mlp.get(p.data(), c->stream);
    FILE* f = std::fopen(path, "wb");
    if (!f) throw Error(kEArg, std::string("cannot write ") + path);
    const int32_t cnt = kNumParams;
    const bool ok = std::fwrite("SEQXMLP1", 1, 8, f) == 8 && std::fwrite(&cnt, sizeof(cnt), 1, f) == 1 &&
                    std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    std::fclose(f);
    if (!ok) throw Error(kEArg, std::string("write failed: ") + path);
  });
}

seqx_status seqx_mlp_load(seqx_ctx* ctx, const char* path) {
  if (!ctx || !path) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    FILE* f = std::fopen(path, "rb");
    if (!f) throw Error(kEArg, std::string("cannot read ") + path);
    char tag[8] = {};
    int32_t cnt = 0;
    std::vector<float> p(kNumParams);
    const bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "SEQXMLP1", 8) == 0 &&
                    std::fread(&cnt, sizeof(cnt), 1, f) == 1 && cnt == kNumParams &&
                    std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    std::fclose(f);
    if (!ok) throw Error(kEArg, std::string("not a network parameter file: ") + path);
    ctx->mlp.set(p.data(), ctx->stream);
  });
}

seqx_status seqx_mlp_train(seqx_job* job, const seqx_train_opts* opts, seqx_train_log* log) {
  if (!job || !opts) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    std::vector<DeviceMolecule*> ms;
    for (size_t mi = 0; mi < job->mols.size(); ++mi) ms.push_back(&scf_mol_of(job, static_cast<int32_t>(mi)));
    TrainOptions t;
    t.epochs = opts->epochs > 0 ? opts->epochs : 30;
    t.batch = opts->batch > 0 ? opts->batch : 32;
    t.lr = opts->lr > 0 ? opts->lr : 2e-3;
    t.seed = opts->seed;
    t.init = opts->init != 0;
    TrainLog tl;
    mlp_train(job->ctx->mlp, ms, t, tl, job->ctx->mw, job->ctx->stream);
    if (log) {
      log->n_epochs = static_cast<int32_t>(tl.loss.size());
      log->seconds = tl.seconds;
      for (size_t e = 0; e < tl.loss.size() && e < 256; ++e) log->loss[e] = tl.loss[e];
    }
  });
}

seqx_status seqx_features(const seqx_job* job, int32_t mol, float* out, size_t cap) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = scf_mol_of(job, mol);
    const size_t n = static_cast<size_t>(m.nocc) * m.nvirt * kNumFeatures;
    if (!out || cap < n) throw Error(kEBufSize, "feature buffer too small");
    DBuf<float> d(n);
    mlp_features(m, d.p, job->ctx->mw, job->ctx->stream);
    d2h(out, d.p, n, job->ctx->stream);
    SEQX_HIP(hipStreamSynchronize(job->ctx->stream));
  });
}

seqx_status seqx_mlp_scores(const seqx_job* job, int32_t mol, float* z, size_t cap) {
  if (!job) return SEQX_E_ARG;
  return guarded(job->ctx, [&] {
    const DeviceMolecule& m = scf_mol_of(job, mol);
    const long nov = static_cast<long>(m.nocc) * m.nvirt;
    if (!z || cap < static_cast<size_t>(nov)) throw Error(kEBufSize, "score buffer too small");
    DBuf<float> fe(static_cast<size_t>(nov) * kNumFeatures), dz(nov);
    mlp_features(m, fe.p, job->ctx->mw, job->ctx->stream);
    mlp_scores(job->ctx->mlp, nov, fe.p, dz.p, job->ctx->stream);
    d2h(z, dz.p, nov, job->ctx->stream);
    SEQX_HIP(hipStreamSynchronize(job->ctx->stream));
  });
}

seqx_status seqx_mlp_loss_grad(seqx_ctx* ctx, int64_t npairs, const float* feats, const float* w, int32_t nmol,
                               const int64_t* seg, double* loss, float* grad) {
  if (!ctx) return SEQX_E_ARG;
  return guarded(ctx, [&] {
    if (npairs < 1 || !feats || !w || nmol < 1 || !seg || !grad) throw Error(kEArg, "bad loss arguments");
    hipStream_t st = ctx->stream;
    DBuf<float> df(static_cast<size_t>(npairs) * kNumFeatures), dw(npairs), dg(kNumWeights);
    SEQX_HIP(hipMemcpyAsync(df.p, feats, df.n * sizeof(float), hipMemcpyHostToDevice, st));
    SEQX_HIP(hipMemcpyAsync(dw.p, w, dw.n * sizeof(float), hipMemcpyHostToDevice, st));
    std::vector<long> sg(seg, seg + nmol + 1);
    const double L = mlp_loss_grad(ctx->mlp, npairs, df.p, dw.p, nmol, sg.data(), dg.p, ctx->mw, st);
    d2h(grad, dg.p, kNumWeights, st);
    SEQX_HIP(hipStreamSynchronize(st));
    if (loss) *loss = L;
  });
}
