// Shared definitions of libseqx: errors, device buffers, element data and the
// packed pair-index tables of the NDDO integral layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace seqx {

constexpr double kHartreeEV = 27.211386245988;
constexpr double kBohrAng = 0.529177210903;

// Status values mirror seqx_status in include/seqx.h.
enum Status : int {
  kOK = 0, kEArg = 1, kEElement = 2, kEOpenShell = 3, kEGeometry = 4, kENoMem = 5,
  kEDevice = 6, kEScfNoConv = 7, kEDavNoConv = 8, kEUnstable = 9, kEBufSize = 10, kEState = 11
};

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define SEQX_HIP(call)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw ::seqx::Error(e_ == hipErrorOutOfMemory ? ::seqx::kENoMem : ::seqx::kEDevice,     \
                          std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

#define SEQX_LAUNCH_CHECK() SEQX_HIP(hipGetLastError())

// Caller-provided device allocator (seqx_set_allocator).  The ABI entry
// points make the allocator of their context current for the call; buffers
// remember the allocator that made them and hand their memory back to it.
struct DeviceAllocator {
  void* (*alloc)(size_t bytes, void* user) = nullptr;
  void (*release)(void* ptr, void* user) = nullptr;
  void* user = nullptr;
};
extern thread_local const DeviceAllocator* g_device_allocator;  // nullptr: hipMalloc / hipFree

// Owning device buffer, move-only: hipMalloc / hipFree, or the current
// caller-provided allocator.  Before memory goes back to a caller's allocator
// the device is synchronised, so that a stream-ordered allocator cannot give
// it to other work while kernels of this library may still use it.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  const DeviceAllocator* a = nullptr;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), a(o.a) { o.p = nullptr; o.n = 0; o.a = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; a = o.a; o.p = nullptr; o.n = 0; o.a = nullptr; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    a = g_device_allocator;
    if (a) {
      p = static_cast<T*>(a->alloc(count * sizeof(T), a->user));
      if (!p) throw Error(kENoMem, "caller allocator returned null for " + std::to_string(count * sizeof(T)) + " bytes");
    } else {
      SEQX_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
    }
    n = count;
  }
  // grow-only reallocation; contents are not preserved
  void ensure(size_t count) { if (count > n) alloc(count); }
  void release() {
    if (p) {
      if (a) {
        (void)hipDeviceSynchronize();
        a->release(p, a->user);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = 0;
    a = nullptr;
  }
  operator T*() const { return p; }
  T* get() const { return p; }
};

// Per-element data in atomic units, plain-old-data so it can live on the device.
struct Elem {
  int Z;       // atomic number
  int nao;     // 1 (s) or 4 (s, px, py, pz)
  int n;       // principal quantum number of the valence shell
  int pad;
  double core; // core charge Z' (valence electrons)
  double zs, zp;
  double Uss, Upp, bs, bp;
  double gss, gsp, gpp, gp2, hsp, hpp;
  double D1, D2;           // dipole and quadrupole charge separations (bohr)
  double rho0, rho1, rho2; // additive terms of monopole, dipole, quadrupole (bohr)
};

// Packed index of the same-atom AO pair (mu <= nu), AOs 0=s 1=px 2=py 3=pz:
// ss, s px, s py, s pz, px px, px py, px pz, py py, py pz, pz pz.
__host__ __device__ constexpr int pair_index(int mu, int nu) {
  return mu <= nu ? (mu * 4 - (mu * (mu - 1)) / 2 + (nu - mu)) : (nu * 4 - (nu * (nu - 1)) / 2 + (mu - nu));
}
__host__ __device__ constexpr int pair_first(int P) {
  return P < 4 ? 0 : (P < 7 ? 1 : (P < 9 ? 2 : 3));
}
__host__ __device__ constexpr int pair_second(int P) {
  return P < 4 ? P : (P < 7 ? P - 3 : (P < 9 ? P - 5 : 3));
}

inline size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

}  // namespace seqx
