// Shared host/device helpers for the HIP library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace ambddc {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define AMB_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::ambddc::Error(6, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define AMB_LAUNCH_CHECK() AMB_HIP(hipGetLastError())

// Owning device buffer.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      n = 0;
      (void)hipGetLastError();
      throw Error(5, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
  }
  void zero(hipStream_t st) {
    if (n) AMB_HIP(hipMemsetAsync(p, 0, n * sizeof(T), st));
  }
  // Same-size uploads keep the allocation, so device pointers taken into the
  // buffer (e.g. per-pair flags referenced by GEMM descriptors) stay valid.
  void upload(const std::vector<T>& v, hipStream_t st) {
    if (v.size() != n || !p) alloc(v.size());
    if (n) {
      AMB_HIP(hipMemcpyAsync(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
      AMB_HIP(hipStreamSynchronize(st));   // the host vector may be a temporary
    }
  }
  std::vector<T> download(hipStream_t st) const {
    std::vector<T> v(n);
    if (n) {
      AMB_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, st));
      AMB_HIP(hipStreamSynchronize(st));
    }
    return v;
  }
};

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

}  // namespace ambddc
