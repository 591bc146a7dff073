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

// Device memory through a cache of freed blocks (devmem.cpp): dev_free keeps
// the block for later dev_malloc calls of the same rounded size on the same
// device and for the same stream, the one set by the innermost
// DevStreamScope on this thread.  A block may be handed out again while
// earlier work on that stream still uses it; the new owner's work is queued
// after it on the same stream.
void* dev_malloc(size_t bytes);
void dev_free(void* p, size_t bytes);
void dev_cache_release();      // return every cached block to HIP
size_t dev_cache_bytes();
struct DevStreamScope {        // allocations and frees below are for stream st
  explicit DevStreamScope(hipStream_t st);
  ~DevStreamScope();
  DevStreamScope(const DevStreamScope&) = delete;
  DevStreamScope& operator=(const DevStreamScope&) = delete;
 private:
  hipStream_t prev_;
};
void dev_stream_acquire(hipStream_t st);   // a handle starts using st
void dev_stream_release(hipStream_t st);   // ... stops; frees st's cache when unused
// Queues a host-to-device copy on st through pinned staging memory; the host
// buffer may be reused or freed as soon as the call returns.
void upload_async(void* dst, const void* src, size_t bytes, hipStream_t st);

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
    if (p) dev_free(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    p = static_cast<T*>(dev_malloc(count * sizeof(T)));
    n = count;
  }
  void zero(hipStream_t st) {
    if (n) AMB_HIP(hipMemsetAsync(p, 0, n * sizeof(T), st));
  }
  // Same-size uploads keep the allocation, so device pointers taken into the
  // buffer (e.g. per-pair flags referenced by GEMM descriptors) stay valid.
  // The copy is queued on st; the host vector may be a temporary.
  void upload(const std::vector<T>& v, hipStream_t st) {
    if (v.size() != n || !p) alloc(v.size());
    if (n) upload_async(p, v.data(), n * sizeof(T), st);
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

// Timing of selected classes of kernel launches with HIP events recorded on
// the launch stream, with the algorithmic flops and bytes the caller
// attributes to each timed launch.
struct KTimer {
  struct Acc {
    int launches = 0;
    double flops = 0.0, bytes = 0.0, ms = 0.0;
  };
  struct Pending {
    int cls;
    hipEvent_t e0, e1;
  };
  std::vector<std::string> names;
  std::vector<Acc> acc;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pend;
  int cur = -1;
  hipEvent_t cur_e = nullptr;

  int find(const char* cls) const {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == cls) return int(i);
    return -1;
  }
  void enable(const std::string& list) {
    collect();
    names.clear();
    size_t a = 0;
    while (a < list.size()) {
      size_t b = list.find(',', a);
      if (b == std::string::npos) b = list.size();
      if (b > a) names.push_back(list.substr(a, b - a));
      a = b + 1;
    }
    acc.assign(names.size(), Acc());
  }
  bool any() const { return !names.empty(); }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    AMB_HIP(hipEventCreate(&e));
    return e;
  }
  void begin(const char* cls, hipStream_t st) {
    if (names.empty()) return;
    const int i = find(cls);
    if (i < 0) return;
    cur = i;
    cur_e = get();
    AMB_HIP(hipEventRecord(cur_e, st));
  }
  void end(const char* cls, hipStream_t st, double f, double b) {
    if (cur < 0 || names[cur] != cls) return;
    hipEvent_t e = get();
    AMB_HIP(hipEventRecord(e, st));
    pend.push_back({cur, cur_e, e});
    acc[cur].launches += 1;
    acc[cur].flops += f;
    acc[cur].bytes += b;
    cur = -1;
    cur_e = nullptr;
  }
  // correct the work attributed to a class after the fact (for a launch that
  // was recorded before the caller knew its exact work)
  void amend(const char* cls, double df, double db) {
    const int i = find(cls);
    if (i < 0) return;
    acc[i].flops += df;
    acc[i].bytes += db;
  }
  void collect() {
    for (auto& q : pend) {
      AMB_HIP(hipEventSynchronize(q.e1));
      float t = 0.f;
      AMB_HIP(hipEventElapsedTime(&t, q.e0, q.e1));
      if (q.cls < int(acc.size())) acc[q.cls].ms += t;
      pool.push_back(q.e0);
      pool.push_back(q.e1);
    }
    pend.clear();
  }
  ~KTimer() {
    for (auto& q : pend) {
      (void)hipEventDestroy(q.e0);
      (void)hipEventDestroy(q.e1);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace ambddc
