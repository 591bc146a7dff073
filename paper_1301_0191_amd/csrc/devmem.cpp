// Device memory cache behind DBuf.  A set-up allocates and frees the same
// buffers every time it runs (work arrays, descriptors, factor storage);
// hipFree synchronises the whole device and hipMalloc is slow, so freed
// blocks are kept per (device, stream, rounded size) and handed out again to
// allocations made for the same stream, whose work is ordered after every use
// of the block.  The stream is the one of the handle whose entry point is
// running on this thread (DevStreamScope).  A stream's blocks go back to HIP
// when the last handle on it is destroyed; all blocks go back when an
// allocation fails.
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "common.hpp"

namespace ambddc {

namespace {

struct Key {
  int dev;
  hipStream_t st;
  size_t bytes;
  bool operator<(const Key& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (st != o.st) return st < o.st;
    return bytes < o.bytes;
  }
};

// Pinned staging ring per stream for host-to-device uploads: the host data is
// copied into the ring and the device copy is queued without waiting.  A
// region of the ring is written again only after the stream has been
// synchronised, which happens when the ring wraps.
constexpr size_t STAGE_BYTES = size_t(32) << 20;
struct Stage {
  char* buf = nullptr;
  size_t off = 0;
};

std::mutex g_mu;
std::map<hipStream_t, Stage> g_stage;
std::multimap<Key, void*> g_free;
std::map<hipStream_t, int> g_users;   // live handles per stream
size_t g_cached = 0;
thread_local hipStream_t t_stream = nullptr;

size_t round_bytes(size_t b) {
  const size_t q = b < (size_t(1) << 20) ? 512 : (size_t(1) << 20);
  return (b + q - 1) / q * q;
}

// Frees the cached blocks of one stream (all streams if all_streams).
void release_locked(bool all_streams, hipStream_t st) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto it = g_free.begin(); it != g_free.end();) {
    if (all_streams || it->first.st == st) {
      (void)hipSetDevice(it->first.dev);
      (void)hipFree(it->second);
      g_cached -= it->first.bytes;
      it = g_free.erase(it);
    } else {
      ++it;
    }
  }
  (void)hipSetDevice(cur);
}

}  // namespace

void* dev_malloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  const size_t rb = round_bytes(bytes);
  int dev = 0;
  AMB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_free.find(Key{dev, t_stream, rb});
  if (it != g_free.end()) {
    void* p = it->second;
    g_free.erase(it);
    g_cached -= rb;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, rb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();   // blocks of other streams may still be in use
    release_locked(true, nullptr);
    e = hipMalloc(&p, rb);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(5, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

// The block may still be read or written by work queued on the current
// stream; it is only handed out again for that stream, whose later work is
// ordered after it.
void dev_free(void* p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p);
    return;
  }
  const size_t rb = round_bytes(bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  g_free.emplace(Key{dev, t_stream, rb}, p);
  g_cached += rb;
}

void dev_cache_release() {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_mu);
  release_locked(true, nullptr);
}

DevStreamScope::DevStreamScope(hipStream_t st) : prev_(t_stream) { t_stream = st; }
DevStreamScope::~DevStreamScope() { t_stream = prev_; }

void dev_stream_acquire(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  ++g_users[st];
}

void dev_stream_release(hipStream_t st) {
  (void)hipStreamSynchronize(st);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_users.find(st);
  if (it != g_users.end() && --it->second > 0) return;
  if (it != g_users.end()) g_users.erase(it);
  release_locked(false, st);
  auto sg = g_stage.find(st);
  if (sg != g_stage.end()) {
    if (sg->second.buf) (void)hipHostFree(sg->second.buf);
    g_stage.erase(sg);
  }
}

void upload_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  if (bytes > STAGE_BYTES / 4) {
    // large uploads go directly; the host buffer may be a temporary
    AMB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    AMB_HIP(hipStreamSynchronize(st));
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Stage& sg = g_stage[st];
  if (!sg.buf) AMB_HIP(hipHostMalloc(reinterpret_cast<void**>(&sg.buf), STAGE_BYTES));
  if (sg.off + bytes > STAGE_BYTES) {
    AMB_HIP(hipStreamSynchronize(st));   // every copy out of the ring has completed
    sg.off = 0;
  }
  std::memcpy(sg.buf + sg.off, src, bytes);
  AMB_HIP(hipMemcpyAsync(dst, sg.buf + sg.off, bytes, hipMemcpyHostToDevice, st));
  sg.off = (sg.off + bytes + 255) / 256 * 256;
}

size_t dev_cache_bytes() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_cached;
}

}  // namespace ambddc
