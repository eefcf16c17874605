// Shared host/device helpers of librisp: status handling, device buffers, launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "risp.h"

namespace risp {

// Error raised inside the library and turned into a status at the ABI boundary.
struct Error : std::runtime_error {
  risp_status code;
  Error(risp_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define RISP_HIP(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::risp::Error(e_ == hipErrorOutOfMemory ? RISP_E_NOMEM : RISP_E_HIP,              \
                          std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define RISP_CHECK(cond, code, msg)                                                           \
  do {                                                                                        \
    if (!(cond)) throw ::risp::Error((code), (msg));                                          \
  } while (0)

// Kernel launch error check (does not synchronise).
#define RISP_LAUNCHED() RISP_HIP(hipGetLastError())

// Device bytes held by DevBuf allocations of this process and their high-water mark (pinned host
// buffers are not counted); read through risp_device_usage.
struct DeviceUsage {
  std::atomic<int64_t> live{0}, peak{0};
  void add(int64_t n) {
    const int64_t now = live.fetch_add(n) + n;
    int64_t p = peak.load();
    while (now > p && !peak.compare_exchange_weak(p, now)) {
    }
  }
  void sub(int64_t n) { live.fetch_sub(n); }
};
inline DeviceUsage g_device_usage;

// Owning device allocation (or pinned host allocation, see alloc_pinned).
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), host_(o.host_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; host_ = o.host_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  // pinned host memory mapped into the device address space (kernels read and write it over the
  // host link)
  void alloc_pinned(size_t bytes) {
    release();
    if (bytes == 0) return;
    hipError_t e = hipHostMalloc(&p_, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      p_ = nullptr;
      (void)hipGetLastError();
      throw Error(RISP_E_NOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    n_ = bytes;
    host_ = true;
  }
  bool pinned() const { return host_; }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    hipError_t e = hipMalloc(&p_, bytes);
    if (e != hipSuccess) {
      p_ = nullptr;
      (void)hipGetLastError();
      throw Error(RISP_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    n_ = bytes;
    g_device_usage.add((int64_t)bytes);
  }
  void release() {
    if (p_ && !host_) g_device_usage.sub((int64_t)n_);
    if (p_) (void)(host_ ? hipHostFree(p_) : hipFree(p_));
    p_ = nullptr;
    n_ = 0;
    host_ = false;
  }
  template <typename T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
  bool host_ = false;
};

template <typename T>
inline DevBuf upload(const T* host, size_t n, hipStream_t s) {
  DevBuf b(n * sizeof(T));
  if (n) RISP_HIP(hipMemcpyAsync(b.get(), host, n * sizeof(T), hipMemcpyHostToDevice, s));
  return b;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

using bf16 = __hip_bfloat16;

}  // namespace risp
