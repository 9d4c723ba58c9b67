// Internal helpers shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "gvt.h"

namespace gvt {

// ---- error reporting ------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

struct Error {
  int code;
  std::string msg;
};

#define GVT_HIP_CHECK(expr)                                                              \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      throw ::gvt::Error{GVT_ERR_HIP,                                                    \
                         std::string(#expr) + ": " + hipGetErrorString(e_)};             \
    }                                                                                    \
  } while (0)

#define GVT_REQUIRE(cond, code, what)                                                    \
  do {                                                                                   \
    if (!(cond)) throw ::gvt::Error{(code), (what)};                                     \
  } while (0)

// Run `body` and convert exceptions into a status code + message.
template <class F> int guarded(F &&body) {
  try {
    clear_error();
    return body();
  } catch (const Error &e) {
    set_error("%s", e.msg.c_str());
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return GVT_ERR_NOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return GVT_ERR_HIP;
  }
}

// ---- device memory ----------------------------------------------------------
// Device blocks for DevMem: released blocks are kept per device for reuse
// (see api.hip); get throws GVT_ERR_NOMEM when the device is full.
void *dev_block_get(size_t want, size_t *got);
void dev_block_put(void *p, size_t got);

struct DevMem {
  void *p = nullptr;
  size_t bytes = 0;
  bool owned = true;  // false: a view into memory owned elsewhere
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  DevMem(DevMem &&o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; }
  DevMem &operator=(DevMem &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; owned = o.owned;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevMem() { release(); }
  void release() {
    if (p && owned) dev_block_put(p, bytes);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  void view(void *ptr, size_t nbytes) {
    release();
    p = ptr;
    bytes = nbytes;
    owned = false;
  }
  // Grow-only; contents are not preserved.  `bytes` is the block's capacity.
  void *ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return p;
    release();
    size_t got = 0;
    p = dev_block_get(nbytes ? nbytes : 256, &got);
    bytes = got;
    return p;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Host-to-device staging for plan data: arrays are collected on the host
// (moved in, not copied) and copied in one transfer through a pinned staging
// buffer into one device allocation (commit), each DevMem becoming a view
// into it.
struct Uploads {
  struct Item {
    DevMem *m;
    std::shared_ptr<void> keep;
    const void *data;
    size_t bytes;
  };
  std::vector<Item> items;
  template <class T> void add(DevMem &m, std::vector<T> &&h) {
    auto sp = std::make_shared<std::vector<T>>(std::move(h));
    items.push_back({&m, sp, sp->data(), sp->size() * sizeof(T)});
  }
  template <class T> void add(DevMem &m, const std::vector<T> &h) {
    add(m, std::vector<T>(h));
  }
  void commit(DevMem &blob);  // synchronous
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Report a failed launch, except while `s` is being captured into a graph
// (the runtime refuses error polling then; the capture itself reports it).
inline void check_launch(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
  GVT_HIP_CHECK(hipGetLastError());
}

}  // namespace gvt
