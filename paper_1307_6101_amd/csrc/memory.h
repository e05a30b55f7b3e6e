// Device memory of the library's handles.
//
// By default every array is a hipMalloc of its own.  A handle created with
// a caller-owned workspace carves its arrays out of the caller's bytes
// instead: a first-fit free list over [base, base + capacity) with 256-byte
// granules, selected for the duration of a call on that handle by a
// thread-local scope (WorkspaceScope).  The same allocation sequence run
// against a counting workspace hands out placeholder addresses that nothing
// dereferences and only adds up the sizes: that is how the workspace query
// sizes a handle without a GPU, and why the count equals what the real
// build takes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/ddamg.h"
#include "common.h"

namespace ddamg {

class Workspace {
 public:
  static constexpr size_t ALIGN = 256;
  // carve the caller's [base, base + cap); base must be ALIGN-aligned
  Workspace(void* base, size_t cap) : base_(static_cast<char*>(base)), cap_(cap) {
    free_[0] = cap - cap % ALIGN;
  }
  // a counting workspace: unbounded, hands out no memory
  Workspace() : counting_(true) {}
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;

  bool counting() const { return counting_; }
  size_t peak() const { return peak_; }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_; }

  static size_t round(size_t bytes) { return (bytes + ALIGN - 1) / ALIGN * ALIGN; }

  void* take(size_t bytes) {
    const size_t b = round(bytes);
    if (counting_) {
      const size_t off = used_;
      used_ += b;
      if (used_ > peak_) peak_ = used_;
      // placeholder: distinct, aligned, never dereferenced
      return reinterpret_cast<void*>(uintptr_t(1) << 40 | (off + ALIGN));
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > b) free_[off + b] = len - b;
      used_ += b;
      if (used_ > peak_) peak_ = used_;
      return base_ + off;
    }
    throw Error(DDAMG_ENOMEM, "the workspace (" + std::to_string(cap_) + " bytes, " + std::to_string(cap_ - used_) +
                                  " free) cannot hold a further " + std::to_string(b) + " bytes");
  }

  void give(void* p, size_t bytes) {
    const size_t b = round(bytes);
    used_ -= b;
    if (counting_) return;
    size_t off = static_cast<size_t>(static_cast<char*>(p) - base_), len = b;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  bool counting_ = false;
  std::map<size_t, size_t> free_;   // offset -> length of the free ranges
};

// the workspace new arrays come from on this thread (nullptr: hipMalloc)
inline Workspace*& current_workspace() {
  static thread_local Workspace* w = nullptr;
  return w;
}
inline bool counting_only() {
  const Workspace* w = current_workspace();
  return w && w->counting();
}

struct WorkspaceScope {
  Workspace* prev;
  explicit WorkspaceScope(Workspace* w) : prev(current_workspace()) { current_workspace() = w; }
  ~WorkspaceScope() { current_workspace() = prev; }
  WorkspaceScope(const WorkspaceScope&) = delete;
  WorkspaceScope& operator=(const WorkspaceScope&) = delete;
};

// RAII device array, from the current workspace or from hipMalloc
template <typename E>
struct DevArray {
  E* p = nullptr;
  size_t n = 0;
  Workspace* ws = nullptr;   // where p came from (nullptr: hipMalloc)
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  DevArray(DevArray&& o) noexcept : p(o.p), n(o.n), ws(o.ws) { o.p = nullptr; o.n = 0; o.ws = nullptr; }
  DevArray& operator=(DevArray&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p, n = o.n, ws = o.ws;
      o.p = nullptr, o.n = 0, o.ws = nullptr;
    }
    return *this;
  }
  ~DevArray() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    if (Workspace* w = current_workspace()) {
      p = static_cast<E*>(w->take(count * sizeof(E)));
      ws = w;
    } else if (hipMalloc(&p, count * sizeof(E)) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(DDAMG_ENOMEM, "device allocation of " + std::to_string(count * sizeof(E)) + " bytes failed");
    }
    n = count;
  }
  void upload(const std::vector<E>& v, hipStream_t s) {
    alloc(v.size());
    if (!v.empty() && !(ws && ws->counting()))
      DD_CHECK_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice, s));
  }
  void release() {
    if (p) {
      if (ws) ws->give(p, n * sizeof(E));
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    ws = nullptr;
  }
};

}  // namespace ddamg
