// cp_workspace.hpp -- bookkeeping of the library-owned adjoint buffers, one
// per (device, stream).  Plain C++ (no HIP types): the allocator is passed
// in, so the same code runs in the library (hipMalloc / hipFree) and in a
// host-only test of the bookkeeping.
//
// Rules: calls ordered on one stream reuse its buffer, calls on different
// streams or devices never share one; a call that needs more than the
// current buffer gets a new one, and the old one is retired, not freed,
// because a graph captured from an earlier call may still write it; retired
// and current buffers are freed together by release().
#pragma once

#include <cstddef>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

namespace cp {

struct PoolOps {
  int (*alloc)(void** out, size_t bytes);  // 0 on success
  void (*free)(int device, void* ptr);
};

class WorkspacePool {
 public:
  // The buffer of (device, stream) with at least `bytes`; 0 or the
  // allocator's error code.
  int get(int device, const void* stream, size_t bytes, const PoolOps& ops, void** out) {
    std::lock_guard<std::mutex> lk(mu_);
    Buf& b = cur_[{device, stream}];
    if (bytes > b.bytes || !b.ptr) {
      void* p = nullptr;
      const int e = ops.alloc(&p, bytes > 0 ? bytes : 1);
      if (e != 0) return e;
      if (b.ptr) retired_.emplace_back(device, b.ptr);
      b.ptr = p;
      b.bytes = bytes;
    }
    *out = b.ptr;
    return 0;
  }

  // buffers held (current and retired)
  size_t held() {
    std::lock_guard<std::mutex> lk(mu_);
    size_t n = retired_.size();
    for (auto& kv : cur_) n += kv.second.ptr != nullptr;
    return n;
  }

  void release(const PoolOps& ops) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : cur_)
      if (kv.second.ptr) ops.free(kv.first.first, kv.second.ptr);
    for (auto& r : retired_) ops.free(r.first, r.second);
    cur_.clear();
    retired_.clear();
  }

 private:
  struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::mutex mu_;
  std::map<std::pair<int, const void*>, Buf> cur_;
  std::vector<std::pair<int, void*>> retired_;
};

}  // namespace cp
