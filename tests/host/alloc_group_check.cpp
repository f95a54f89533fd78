// Host-only check of ddi::alloc_group (csrc/alloc_group.h), the all-or-nothing allocation of the
// GPE workspace: an allocator that fails at call k (k = 0 .. n) must leave every pointer null and
// every allocated buffer released, and the next attempt with a working allocator must fill all of
// them.  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "../../paper_1504_02897_amd/csrc/alloc_group.h"

int main() {
  constexpr int n = 6;
  for (int fail_at = 0; fail_at <= n; ++fail_at) {
    void* p[n] = {};
    void** ptrs[n];
    size_t bytes[n];
    for (int i = 0; i < n; ++i) {
      ptrs[i] = &p[i];
      bytes[i] = 64 * (i + 1);
    }
    std::set<void*> live;
    int calls = 0;
    auto alloc = [&](void** q, size_t b) {
      if (calls++ == fail_at) return 2;      // an out-of-memory status
      *q = std::malloc(b);
      live.insert(*q);
      return 0;
    };
    auto release = [&](void* q) {
      if (!live.erase(q)) std::abort();        // only what was allocated, once
      std::free(q);
    };
    const int st = ddi::alloc_group(ptrs, bytes, n, alloc, release);
    if (fail_at < n) {
      if (st != 2) { std::printf("fail_at %d: status %d\n", fail_at, st); return 1; }
      for (int i = 0; i < n; ++i)
        if (p[i]) { std::printf("fail_at %d: pointer %d left set\n", fail_at, i); return 1; }
      if (!live.empty()) { std::printf("fail_at %d: %zu buffers leaked\n", fail_at, live.size()); return 1; }
      // a later call (the allocator works again) allocates the whole group
      calls = n + 1;
      if (ddi::alloc_group(ptrs, bytes, n, alloc, release) != 0) return 1;
    } else if (st != 0) {
      std::printf("no failure: status %d\n", st);
      return 1;
    }
    for (int i = 0; i < n; ++i)
      if (!p[i]) { std::printf("fail_at %d: pointer %d not set after success\n", fail_at, i); return 1; }
    if (live.size() != static_cast<size_t>(n)) return 1;
    for (int i = 0; i < n; ++i) release(p[i]);
  }
  std::printf("ok\n");
  return 0;
}
