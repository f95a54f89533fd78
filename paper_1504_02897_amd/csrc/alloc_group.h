// All-or-nothing allocation of a group of buffers (host logic only, no device code), so that a
// workspace is either wholly present or wholly absent after a failed allocation.
#pragma once

#include <cstddef>

namespace ddi {

// Allocates bytes[i] into *ptrs[i] for i < n with alloc(void**, size_t) -> status (0 = success).
// On the first failure every buffer this call allocated is released with release(void*), every
// *ptrs[i] is left null, and that status is returned.  On success every *ptrs[i] is set and 0 is
// returned.  The pointers must be null on entry.
template <typename Alloc, typename Release>
int alloc_group(void** const* ptrs, const size_t* bytes, int n, Alloc alloc, Release release) {
  for (int i = 0; i < n; ++i) {
    void* p = nullptr;
    const int st = static_cast<int>(alloc(&p, bytes[i]));
    if (st != 0 || p == nullptr) {
      for (int j = 0; j < i; ++j) {
        release(*ptrs[j]);
        *ptrs[j] = nullptr;
      }
      return st != 0 ? st : -1;
    }
    *ptrs[i] = p;
  }
  return 0;
}

}  // namespace ddi
