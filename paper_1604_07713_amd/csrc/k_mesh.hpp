// Declarations of the particle-order (counting sort) launcher.
#pragma once
#include "pic_internal.hpp"

namespace pic {

template <class T>
struct SortDst {
  T *s0, *s1, *v0, *v1, *v2;
  uint32_t *w, *id, *cell;
};

// Reorder one species by cell into the arrays of d, dropping holes; the new
// particle count is written to the instance counters.  off: ncell + 1 words.
template <class T>
hipError_t launch_sort(const InstDev<T>& I, int sp, uint32_t ncell, uint32_t* off, const SortDst<T>& d, int grid,
                       hipStream_t s);

}  // namespace pic
