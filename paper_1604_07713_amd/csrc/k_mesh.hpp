// Declarations of the particle-order (counting sort) launcher.
#pragma once
#include "pic_internal.hpp"

namespace pic {

template <class T>
struct SortDst {
  T *s0, *s1, *v0, *v1, *v2;
  uint32_t *w, *id, *cell;
  T* s2;    // 3D only
  T* acc;   // direct implicit only
};

// One (slot, species) of a batched sort: its offsets (ncell + 1 words, or
// null to skip), its cell count and its destination arrays.
template <class T>
struct SortJob {
  uint32_t* off;
  uint32_t ncell;
  SortDst<T> dst;
};

// Batched sort of many slots: jobs[2 * slot + species], work items as in the
// batched step (slot, species, particle range); every job's species is
// reordered by cell and its count set.
template <class T>
hipError_t launch_sort_batched(const InstDev<T>* insts, const SortJob<T>* jobs, int njobs, uint32_t max_ncell,
                               const WorkItem* items, uint32_t nitems, int grid, hipStream_t s);

// Reorder one species by cell into the arrays of d, dropping holes; the new
// particle count is written to the instance counters.  off: ncell + 1 words;
// tmp: scratch of the multi-block scan (scan_tmp_words(ncell) words) used
// when ncell > 8192, or null.
template <class T>
hipError_t launch_sort(const InstDev<T>& I, int sp, uint32_t ncell, uint32_t* off, uint32_t* tmp, const SortDst<T>& d,
                       int grid, hipStream_t s);

}  // namespace pic
