// Declarations of the quadtree-adaptation and split/merge launchers.
#pragma once
#include "pic_internal.hpp"

namespace pic {

constexpr uint32_t kMergeMax = 2048;   // particles of one species in one leaf that a merge round can sort

struct TreeView {
  const uint32_t* key;
  const uint8_t* lv;
  const uint32_t* lut;
  int lut_level;
  uint32_t n;
  int min_level, max_level;
};

__device__ __forceinline__ float prev_toward_zero(float x) { return __int_as_float(__float_as_int(x) - 1); }
__device__ __forceinline__ double prev_toward_zero(double x) {
  return __longlong_as_double(__double_as_longlong(x) - 1ll);
}

uint32_t scan_tmp_words(uint32_t n);
hipError_t launch_scan_u32(uint32_t* a, uint32_t n, uint32_t* tmp, hipStream_t s);   // exclusive; a[n] = total
hipError_t launch_fill_u32(uint32_t* a, uint32_t n, uint32_t v, hipStream_t s);
hipError_t launch_coarsen_flags(const TreeView& t, const uint32_t* cnt, int nspecies, int n_lo, int n_hi,
                                uint32_t* cflag, hipStream_t s);
// emit counts: mode 0 coarsen (cflag) + refine, mode 1 refine only, mode 2 refine marked leaves
hipError_t launch_tree_flags(const TreeView& t, const uint32_t* cnt, int nspecies, int n_hi, int mode,
                             const uint32_t* mark, const uint32_t* cflag, uint32_t* emit, uint32_t* nchanged,
                             hipStream_t s);
hipError_t launch_balance_mark(const TreeView& t, uint32_t* mark, uint32_t* nmark, hipStream_t s);
hipError_t launch_tree_emit(const TreeView& t, const uint32_t* off, const uint32_t* cflag, uint32_t* nkey,
                            uint8_t* nlv, uint32_t* maxlv, hipStream_t s);
template <class T> hipError_t launch_count(const InstDev<T>& I, int sp, uint32_t* cnt, int grid, hipStream_t s);
template <class T> hipError_t launch_split_mark(const InstDev<T>& I, int sp, const uint32_t* cnt, int n_lo,
                                                uint32_t* bitmap, uint32_t* nparents, int grid, hipStream_t s);
hipError_t launch_popc(const uint32_t* bitmap, uint32_t nw, uint32_t* pc, hipStream_t s);
template <class T> hipError_t launch_split_emit(const InstDev<T>& I, int sp, const uint32_t* cnt, int n_lo,
                                                const uint32_t* bitmap, const uint32_t* prefix, uint32_t* cursor,
                                                int grid, hipStream_t s);
hipError_t launch_split_commit(Counters* ctr, const uint32_t* nparents, int nspecies, hipStream_t s);
hipError_t launch_merge_groups(const uint32_t* cnt, uint32_t nleaves, int sp, int n_hi, uint32_t* groups,
                               uint32_t* ngroups, hipStream_t s);
template <class T> hipError_t launch_merge(const InstDev<T>& I, int sp, const uint32_t* groups, uint32_t ngroups,
                                           const uint32_t* cnt, const uint32_t* end_off, int n_hi, uint32_t* flags,
                                           double* energy, uint32_t* npairs, hipStream_t s);

}  // namespace pic
