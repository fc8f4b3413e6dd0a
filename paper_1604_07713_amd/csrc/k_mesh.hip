// Quadtree and particle-order kernels: the locate lookup table, leaf corner
// coordinates, and the counting sort that keeps particles ordered by cell
// (the GPU form of the paper's cell-based particle lists, Sec. 3.1: each
// leaf's particles are a contiguous range of the arrays).
#include "device_util.hpp"
#include "pic_internal.hpp"
#include "k_mesh.hpp"
#include "k_adapt.hpp"

namespace pic {

__device__ __forceinline__ uint32_t compact16(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}

__global__ void k_leaf_xy(const uint32_t* key, uint32_t n, uint32_t* xy) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) xy[l] = (compact16(key[l]) << 16) | compact16(key[l] >> 1);
}

hipError_t launch_leaf_xy(const uint32_t* key, const uint8_t* lv, uint32_t n, uint32_t* xy, hipStream_t s) {
  (void)lv;
  hipLaunchKernelGGL(k_leaf_xy, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, key, n, xy);
  return hipGetLastError();
}

// Cell values carried over to a new tree (the starting guess of the next
// field solve): each new leaf takes the value of the old leaf holding its
// centre.
__global__ void k_remap_cells(const uint32_t* __restrict__ nxy, const uint8_t* __restrict__ nlv, uint32_t n,
                              const uint32_t* okey, const uint8_t* olv, const uint32_t* olut, int olut_level,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  const uint32_t xy = nxy[l];
  const uint32_t half = (1u << (16 - nlv[l])) >> 1;
  dst[l] = src[locate_leaf(okey, olv, olut, olut_level, (xy >> 16) + half, (xy & 0xFFFFu) + half)];
}

hipError_t launch_remap_cells(const uint32_t* nxy, const uint8_t* nlv, uint32_t n, const uint32_t* okey,
                              const uint8_t* olv, const uint32_t* olut, int olut_level, const double* src, double* dst,
                              hipStream_t s) {
  if (n == 0u) return hipSuccess;
  hipLaunchKernelGGL(k_remap_cells, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, nxy, nlv, n, okey, olv, olut,
                     olut_level, src, dst);
  return hipGetLastError();
}

// lut[c] = last leaf whose key <= key of cell c's low corner; lut[4^L] = n
__global__ void k_build_lut(const uint32_t* key, uint32_t n, uint32_t* lut, int L) {
  const uint32_t ncell = 1u << (2 * L);
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncell) return;
  if (c == ncell) {
    lut[c] = n;
    return;
  }
  const uint32_t k = c << (2 * (16 - L));
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (key[mid] <= k) lo = mid; else hi = mid - 1u;
  }
  lut[c] = lo;
}

hipError_t launch_build_lut(const uint32_t* key, const uint8_t* lv, uint32_t n, uint32_t* lut, int L, hipStream_t s) {
  (void)lv;
  hipLaunchKernelGGL(k_build_lut, dim3(ceil_div((1u << (2 * L)) + 1u, kBlock)), dim3(kBlock), 0, s, key, n, lut, L);
  return hipGetLastError();
}

// ---- octree (3D): corner coordinates and lookup table ----
__device__ __forceinline__ uint32_t compact10(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

__global__ void k_leaf_xyz(const uint32_t* key, uint32_t n, uint32_t* xyz) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) xyz[l] = compact10(key[l]) | (compact10(key[l] >> 1) << 10) | (compact10(key[l] >> 2) << 20);
}

hipError_t launch_leaf_xyz(const uint32_t* key, uint32_t n, uint32_t* xyz, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_xyz, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, key, n, xyz);
  return hipGetLastError();
}

// lut[c] = last leaf whose key <= key of level-L cell c's low corner; lut[8^L] = n
__global__ void k_build_lut3(const uint32_t* key, uint32_t n, uint32_t* lut, int L) {
  const uint32_t ncell = 1u << (3 * L);
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncell) return;
  if (c == ncell) {
    lut[c] = n;
    return;
  }
  const uint32_t k = c << (3 * (10 - L));
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (key[mid] <= k) lo = mid; else hi = mid - 1u;
  }
  lut[c] = lo;
}

hipError_t launch_build_lut3(const uint32_t* key, uint32_t n, uint32_t* lut, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_build_lut3, dim3(ceil_div((1u << (3 * L)) + 1u, kBlock)), dim3(kBlock), 0, s, key, n, lut, L);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counting sort of one species by cell (1D: the bin floor(s N) >> sort_shift
// of consecutive cells; 2D and 3D: the leaf), dropping holes.  hist/off has
// ncell + 1 entries (1D: one per bin).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ uint32_t sort_cell(const InstDev<T>& I, int sp, uint32_t i) {
  if (I.dim >= 2) return G(I.cell[sp])[i];
  const T g = G(I.s[sp][0])[i] * (T)I.N;
  int ic = (int)floor(g);
  if (ic > I.N - 1) ic = I.N - 1;
  if (ic < 0) ic = 0;
  return (uint32_t)ic >> I.sort_shift;
}

constexpr uint32_t kSortWin = 1024;

// Base of the LDS window of cells of the particle range [begin, end): the
// window is centred on the median of the cells of three live particles
// sampled at the start, middle and end of the range.  Particles are ordered
// by cell as of the last sort and drift since, and in Morton order a small
// move can change a leaf index a lot; a window anchored on one sample would
// miss the whole range whenever that sample has jumped.  Window slots map to
// cells base + slot.
// The three samples are taken by lanes 0-2 at once (each loads the weight
// and the cell together), then every thread forms the same base after a
// barrier; smp is a three-word LDS array.  Every thread of the workgroup
// calls it.
template <class T>
__device__ __forceinline__ uint32_t sort_window_base(const InstDev<T>& I, int sp, uint32_t begin, uint32_t end,
                                                     uint32_t* smp) {
  if (threadIdx.x < 3u) {
    const uint32_t k = threadIdx.x;
    uint32_t key = kNoKey;
    if (begin < end) {
      const uint32_t at = k == 0u ? begin : k == 1u ? begin + (end - begin) / 2u : end - 1u;
      const uint32_t w = G(I.w[sp])[at];
      const uint32_t c = sort_cell<T>(I, sp, at);
      key = w != 0u ? c : kNoKey;
    }
    smp[k] = key;
  }
  __syncthreads();
  uint32_t c[3];
  int n = 0;
  for (int k = 0; k < 3; ++k)
    if (smp[k] != kNoKey) c[n++] = smp[k];
  uint32_t m = 0u;
  if (n == 1) m = c[0];
  else if (n == 2) m = c[0] < c[1] ? c[0] : c[1];
  else if (n == 3) m = c[0] < c[1] ? (c[1] < c[2] ? c[1] : (c[0] < c[2] ? c[2] : c[0]))
                                   : (c[0] < c[2] ? c[0] : (c[1] < c[2] ? c[2] : c[1]));
  return m > kSortWin / 2u ? m - kSortWin / 2u : 0u;
}

// Histogram of cells over one contiguous range [begin, end) per workgroup,
// pre-aggregated in an LDS window of cells; within a wave, a run of equal
// cells (particles are nearly cell-ordered) costs one atomic.
template <class T>
__device__ void sort_hist_range(const InstDev<T>& I, int sp, uint32_t* hist, uint32_t begin, uint32_t end) {
  __shared__ uint32_t win[kSortWin];
  __shared__ uint32_t smp[3];
  __syncthreads();   // the window may still be read by a previous range
  for (uint32_t j = threadIdx.x; j < kSortWin; j += kBlock) win[j] = 0u;
  const uint32_t base = sort_window_base<T>(I, sp, begin, end, smp);   // (its barrier also orders the zeroing)
  for (uint32_t i0 = begin; i0 < end; i0 += kBlock) {
    const uint32_t i = i0 + threadIdx.x;
    const bool live = i < end && G(I.w[sp])[i] != 0u;
    const uint32_t c = live ? sort_cell<T>(I, sp, i) : 0u;
    const uint32_t o = c - base;
    const bool inwin = live && o < kSortWin;
    (void)lds_seg_claim(win, o, inwin);
    (void)seg_atomic_claim(hist, (live && !inwin) ? c : kNoKey);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < kSortWin; j += kBlock)
    if (win[j]) gadd32(hist + (uint32_t)(base + j), win[j]);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_hist(InstDev<T> I, int sp, uint32_t* hist, uint32_t chunk) {
  const uint32_t count = I.ctr->count[sp];
  const uint32_t begin = blockIdx.x * chunk;
  const uint32_t end = begin + chunk < count ? begin + chunk : count;
  sort_hist_range<T>(I, sp, hist, begin, end);
}

// Single-workgroup exclusive scan of n counts in place; a[n] = total.
__device__ void scan_excl_body(uint32_t* a, uint32_t n) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t chunk = (n + 1023u) / 1024u;
  const uint32_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
  uint32_t s = 0;
  for (uint32_t i = b; i < e; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (uint32_t off = 1; off < 1024u; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;
  for (uint32_t i = b; i < e; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  if (t == 1023u) a[n] = part[1023];
}

__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* a, uint32_t n) { scan_excl_body(a, n); }

// Scatter to the sorted position: per tile of 4 x kBlock particles, slots
// within the tile come from LDS atomics on a window of cells (one per run of
// equal cells in a wave), and one global atomic per touched cell reserves the
// tile's range in that cell; particles outside the window claim their slot
// from the global cursor directly (again one atomic per run).
template <class T>
__device__ void sort_scatter_range(const InstDev<T>& I, int sp, uint32_t* off, uint32_t begin, uint32_t end,
                                   const SortDst<T>& d) {
#ifndef PIC_SORT_SUB
#define PIC_SORT_SUB 4
#endif
  constexpr uint32_t kSub = PIC_SORT_SUB;   // particles per lane per window pass
  __shared__ uint32_t lcnt[kSortWin];
  __shared__ uint32_t gbase[kSortWin];
  __shared__ uint32_t smp[3];
  for (uint32_t t0 = begin; t0 < end; t0 += kSub * kBlock) {
    for (uint32_t j = threadIdx.x; j < kSortWin; j += kBlock) lcnt[j] = 0u;
    // (the sampling's barrier also orders the zeroing)
    const uint32_t base = sort_window_base<T>(I, sp, t0, t0 + kSub * kBlock < end ? t0 + kSub * kBlock : end, smp);
    uint32_t o[kSub], slot[kSub];
    bool live[kSub], inwin[kSub];
#pragma unroll
    for (uint32_t q = 0; q < kSub; ++q) {
      const uint32_t i = t0 + q * kBlock + threadIdx.x;
      live[q] = i < end && G(I.w[sp])[i] != 0u;
      const uint32_t c = live[q] ? sort_cell<T>(I, sp, i) : 0u;
      o[q] = c - base;
      inwin[q] = live[q] && o[q] < kSortWin;
      const uint32_t r = lds_seg_claim(lcnt, o[q], inwin[q]);
      const uint32_t g = seg_atomic_claim(off, (live[q] && !inwin[q]) ? c : kNoKey);
      slot[q] = inwin[q] ? r : g;
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < kSortWin; j += kBlock)
      if (lcnt[j]) gbase[j] = gadd32(off + (uint32_t)(base + j), lcnt[j]);
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kSub; ++q) {
      if (!live[q]) continue;
      const uint32_t i = t0 + q * kBlock + threadIdx.x;
      const uint32_t pos = inwin[q] ? gbase[o[q]] + slot[q] : slot[q];
      G(d.s0)[pos] = G(I.s[sp][0])[i];
      if (I.dim >= 2) {
        G(d.s1)[pos] = G(I.s[sp][1])[i];
        G(d.cell)[pos] = G(I.cell[sp])[i];
      }
      if (I.dim == 3) G(d.s2)[pos] = G(I.s[sp][2])[i];
      if (I.dipic) G(d.acc)[pos] = G(I.acc[sp])[i];
      G(d.v0)[pos] = G(I.v[sp][0])[i];
      G(d.v1)[pos] = G(I.v[sp][1])[i];
      G(d.v2)[pos] = G(I.v[sp][2])[i];
      G(d.w)[pos] = G(I.w[sp])[i];
      G(d.id)[pos] = G(I.id[sp])[i];
    }
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(InstDev<T> I, int sp, uint32_t* off, uint32_t chunk,
                                                         SortDst<T> d) {
  const uint32_t count = I.ctr->count[sp];
  const uint32_t begin = blockIdx.x * chunk;
  const uint32_t end = begin + chunk < count ? begin + chunk : count;
  sort_scatter_range<T>(I, sp, off, begin, end, d);
}

// ---- batched: one launch per phase over (slot, species) jobs ----
// Work items are (slot, species, particle range) as in the batched step;
// job 2 * slot + species holds that species' counters and destination.
template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_fill_batched(const SortJob<T>* jobs) {
  const SortJob<T>& J = jobs[blockIdx.y];
  if (!J.off) return;   // no such species in the slot
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i <= J.ncell; i += gridDim.x * kBlock) J.off[i] = 0u;
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_hist_batched(const InstDev<T>* insts, const SortJob<T>* jobs,
                                                              const WorkItem* items, uint32_t nitems) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const SortJob<T>& J = jobs[2u * wi.inst + wi.species];
    if (!J.off) continue;
    const InstDev<T>& I = insts[wi.inst];
    const uint32_t count = I.ctr->count[wi.species];
    const uint32_t end = wi.end < count ? wi.end : count;
    if (wi.begin < end) sort_hist_range<T>(I, (int)wi.species, J.off, wi.begin, end);
  }
}
template <class T>
__global__ __launch_bounds__(1024) void k_sort_scan_batched(const SortJob<T>* jobs) {
  const SortJob<T>& J = jobs[blockIdx.x];
  if (J.off) scan_excl_body(J.off, J.ncell);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_scatter_batched(const InstDev<T>* insts, const SortJob<T>* jobs,
                                                                 const WorkItem* items, uint32_t nitems) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const SortJob<T>& J = jobs[2u * wi.inst + wi.species];
    if (!J.off) continue;
    const InstDev<T>& I = insts[wi.inst];
    const uint32_t count = I.ctr->count[wi.species];
    const uint32_t end = wi.end < count ? wi.end : count;
    if (wi.begin < end) sort_scatter_range<T>(I, (int)wi.species, J.off, wi.begin, end, J.dst);
  }
}
template <class T>
__global__ void k_sort_count_batched(const InstDev<T>* insts, const SortJob<T>* jobs) {
  const SortJob<T>& J = jobs[blockIdx.x];
  if (threadIdx.x == 0 && J.off) insts[blockIdx.x / 2u].ctr->count[blockIdx.x % 2u] = J.off[J.ncell];
}

__global__ void k_fill_u32(uint32_t* a, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_set_count(Counters* ctr, int sp, const uint32_t* total) { ctr->count[sp] = *total; }

template <class T>
hipError_t launch_sort(const InstDev<T>& I, int sp, uint32_t ncell, uint32_t* off, uint32_t* tmp, const SortDst<T>& d,
                       int grid, hipStream_t s) {
  const uint32_t chunk = (ceil_div(I.cap[sp], (uint32_t)grid) + kBlock - 1) / kBlock * kBlock;
  hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(ncell + 1u, kBlock) < 1024 ? ceil_div(ncell + 1u, kBlock) : 1024),
                     dim3(kBlock), 0, s, off, ncell + 1u, 0u);
  hipLaunchKernelGGL(k_sort_hist<T>, dim3(grid), dim3(kBlock), 0, s, I, sp, off, chunk);
  if (ncell > 8192u && tmp) {
    const hipError_t e = launch_scan_u32(off, ncell, tmp, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, off, ncell);
  }
  hipLaunchKernelGGL(k_sort_scatter<T>, dim3(grid), dim3(kBlock), 0, s, I, sp, off, chunk, d);
  hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, I.ctr, sp, off + ncell);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sort_batched(const InstDev<T>* insts, const SortJob<T>* jobs, int njobs, uint32_t max_ncell,
                               const WorkItem* items, uint32_t nitems, int grid, hipStream_t s) {
  const uint32_t fill_x = ceil_div(max_ncell + 1u, kBlock) < 64u ? ceil_div(max_ncell + 1u, kBlock) : 64u;
  hipLaunchKernelGGL(k_sort_fill_batched<T>, dim3(fill_x, njobs), dim3(kBlock), 0, s, jobs);
  hipLaunchKernelGGL(k_sort_hist_batched<T>, dim3(grid), dim3(kBlock), 0, s, insts, jobs, items, nitems);
  hipLaunchKernelGGL(k_sort_scan_batched<T>, dim3(njobs), dim3(1024), 0, s, jobs);
  hipLaunchKernelGGL(k_sort_scatter_batched<T>, dim3(grid), dim3(kBlock), 0, s, insts, jobs, items, nitems);
  hipLaunchKernelGGL(k_sort_count_batched<T>, dim3(njobs), dim3(64), 0, s, insts, jobs);
  return hipGetLastError();
}

template hipError_t launch_sort_batched<float>(const InstDev<float>*, const SortJob<float>*, int, uint32_t,
                                               const WorkItem*, uint32_t, int, hipStream_t);
template hipError_t launch_sort_batched<double>(const InstDev<double>*, const SortJob<double>*, int, uint32_t,
                                                const WorkItem*, uint32_t, int, hipStream_t);
template hipError_t launch_sort<float>(const InstDev<float>&, int, uint32_t, uint32_t*, uint32_t*,
                                       const SortDst<float>&, int, hipStream_t);
template hipError_t launch_sort<double>(const InstDev<double>&, int, uint32_t, uint32_t*, uint32_t*,
                                        const SortDst<double>&, int, hipStream_t);

}  // namespace pic
