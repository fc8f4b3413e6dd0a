// Quadtree adaptation to the particle count and particle split/merge
// (arXiv:1604.07713, Sec. 3.1: particles are reassigned by position when
// cells refine or coarsen; Sec. 4.3: splitting one particle into four in 2D,
// merging, AMR holding the particles-per-cell count while particles multiply).
//
// The tree is a Morton-ordered array of leaves (key, level).  Refining a leaf
// replaces it by its four children in Z order, coarsening replaces four
// sibling leaves by their parent, so a flag pass, an exclusive scan of the
// emitted counts and an emit pass rebuild the array in order.  2:1 balance
// (faces and corners) is reached by repeated refinement of leaves that a
// probe one unit outside a finer leaf finds two or more levels coarser.
#include "device_util.hpp"
#include "k_adapt.hpp"
#include "pic_internal.hpp"

namespace pic {

__device__ __forceinline__ uint32_t cnt_max(const uint32_t* cnt, uint32_t nleaves, int nspecies, uint32_t l) {
  uint32_t m = cnt[l];
  if (nspecies > 1 && cnt[nleaves + l] > m) m = cnt[nleaves + l];
  return m;
}

__device__ __forceinline__ void leaf_xyS(const uint32_t* key, const uint8_t* lv, uint32_t l, uint32_t& X,
                                         uint32_t& Y, uint32_t& S) {
  const uint32_t k = key[l];
  uint32_t x = k & 0x55555555u, y = (k >> 1) & 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  y = (y | (y >> 1)) & 0x33333333u;
  y = (y | (y >> 2)) & 0x0F0F0F0Fu;
  y = (y | (y >> 4)) & 0x00FF00FFu;
  y = (y | (y >> 8)) & 0x0000FFFFu;
  X = x;
  Y = y;
  S = 1u << (16 - lv[l]);
}

// ---- particle counts per leaf and species ----
template <class T>
__global__ __launch_bounds__(kBlock) void k_count(InstDev<T> I, int sp, uint32_t* cnt) {
  const uint32_t count = I.ctr->count[sp];
  for (uint32_t base = blockIdx.x * kBlock; base < count; base += gridDim.x * kBlock) {
    const uint32_t i = base + threadIdx.x;
    const bool live = i < count && G(I.w[sp])[i] != 0u;
    (void)seg_atomic_claim(cnt + (size_t)sp * I.nleaves, live ? G(I.cell[sp])[i] : kNoKey);
  }
}

// ---- coarsening decision on the current tree ----
// cflag[l] = 1 if l is the first of four sibling leaves whose parent is
// coarsened: children above min_level, at most n_hi particles of any species
// in the four together, some child below n_lo, and no leaf touching the
// parent finer than the children (probes one unit outside the parent at the
// midpoints of its quarter-sides and at its corners; with a 2:1 tree the only
// such leaves are one level finer than the children).
__global__ void k_coarsen_flags(TreeView t, const uint32_t* __restrict__ cnt, int nspecies, int n_lo, int n_hi,
                                uint32_t* __restrict__ cflag) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t.n) return;
  const int L = t.lv[l];
  uint32_t flag = 0u;
  uint32_t X, Y, S;
  leaf_xyS(t.key, t.lv, l, X, Y, S);
  bool first = L > t.min_level && ((X / S) & 1u) == 0u && ((Y / S) & 1u) == 0u && l + 3u < t.n;
  if (first) {
    const uint32_t step = S * S;   // Morton key distance between siblings
    for (uint32_t k = 1; k < 4; ++k) first = first && t.lv[l + k] == L && t.key[l + k] == t.key[l] + k * step;
  }
  if (first) {
    uint32_t smax = 0, cmin = 0xFFFFFFFFu;
    for (int sp = 0; sp < nspecies; ++sp) {
      uint32_t s = 0;
      for (uint32_t k = 0; k < 4; ++k) s += cnt[(size_t)sp * t.n + l + k];
      smax = s > smax ? s : smax;
    }
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t m = cnt_max(cnt, t.n, nspecies, l + k);
      cmin = m < cmin ? m : cmin;
    }
    if (smax <= (uint32_t)n_hi && cmin < (uint32_t)n_lo) {
      const int PX = (int)X, PY = (int)Y, P2 = 2 * (int)S, q = (int)S / 4, hh = (int)S / 2;
      bool ok = true;
      for (int side = 0; side < 4 && ok; ++side) {
        for (int k = 0; k < 4 && ok; ++k) {
          int px, py;
          const int along = q + k * hh;
          switch (side) {
            case 0: px = PX - 1; py = PY + along; break;
            case 1: px = PX + P2; py = PY + along; break;
            case 2: px = PX + along; py = PY - 1; break;
            default: px = PX + along; py = PY + P2; break;
          }
          if (px < 0 || py < 0 || px >= 65536 || py >= 65536) continue;
          const uint32_t m = locate_leaf(t.key, t.lv, t.lut, t.lut_level, (uint32_t)px, (uint32_t)py);
          if (t.lv[m] > L) ok = false;
        }
      }
      const int cx[4] = {PX - 1, PX + P2, PX - 1, PX + P2};
      const int cy[4] = {PY - 1, PY - 1, PY + P2, PY + P2};
      for (int k = 0; k < 4 && ok; ++k) {
        if (cx[k] < 0 || cy[k] < 0 || cx[k] >= 65536 || cy[k] >= 65536) continue;
        const uint32_t m = locate_leaf(t.key, t.lv, t.lut, t.lut_level, (uint32_t)cx[k], (uint32_t)cy[k]);
        if (t.lv[m] > L) ok = false;
      }
      flag = ok ? 1u : 0u;
    }
  }
  cflag[l] = flag;
}

// index of the first sibling of l's coarsened group, or kNoKey
__device__ __forceinline__ uint32_t coarsened_group(const TreeView& t, const uint32_t* cflag, uint32_t l) {
  if (!cflag) return kNoKey;
  uint32_t X, Y, S;
  leaf_xyS(t.key, t.lv, l, X, Y, S);
  const uint32_t c = ((X / S) & 1u) | (((Y / S) & 1u) << 1);
  if (l < c) return kNoKey;
  return cflag[l - c] ? l - c : kNoKey;
}

// ---- emit count per leaf: 0 (absorbed into a parent), 1 (kept, or the
// first child that becomes the parent) or 4 (refined) ----
__global__ void k_tree_flags(TreeView t, const uint32_t* __restrict__ cnt, int nspecies, int n_hi, int mode,
                             const uint32_t* __restrict__ mark, const uint32_t* __restrict__ cflag,
                             uint32_t* __restrict__ emit, uint32_t* __restrict__ nchanged) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t.n) return;
  uint32_t e = 1u;
  if (mode == 2) {
    e = mark[l] ? 4u : 1u;
  } else {
    const uint32_t g = mode == 0 ? coarsened_group(t, cflag, l) : kNoKey;
    if (g != kNoKey) {
      e = (g == l) ? 1u : 0u;
      if (g == l) atomicAdd(nchanged + 1, 1u);
    } else if (cnt_max(cnt, t.n, nspecies, l) > (uint32_t)n_hi && (int)t.lv[l] < t.max_level) {
      e = 4u;
    }
  }
  emit[l] = e;
  if (e == 4u) atomicAdd(nchanged + 2, 1u);
  if (e != 1u || (mode == 0 && coarsened_group(t, cflag, l) == l)) atomicAdd(nchanged, 1u);
}

// balance probes: mark coarse leaves touched by a leaf two or more levels finer
__global__ void k_balance_mark(TreeView t, uint32_t* __restrict__ mark, uint32_t* __restrict__ nmark) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t.n) return;
  uint32_t X, Y, S;
  leaf_xyS(t.key, t.lv, l, X, Y, S);
  const int L = t.lv[l];
  const int x0 = (int)X, y0 = (int)Y, s = (int)S, h = (int)S / 2;
  const int px[8] = {x0 - 1, x0 + s, x0 + h, x0 + h, x0 - 1, x0 + s, x0 - 1, x0 + s};
  const int py[8] = {y0 + h, y0 + h, y0 - 1, y0 + s, y0 - 1, y0 - 1, y0 + s, y0 + s};
  for (int k = 0; k < 8; ++k) {
    if (px[k] < 0 || py[k] < 0 || px[k] >= 65536 || py[k] >= 65536) continue;
    const uint32_t m = locate_leaf(t.key, t.lv, t.lut, t.lut_level, (uint32_t)px[k], (uint32_t)py[k]);
    if ((int)t.lv[m] < L - 1) {
      if (atomicExch(mark + m, 1u) == 0u) atomicAdd(nmark, 1u);
    }
  }
}

// write the new leaf array from the emit offsets
__global__ void k_tree_emit(TreeView t, const uint32_t* __restrict__ off, const uint32_t* __restrict__ cflag,
                            uint32_t* __restrict__ nkey, uint8_t* __restrict__ nlv, uint32_t* __restrict__ maxlv) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t.n) return;
  const uint32_t e = off[l + 1] - off[l];
  if (e == 0u) return;
  const uint32_t o = off[l];
  const int L = t.lv[l];
  if (e == 1u) {
    const bool parent = cflag && cflag[l];
    const int nl = parent ? L - 1 : L;
    nkey[o] = t.key[l];
    nlv[o] = (uint8_t)nl;
    atomicMax(maxlv, (uint32_t)nl);
    return;
  }
  const uint32_t half = 1u << (16 - L - 1);
  const uint32_t step = half * half;
  for (uint32_t c = 0; c < 4; ++c) {
    nkey[o + c] = t.key[l] + c * step;
    nlv[o + c] = (uint8_t)(L + 1);
  }
  atomicMax(maxlv, (uint32_t)(L + 1));
}

// ---- device-wide exclusive scan of u32 (a[n] receives the total) ----
__global__ __launch_bounds__(1024) void k_scan_tiles(const uint32_t* __restrict__ a, uint32_t n,
                                                     uint32_t* __restrict__ part) {
  __shared__ uint32_t red[16];
  const uint32_t i0 = blockIdx.x * 4096u;
  uint32_t s = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k * 1024u + threadIdx.x;
    if (i < n) s += a[i];
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < 16; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_part(uint32_t* part, uint32_t np) {
  __shared__ uint32_t sh[1024];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < np; b0 += 1024u) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < np ? part[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
      const uint32_t u = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
      __syncthreads();
      sh[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < np) part[i] = carry + sh[threadIdx.x] - v;
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[np] = carry;
}

__global__ __launch_bounds__(1024) void k_scan_apply(uint32_t* a, uint32_t n, const uint32_t* __restrict__ part,
                                                     uint32_t np) {
  __shared__ uint32_t sh[1024];
  const uint32_t i0 = blockIdx.x * 4096u;
  uint32_t carry = part[blockIdx.x];
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k * 1024u + threadIdx.x;
    const uint32_t v = i < n ? a[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
      const uint32_t u = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
      __syncthreads();
      sh[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < n) a[i] = carry + sh[threadIdx.x] - v;
    carry += sh[1023];
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a[n] = part[np];
}

uint32_t scan_tmp_words(uint32_t n) { return ceil_div(n, 4096u) + 2u; }

hipError_t launch_scan_u32(uint32_t* a, uint32_t n, uint32_t* tmp, hipStream_t s) {
  const uint32_t np = ceil_div(n, 4096u) > 0 ? ceil_div(n, 4096u) : 1u;
  hipLaunchKernelGGL(k_scan_tiles, dim3(np), dim3(1024), 0, s, a, n, tmp);
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(1024), 0, s, tmp, np);
  hipLaunchKernelGGL(k_scan_apply, dim3(np), dim3(1024), 0, s, a, n, tmp, np);
  return hipGetLastError();
}

__global__ void k_fill(uint32_t* a, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = v;
}
hipError_t launch_fill_u32(uint32_t* a, uint32_t n, uint32_t v, hipStream_t s) {
  uint32_t g = ceil_div(n, kBlock);
  g = g < 1u ? 1u : (g > 4096u ? 4096u : g);
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(kBlock), 0, s, a, n, v);
  return hipGetLastError();
}

hipError_t launch_coarsen_flags(const TreeView& t, const uint32_t* cnt, int nspecies, int n_lo, int n_hi,
                                uint32_t* cflag, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_flags, dim3(ceil_div(t.n, kBlock)), dim3(kBlock), 0, s, t, cnt, nspecies, n_lo, n_hi,
                     cflag);
  return hipGetLastError();
}
hipError_t launch_tree_flags(const TreeView& t, const uint32_t* cnt, int nspecies, int n_hi, int mode,
                             const uint32_t* mark, const uint32_t* cflag, uint32_t* emit, uint32_t* nchanged,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_tree_flags, dim3(ceil_div(t.n, kBlock)), dim3(kBlock), 0, s, t, cnt, nspecies, n_hi, mode,
                     mark, cflag, emit, nchanged);
  return hipGetLastError();
}
hipError_t launch_balance_mark(const TreeView& t, uint32_t* mark, uint32_t* nmark, hipStream_t s) {
  hipLaunchKernelGGL(k_balance_mark, dim3(ceil_div(t.n, kBlock)), dim3(kBlock), 0, s, t, mark, nmark);
  return hipGetLastError();
}
hipError_t launch_tree_emit(const TreeView& t, const uint32_t* off, const uint32_t* cflag, uint32_t* nkey,
                            uint8_t* nlv, uint32_t* maxlv, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_emit, dim3(ceil_div(t.n, kBlock)), dim3(kBlock), 0, s, t, off, cflag, nkey, nlv, maxlv);
  return hipGetLastError();
}
template <class T>
hipError_t launch_count(const InstDev<T>& I, int sp, uint32_t* cnt, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_count<T>, dim3(grid), dim3(kBlock), 0, s, I, sp, cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Split: in a (leaf, species) holding 0 < n < n_lo particles, every particle
// whose weight is divisible by 4 becomes four copies of a quarter weight at
// the same position and velocity.  The parent keeps its id; the copies get
// next_id + 3r + {0,1,2}, r = rank of the parent id among this round's split
// parents (ranked through a bitmap over the id space).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool split_parent(const InstDev<T>& I, const uint32_t* cnt, int sp, uint32_t i, int n_lo) {
  const uint32_t w = G(I.w[sp])[i];
  if (w == 0u || (w & 3u) != 0u) return false;
  const uint32_t n = cnt[(size_t)sp * I.nleaves + G(I.cell[sp])[i]];
  return n > 0u && n < (uint32_t)n_lo;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_split_mark(InstDev<T> I, int sp, const uint32_t* cnt, int n_lo,
                                                       uint32_t* bitmap, uint32_t* nparents) {
  const uint32_t count = I.ctr->count[sp];
  uint32_t mine = 0;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    if (!split_parent<T>(I, cnt, sp, i, n_lo)) continue;
    const uint32_t id = G(I.id[sp])[i];
    atomicOr(bitmap + (id >> 5), 1u << (id & 31u));
    ++mine;
  }
  mine = wave_sum(mine);
  if (lane_id() == 0 && mine) atomicAdd(nparents + sp, mine);
}

__global__ void k_popc(const uint32_t* bitmap, uint32_t nw, uint32_t* pc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) pc[i] = __popc(bitmap[i]);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_split_emit(InstDev<T> I, int sp, const uint32_t* cnt, int n_lo,
                                                       const uint32_t* bitmap, const uint32_t* prefix,
                                                       uint32_t* cursor) {
  const uint32_t count = I.ctr->count[sp];
  const uint32_t nid = I.ctr->next_id;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    if (!split_parent<T>(I, cnt, sp, i, n_lo)) continue;
    const uint32_t id = G(I.id[sp])[i];
    const uint32_t r = prefix[id >> 5] + __popc(bitmap[id >> 5] & ((1u << (id & 31u)) - 1u));
    const uint32_t w = G(I.w[sp])[i] >> 2;
    const uint32_t slot = count + atomicAdd(cursor + sp, 3u);
    G(I.w[sp])[i] = w;
    const T s0 = G(I.s[sp][0])[i], s1 = G(I.s[sp][1])[i];
    const T v0 = G(I.v[sp][0])[i], v1 = G(I.v[sp][1])[i], v2 = G(I.v[sp][2])[i];
    const uint32_t c = G(I.cell[sp])[i];
    for (uint32_t k = 0; k < 3; ++k) {
      const uint32_t j = slot + k;
      G(I.s[sp][0])[j] = s0;
      G(I.s[sp][1])[j] = s1;
      G(I.v[sp][0])[j] = v0;
      G(I.v[sp][1])[j] = v1;
      G(I.v[sp][2])[j] = v2;
      G(I.w[sp])[j] = w;
      G(I.cell[sp])[j] = c;
      G(I.id[sp])[j] = nid + 3u * r + k;
    }
  }
}

__global__ void k_split_commit(Counters* ctr, const uint32_t* nparents, int nspecies) {
  uint32_t tot = 0;
  for (int sp = 0; sp < nspecies; ++sp) {
    ctr->count[sp] += 3u * nparents[sp];
    tot += nparents[sp];
  }
  ctr->next_id += 3u * tot;
}

template <class T>
hipError_t launch_split_mark(const InstDev<T>& I, int sp, const uint32_t* cnt, int n_lo, uint32_t* bitmap,
                             uint32_t* nparents, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_split_mark<T>, dim3(grid), dim3(kBlock), 0, s, I, sp, cnt, n_lo, bitmap, nparents);
  return hipGetLastError();
}
hipError_t launch_popc(const uint32_t* bitmap, uint32_t nw, uint32_t* pc, hipStream_t s) {
  hipLaunchKernelGGL(k_popc, dim3(ceil_div(nw, kBlock)), dim3(kBlock), 0, s, bitmap, nw, pc);
  return hipGetLastError();
}
template <class T>
hipError_t launch_split_emit(const InstDev<T>& I, int sp, const uint32_t* cnt, int n_lo, const uint32_t* bitmap,
                             const uint32_t* prefix, uint32_t* cursor, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_split_emit<T>, dim3(grid), dim3(kBlock), 0, s, I, sp, cnt, n_lo, bitmap, prefix, cursor);
  return hipGetLastError();
}
hipError_t launch_split_commit(Counters* ctr, const uint32_t* nparents, int nspecies, hipStream_t s) {
  hipLaunchKernelGGL(k_split_commit, dim3(1), dim3(1), 0, s, ctr, nparents, nspecies);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Merge: in a finest-level leaf holding more than n_hi particles of a species,
// sort them by (velocity octant, |v|^2, id), merge pairs (0,1), (2,3), ...:
// w = w1 + w2, s and v the weight-averaged values (FP64, rounded; s clamped
// into the leaf), id = the smaller id.  Particles of a leaf are contiguous
// after the counting sort; one workgroup per leaf sorts them in LDS.
// ---------------------------------------------------------------------------
__global__ void k_merge_groups(const uint32_t* cnt, uint32_t nleaves, int sp, int n_hi, uint32_t* groups,
                               uint32_t* ngroups) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaves) return;
  if (cnt[(size_t)sp * nleaves + l] > (uint32_t)n_hi) groups[atomicAdd(ngroups, 1u)] = l;
}

template <class T>
__device__ __forceinline__ bool merge_less(uint32_t oa, T va, uint32_t ia, uint32_t ob, T vb, uint32_t ib) {
  if (oa != ob) return oa < ob;
  if (va != vb) return va < vb;
  return ia < ib;
}

// One workgroup per leaf runs the merge rounds of that leaf one after the
// other (sort the survivors, merge the pairs) until it holds at most n_hi
// particles or a round merges nothing: the rounds of different leaves are
// independent, so this equals rounds taken over all leaves at once.  A round
// pairs at most kMergeMax / 2 = blockDim particles, one pair per thread.
template <class T>
__global__ __launch_bounds__(1024) void k_merge(InstDev<T> I, int sp, const uint32_t* groups, const uint32_t* cnt,
                                                const uint32_t* end_off, int n_hi, uint32_t* flags, double* energy,
                                                uint32_t* npairs) {
  __shared__ uint32_t soct[kMergeMax];
  __shared__ T sv2[kMergeMax];
  __shared__ uint32_t sid[kMergeMax];
  __shared__ uint32_t sidx[kMergeMax];
  __shared__ uint32_t skipped;
  static_assert(kMergeMax == 2 * 1024, "one pair per thread");
  const uint32_t leaf = groups[blockIdx.x];
  const uint32_t n = cnt[(size_t)sp * I.nleaves + leaf];
  if (n > kMergeMax) {
    if (threadIdx.x == 0) atomicOr(flags, 1u);
    return;
  }
  const uint32_t first = end_off[leaf] - n;
  for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
    const uint32_t i = first + t;
    const T vx = G(I.v[sp][0])[i], vy = G(I.v[sp][1])[i], vz = G(I.v[sp][2])[i];
    soct[t] = (vx < (T)0 ? 1u : 0u) | (vy < (T)0 ? 2u : 0u) | (vz < (T)0 ? 4u : 0u);
    sv2[t] = (vx * vx + vy * vy) + vz * vz;
    sid[t] = G(I.id[sp])[i];
    sidx[t] = i;
  }
  // leaf box for the clamp
  const uint32_t xy = G(I.leaf_xy)[leaf];
  const uint32_t S = 1u << (16 - G(I.leaf_lv)[leaf]);
  const T lo[2] = {(T)(xy >> 16) * (T)1.52587890625e-05, (T)(xy & 0xFFFFu) * (T)1.52587890625e-05};
  const T hi[2] = {(T)((xy >> 16) + S) * (T)1.52587890625e-05, (T)((xy & 0xFFFFu) + S) * (T)1.52587890625e-05};
  double de = 0.0;
  uint32_t pairs = 0;
  uint32_t m = n;   // survivors of the leaf, in sid/soct/sv2/sidx[0, m)
  for (;;) {
    uint32_t np2 = 1;
    while (np2 < m) np2 <<= 1;
    for (uint32_t t = m + threadIdx.x; t < np2; t += blockDim.x) {
      soct[t] = 0xFFFFFFFFu;   // padding sorts last
      sv2[t] = (T)0;
      sid[t] = 0xFFFFFFFFu;
      sidx[t] = 0xFFFFFFFFu;
    }
    if (threadIdx.x == 0) skipped = 0u;
    __syncthreads();
    // bitonic sort on (oct, v2, id)
    for (uint32_t k = 2; k <= np2; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = threadIdx.x; t < np2; t += blockDim.x) {
          const uint32_t p = t ^ j;
          if (p > t) {
            const bool up = (t & k) == 0;
            const bool lt = merge_less<T>(soct[p], sv2[p], sid[p], soct[t], sv2[t], sid[t]);
            if (lt == up) {
              uint32_t a = soct[t]; soct[t] = soct[p]; soct[p] = a;
              T b = sv2[t]; sv2[t] = sv2[p]; sv2[p] = b;
              a = sid[t]; sid[t] = sid[p]; sid[p] = a;
              a = sidx[t]; sidx[t] = sidx[p]; sidx[p] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    // merge pair (2t, 2t+1) in thread t; the survivors' sort keys are kept
    // in registers until every thread has read its pair
    const uint32_t np = m / 2u, t = threadIdx.x;
    bool has = t < np, merged = false;
    uint32_t o1 = 0u, i1 = 0u, x1 = 0u, o2 = 0u, i2 = 0u, x2 = 0u;
    T e1 = (T)0, e2 = (T)0;
    if (has) {
      const uint32_t ia = sidx[2 * t], ib = sidx[2 * t + 1];
      o1 = soct[2 * t]; e1 = sv2[2 * t]; i1 = sid[2 * t]; x1 = ia;
      o2 = soct[2 * t + 1]; e2 = sv2[2 * t + 1]; i2 = sid[2 * t + 1]; x2 = ib;
      const uint32_t wa_u = G(I.w[sp])[ia], wb_u = G(I.w[sp])[ib];
      const uint64_t ws = (uint64_t)wa_u + (uint64_t)wb_u;
      if (ws <= 0xFFFFFFFFull) {
        const double wa = (double)wa_u, wb = (double)wb_u, wt = (double)ws;
        const bool a_keeps = i1 < i2;
        const uint32_t keep = a_keeps ? ia : ib, gone = a_keeps ? ib : ia;
        T ns[2], nv[3];
        for (int c = 0; c < 2; ++c) {
          T x = (T)((wa * (double)G(I.s[sp][c])[ia] + wb * (double)G(I.s[sp][c])[ib]) / wt);
          if (x < lo[c]) x = lo[c];
          if (x >= hi[c]) x = prev_toward_zero(hi[c]);
          ns[c] = x;
        }
        for (int c = 0; c < 3; ++c) nv[c] = (T)((wa * (double)G(I.v[sp][c])[ia] + wb * (double)G(I.v[sp][c])[ib]) / wt);
        const double e_before = wa * (double)e1 + wb * (double)e2;
        G(I.s[sp][0])[keep] = ns[0];
        G(I.s[sp][1])[keep] = ns[1];
        for (int c = 0; c < 3; ++c) G(I.v[sp][c])[keep] = nv[c];
        G(I.w[sp])[keep] = (uint32_t)ws;
        G(I.w[sp])[gone] = 0u;
        const T nv2 = (nv[0] * nv[0] + nv[1] * nv[1]) + nv[2] * nv[2];
        de += wt * (double)nv2 - e_before;
        ++pairs;
        merged = true;
        o1 = (nv[0] < (T)0 ? 1u : 0u) | (nv[1] < (T)0 ? 2u : 0u) | (nv[2] < (T)0 ? 4u : 0u);
        e1 = nv2;
        i1 = a_keeps ? i1 : i2;
        x1 = keep;
      }
    }
    // the odd particle left over keeps its place after the pairs
    const bool odd = (m & 1u) != 0u;
    uint32_t lo_o = 0u, lo_i = 0u, lo_x = 0u;
    T lo_e = (T)0;
    if (odd && t == 0u) {
      lo_o = soct[m - 1u]; lo_e = sv2[m - 1u]; lo_i = sid[m - 1u]; lo_x = sidx[m - 1u];
    }
    __syncthreads();
    if (has) {
      soct[t] = o1; sv2[t] = e1; sid[t] = i1; sidx[t] = x1;
      if (!merged) {
        const uint32_t q = np + (odd ? 1u : 0u) + atomicAdd(&skipped, 1u);
        soct[q] = o2; sv2[q] = e2; sid[q] = i2; sidx[q] = x2;
      }
    }
    if (odd && t == 0u) {
      soct[np] = lo_o; sv2[np] = lo_e; sid[np] = lo_i; sidx[np] = lo_x;
    }
    __syncthreads();
    const uint32_t sk = skipped;
    const uint32_t m2 = np + (odd ? 1u : 0u) + sk;
    __syncthreads();   // every thread has read 'skipped' before the next round resets it
    if (sk == np || m2 <= (uint32_t)n_hi) break;   // nothing merged, or the leaf is within bounds
    m = m2;
  }
  if (pairs) {
    atomicAdd(energy, de);
    atomicAdd(npairs, pairs);
  }
}

template <class T>
hipError_t launch_merge(const InstDev<T>& I, int sp, const uint32_t* groups, uint32_t ngroups, const uint32_t* cnt,
                        const uint32_t* end_off, int n_hi, uint32_t* flags, double* energy, uint32_t* npairs,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_merge<T>, dim3(ngroups), dim3(1024), 0, s, I, sp, groups, cnt, end_off, n_hi, flags, energy,
                     npairs);
  return hipGetLastError();
}
hipError_t launch_merge_groups(const uint32_t* cnt, uint32_t nleaves, int sp, int n_hi, uint32_t* groups,
                               uint32_t* ngroups, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_groups, dim3(ceil_div(nleaves, kBlock)), dim3(kBlock), 0, s, cnt, nleaves, sp, n_hi,
                     groups, ngroups);
  return hipGetLastError();
}

#define PIC_ADAPT_INST(T)                                                                                       \
  template hipError_t launch_count<T>(const InstDev<T>&, int, uint32_t*, int, hipStream_t);                     \
  template hipError_t launch_split_mark<T>(const InstDev<T>&, int, const uint32_t*, int, uint32_t*, uint32_t*,  \
                                           int, hipStream_t);                                                   \
  template hipError_t launch_split_emit<T>(const InstDev<T>&, int, const uint32_t*, int, const uint32_t*,       \
                                           const uint32_t*, uint32_t*, int, hipStream_t);                       \
  template hipError_t launch_merge<T>(const InstDev<T>&, int, const uint32_t*, uint32_t, const uint32_t*,       \
                                      const uint32_t*, int, uint32_t*, double*, uint32_t*, hipStream_t);
PIC_ADAPT_INST(float)
PIC_ADAPT_INST(double)

}  // namespace pic
