// Device helpers for the ES-PIC kernels (gfx950, wave64).
//
//  - Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
//    "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed so that a
//    particle's draws depend only on (seed, instance, particle id, step);
//  - uniform deviates on odd multiples of 2^-24 (exact in FP32 and FP64);
//  - isotropic directions by Marsaglia's (1972) disk rejection;
//  - normal deviates as the Irwin-Hall sum of twelve uniforms minus six;
//  - wave-level segmented reductions that turn a wave's run of equal cell
//    indices into one global atomic (deposits and counting-sort cursors).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// Global-address-space views.  Pointers read from a by-value descriptor lose
// their address space; without these casts every access compiles to a FLAT
// instruction, which also holds the LDS wait counter and serialises LDS
// atomics behind outstanding memory loads.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> G(T* p) { return (gptr<T>)p; }
template <class T>
__device__ __forceinline__ gptr<const T> G(const T* p) { return (gptr<const T>)p; }
// Wave-uniform copy of a pointer (forces it into scalar registers).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t a = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}
// Element i of a global array addressed with a 32-bit byte offset (arrays are
// kept below 4 GiB), so loads and stores use scalar-base + vector-offset form.
template <class T>
__device__ __forceinline__ gptr<T> at(T* base, uint32_t i) {
  return (gptr<T>)((gptr<char>)base + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ gptr<const T> at(const T* base, uint32_t i) {
  return (gptr<const T>)((gptr<const char>)base + i * (uint32_t)sizeof(T));
}
__device__ __forceinline__ void gadd(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_add((gptr<unsigned long long>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t gadd32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add((gptr<uint32_t>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per multiplier gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
}

// Word stream of one particle in one step: blocks with counter (id, step, b, 0).
struct WordStream {
  uint32_t k0, k1, id, step, block;
  uint32_t w0, w1, w2, w3;
  int left;
  __device__ __forceinline__ WordStream(uint32_t key0, uint32_t key1, uint32_t pid, uint32_t n)
      : k0(key0), k1(key1), id(pid), step(n), block(0) {
    gen();
  }
  // The same stream after its first two words were drawn: (a, b) are the
  // remaining words 2 and 3 of block 0.
  __device__ __forceinline__ WordStream(uint32_t key0, uint32_t key1, uint32_t pid, uint32_t n, uint32_t a,
                                        uint32_t b)
      : k0(key0), k1(key1), id(pid), step(n), block(0), w0(a), w1(b), w2(0u), w3(0u), left(2) {}
  __device__ __forceinline__ void gen() {
    w0 = id;
    w1 = step;
    w2 = block;
    w3 = 0u;
    philox4x32_10(w0, w1, w2, w3, k0, k1);
    left = 4;
  }
  __device__ __forceinline__ uint32_t next() {
    if (left == 0) {
      ++block;
      gen();
    }
    const uint32_t r = w0;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    --left;
    return r;
  }
};

template <class T>
__device__ __forceinline__ T unit_uniform(uint32_t r) {
  return (T)(2u * (r >> 9) + 1u) * (T)5.9604644775390625e-08;
}

template <class T>
__device__ __forceinline__ void isotropic(WordStream& ws, T& dx, T& dy, T& dz) {
#pragma unroll 1
  for (int k = 0; k < 32; ++k) {
    const T a = (T)2 * unit_uniform<T>(ws.next()) - (T)1;
    const T b = (T)2 * unit_uniform<T>(ws.next()) - (T)1;
    const T s = a * a + b * b;
    if (s < (T)1) {
      const T t = (T)2 * sqrt((T)1 - s);
      dx = a * t;
      dy = b * t;
      dz = (T)1 - (T)2 * s;
      return;
    }
  }
  dx = (T)0;
  dy = (T)0;
  dz = (T)1;
}

template <class T>
__device__ __forceinline__ T normal12(WordStream& ws) {
  int32_t S = 0;
#pragma unroll 1
  for (int k = 0; k < 12; ++k) S += (int32_t)(2u * (ws.next() >> 9) + 1u);
  return (T)(S - 100663296) * (T)5.9604644775390625e-08;
}

// ---- wave64 helpers -------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanes_le(int lane) {
  return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Lane index of the first lane of this lane's run of equal keys.
__device__ __forceinline__ int run_start(uint32_t key, int lane) {
  const uint32_t kprev = __shfl_up(key, 1u);
  const bool head = (lane == 0) || (kprev != key);
  const uint64_t heads = __ballot(head);
  return 63 - __clzll(heads & lanes_le(lane));
}

__device__ __forceinline__ bool run_tail(uint32_t key, int lane) {
  const uint32_t knext = __shfl_down(key, 1u);
  return (lane == 63) || (knext != key);
}

// Every lane of the wave must call this (no divergence).  Adds val to dst[key]
// with one atomic per run of equal consecutive keys; kNoKey lanes add nothing.
__device__ __forceinline__ void seg_atomic_add(unsigned long long* dst, uint32_t key, unsigned long long val) {
  const int lane = lane_id();
  const int start = run_start(key, lane);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long o = __shfl_up(val, (unsigned)off);
    if (lane - off >= start) val += o;
  }
  if (run_tail(key, lane) && key != kNoKey && val != 0ull) gadd(dst + key, val);
}

// Same for 32-bit counters; returns for each lane its rank in its run and
// the run's base fetched from the atomic (cursor allocation).
__device__ __forceinline__ uint32_t seg_atomic_claim(uint32_t* cursor, uint32_t key) {
  const int lane = lane_id();
  const int start = run_start(key, lane);
  const uint32_t rank = (uint32_t)(lane - start);
  const bool tail = run_tail(key, lane);
  uint32_t base = 0;
  if (tail && key != kNoKey) base = gadd32(cursor + key, rank + 1u);
  // broadcast the base from the tail lane of the run to the whole run
  const uint64_t tails = __ballot(tail);
  const uint64_t above = tails & ~(lanes_le(lane) >> 1);   // tail lanes >= lane
  const int tl = __ffsll((long long)above) - 1;
  base = __shfl(base, tl);
  return base + rank;
}

// LDS version of seg_atomic_claim: for the lanes with valid set, claims
// one slot of counter cnt[o] per lane with one LDS atomic per run of equal
// consecutive o in the wave; returns the lane's slot (counter value before
// its run plus its rank in the run).  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t lds_seg_claim(uint32_t* cnt, uint32_t o, bool valid) {
  const uint32_t key = valid ? o : kNoKey;
  const int lane = lane_id();
  const int start = run_start(key, lane);
  const uint32_t rank = (uint32_t)(lane - start);
  const bool tail = run_tail(key, lane);
  uint32_t base = 0;
  if (tail && key != kNoKey) base = atomicAdd(cnt + key, rank + 1u);
  const uint64_t tails = __ballot(tail);
  const uint64_t above = tails & ~(lanes_le(lane) >> 1);   // tail lanes >= lane
  const int tl = __ffsll((long long)above) - 1;
  base = __shfl(base, tl);
  return base + rank;
}

template <class V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Morton interleave of two 16-bit coordinates (x in even bits).
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__device__ __forceinline__ uint32_t morton2(uint32_t x, uint32_t y) { return spread16(x) | (spread16(y) << 1); }


// Leaf of a Morton-ordered quadtree containing the point (X, Y) given in
// 16-bit units.  lut[c] is the leaf holding the low corner of level-lut_level
// cell c (lut has 4^lut_level + 1 entries, the last = nleaves); when that
// leaf is finer than lut_level, the cell's leaves are lut[c] .. lut[c+1]-1
// and a binary search over their keys finds the last key <= Morton(X, Y).
// lut_direct: no leaf is finer than lut_level, so lut[c] is the answer.
__device__ __forceinline__ uint32_t locate_leaf(const uint32_t* __restrict__ key, const uint8_t* __restrict__ lv,
                                                const uint32_t* __restrict__ lut, int lut_level, uint32_t X,
                                                uint32_t Y, bool lut_direct = false) {
  const int sh = 16 - lut_level;
  const uint32_t c = morton2(X >> sh, Y >> sh);
  uint32_t lo = G(lut)[c];
  if (lut_direct || (int)G(lv)[lo] <= lut_level) return lo;
  uint32_t hi = G(lut)[c + 1] - 1u;
  const uint32_t m = morton2(X, Y);
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (G(key)[mid] <= m) lo = mid; else hi = mid - 1u;
  }
  return lo;
}

// Octree (3D): Morton code of three 10-bit coordinates (x in bits 0, 3, 6,
// ...), and the leaf holding the point (X, Y, Z) in 10-bit units: the lookup
// table at level lut_level gives the leaf holding the table cell's low
// corner; a deeper tree ends in a binary search over the keys of the leaves
// inside the table cell.
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread10(x) | (spread10(y) << 1) | (spread10(z) << 2);
}
__device__ __forceinline__ uint32_t locate_leaf3(const uint32_t* __restrict__ key, const uint8_t* __restrict__ lv,
                                                 const uint32_t* __restrict__ lut, int lut_level, uint32_t X,
                                                 uint32_t Y, uint32_t Z, bool lut_direct = false) {
  const int sh = 10 - lut_level;
  const uint32_t c = morton3(X >> sh, Y >> sh, Z >> sh);
  uint32_t lo = G(lut)[c];
  if (lut_direct || (int)G(lv)[lo] <= lut_level) return lo;
  uint32_t hi = G(lut)[c + 1] - 1u;
  const uint32_t m = morton3(X, Y, Z);
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (G(key)[mid] <= m) lo = mid; else hi = mid - 1u;
  }
  return lo;
}

}  // namespace pic
