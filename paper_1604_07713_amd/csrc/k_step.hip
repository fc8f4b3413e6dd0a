// Particle-loop kernels of the ES-PIC step (arXiv:1604.07713, Sec. 3, 3.1, 4.3):
// gather E at the particle, leapfrog push, wall rule, locate the cell,
// null-collision MCC with ionization births, charge deposit.
//
// One lane per particle.  Particles of a species are stored as structure of
// arrays and kept ordered by cell, so a workgroup's contiguous range of
// particles touches a compact set of cells: its deposits are summed in LDS
// (a window of consecutive cells plus a small hash table) and flushed to
// global memory once per workgroup.  The deposit is integer (64-bit fixed
// point), hence exact and independent of the order in which lanes and
// workgroups add.
#include <algorithm>
#include <atomic>

#include <hip/hip_ext.h>

#include "device_util.hpp"
#include "pic_internal.hpp"

namespace pic {

struct LStat {
  uint32_t alive, absorbed, elastic, ionization, cx, viol, lost;
};

template <class T>
struct BirthRec {
  T ve0, ve1, ve2, vi0, vi1, vi2;
};

// Wall rule on one normalised coordinate.  Returns false if the particle
// leaves the domain (absorbed, or reflected but still outside).  Inside the
// domain it returns at once (a wave with no lane at a wall skips the rest);
// the reflection itself is written with selects.
template <class T>
__device__ __forceinline__ bool wall_rule(bool reflect, T& s, T& v, bool& lost) {
  const bool in0 = s >= (T)0 && s < (T)1;
  if (!reflect) return in0;   // uniform
  if (in0) return true;
  const bool lo = s < (T)0;
  const bool hi = s >= (T)1;
  const T pred1 = (T)1 - (T)(sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16);
  T s2 = lo ? -s : (hi ? (T)2 - s : s);
  s2 = (hi && s2 == (T)1) ? pred1 : s2;
  v = (lo || hi) ? -v : v;
  s = s2;
  const bool in1 = s2 >= (T)0 && s2 < (T)1;
  lost = lost || !in1;
  return in1;
}

// Null-collision MCC of one candidate (v in registers).  collision_kind:
// electron elastic scattering, ionization or a null collision (from u1 = the
// candidate's second word); ions always go on to the charge-exchange test,
// whose partner velocity is needed to decide.  The processes are separate
// functions: elastic scattering runs in place, in the lane of its particle;
// ionization (with its newborn pair) and charge exchange are rarer and
// dearer and run densely from a workgroup queue.  Event counts are kept by
// the callers.
enum : uint32_t { kCollNone = 0u, kCollElastic = 1u, kCollIonize = 2u, kCollCx = 3u };

template <class T>
__device__ __forceinline__ uint32_t collision_kind(const SpeciesK<T>& k, uint32_t r1, T vx, T vy, T vz,
                                                   LStat& st) {
  if (k.mcc != PIC_MCC_ELECTRON) return kCollCx;
  const T u1 = unit_uniform<T>(r1);
  const T v2 = (vx * vx + vy * vy) + vz * vz;
  st.viol += (v2 > k.vmax2) ? 1u : 0u;
  const T vmag = sqrt(v2);
  const T x_el = k.a_el * vmag;
  if (u1 < x_el) return kCollElastic;
  if (v2 >= k.v_iz2 && u1 < x_el + k.a_iz * vmag) return kCollIonize;
  return kCollNone;
}

template <class T>
__device__ __forceinline__ void collide_elastic(const SpeciesK<T>& k, WordStream& ws, T& vx, T& vy, T& vz) {
  const T v2 = (vx * vx + vy * vy) + vz * vz;
  const T vmag = sqrt(v2);
  T dx, dy, dz;
  isotropic<T>(ws, dx, dy, dz);
  const T vd = (vx * dx + vy * dy) + vz * dz;
  T vp2 = v2 - k.mu2 * (v2 - vmag * vd);
  if (vp2 < (T)0) vp2 = (T)0;
  const T vpm = sqrt(vp2);
  vx = vpm * dx;
  vy = vpm * dy;
  vz = vpm * dz;
}

template <class T>
__device__ __forceinline__ void collide_ionize(const SpeciesK<T>& k, WordStream& ws, T& vx, T& vy, T& vz,
                                               BirthRec<T>& rec) {
  const T v2 = (vx * vx + vy * vy) + vz * vz;
  const T u0 = unit_uniform<T>(ws.next());
  const T v2ex = v2 - k.v_iz2;
  const T v2a = u0 * v2ex;
  const T v2b = v2ex - v2a;
  T ax, ay, az, bx, by, bz;
  isotropic<T>(ws, ax, ay, az);
  isotropic<T>(ws, bx, by, bz);
  const T va = sqrt(v2a), vb = sqrt(v2b);
  vx = va * ax;
  vy = va * ay;
  vz = va * az;
  rec.ve0 = vb * bx;
  rec.ve1 = vb * by;
  rec.ve2 = vb * bz;
  rec.vi0 = k.v_thg * normal12<T>(ws);
  rec.vi1 = k.v_thg * normal12<T>(ws);
  rec.vi2 = k.v_thg * normal12<T>(ws);
}

// ion charge exchange with a gas atom drawn from the gas Maxwellian; true
// when it happened
template <class T>
__device__ __forceinline__ bool collide_cx(const SpeciesK<T>& k, uint32_t r1, WordStream& ws, T& vx, T& vy, T& vz,
                                           LStat& st) {
  const T u1 = unit_uniform<T>(r1);
  const T n0 = k.v_thg * normal12<T>(ws);
  const T n1 = k.v_thg * normal12<T>(ws);
  const T n2 = k.v_thg * normal12<T>(ws);
  const T dx = vx - n0, dy = vy - n1, dz = vz - n2;
  const T g = sqrt((dx * dx + dy * dy) + dz * dz);
  st.viol += (g > k.gmax) ? 1u : 0u;
  const bool hit = u1 < k.a_cx * g;
  vx = hit ? n0 : vx;
  vy = hit ? n1 : vy;
  vz = hit ? n2 : vz;
  return hit;
}

// Stage a birth: slot from one atomic per wave.
template <class T>
__device__ __forceinline__ void stage_birth(const InstDev<T>& I, bool birth, uint32_t pid, uint32_t cell, uint32_t w,
                                            T s0, T s1, const BirthRec<T>& rec, T s2 = (T)0) {
  const uint64_t bm = __ballot(birth);
  if (bm == 0ull) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)bm) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(&I.ctr->nbirths, (uint32_t)__popcll(bm));
  base = __shfl(base, leader);
  if (!birth) return;
  const uint32_t slot = base + (uint32_t)__popcll(bm & (lanes_le(lane) >> 1));
  if (slot >= I.birth_cap) {
    atomicOr(&I.ctr->flags, kFlagBirthOverflow);
    return;
  }
  G(I.br.parent)[slot] = pid;
  G(I.br.cell)[slot] = cell;
  G(I.br.w)[slot] = w;
  G(I.br.s[0])[slot] = s0;
  if (I.dim >= 2) G(I.br.s[1])[slot] = s1;
  if (I.dim == 3) G(I.br.s[2])[slot] = s2;
  G(I.br.ve[0])[slot] = rec.ve0;
  G(I.br.ve[1])[slot] = rec.ve1;
  G(I.br.ve[2])[slot] = rec.ve2;
  G(I.br.vi[0])[slot] = rec.vi0;
  G(I.br.vi[1])[slot] = rec.vi1;
  G(I.br.vi[2])[slot] = rec.vi2;
}

template <class T>
struct FixedPoint;
template <>
struct FixedPoint<float> {
  static constexpr int F = 24;
};
template <>
struct FixedPoint<double> {
  static constexpr int F = 32;
};

// the cloud-in-cell gather on the quadtree (defined with its scatter below)
template <class T>
__device__ __forceinline__ void gather_cic(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T& ex, T& ey);

// ---------------------------------------------------------------------------
// Deposit pre-aggregation: each workgroup owns a window of kWin consecutive
// cells in LDS (its particles are a contiguous, cell-ordered range, so their
// cells cluster); deposits inside the window are LDS atomics, the rest go
// straight to global memory, and the window is flushed once per workgroup.
// ---------------------------------------------------------------------------
constexpr uint32_t kWin = 1024;
constexpr uint32_t kHash = 512;      // open-addressed LDS table for cells outside the window
constexpr uint32_t kHashProbe = 8;

struct DepCache {
  unsigned long long* win;     // [kWin]
  uint32_t* hkey;              // [kHash], kNoKey = empty
  unsigned long long* hval;    // [kHash]
  uint32_t base;
};

// The workgroup's deposit window and hash in LDS (one allocation, whichever
// variant of the particle loop a kernel runs).
struct DepLds {
  unsigned long long* win;
  uint32_t* hkey;
  unsigned long long* hval;
  uint32_t* wbase;
};
__device__ __forceinline__ DepLds dep_lds() {
  __shared__ unsigned long long win[kWin];
  __shared__ uint32_t hkey[kHash];
  __shared__ unsigned long long hval[kHash];
  __shared__ uint32_t wbase;
  return DepLds{win, hkey, hval, &wbase};
}

__device__ __forceinline__ void dep_add(DepCache& D, unsigned long long* g, uint32_t key, unsigned long long val) {
  if (key == kNoKey || val == 0ull) return;
  const uint32_t o = key - D.base;
  if (o < kWin) {
    atomicAdd(D.win + o, val);
    return;
  }
  uint32_t h = (key * 2654435761u) >> 23;   // 9 bits
  for (uint32_t p = 0; p < kHashProbe; ++p) {
    const uint32_t slot = (h + p) & (kHash - 1u);
    const uint32_t k = atomicCAS(D.hkey + slot, kNoKey, key);
    if (k == kNoKey || k == key) {
      atomicAdd(D.hval + slot, val);
      return;
    }
  }
  gadd(g + key, val);
}

__device__ __forceinline__ void dep_zero(DepCache& D) {
  for (uint32_t j = threadIdx.x; j < kWin; j += kBlock) D.win[j] = 0ull;
  for (uint32_t j = threadIdx.x; j < kHash; j += kBlock) {
    D.hkey[j] = kNoKey;
    D.hval[j] = 0ull;
  }
}

__device__ __forceinline__ void dep_flush(const DepCache& D, unsigned long long* g, uint32_t nq) {
  for (uint32_t j = threadIdx.x; j < kWin; j += kBlock) {
    const unsigned long long v = D.win[j];
    const uint32_t key = D.base + j;   // the same modular key dep_add used
    if (v && key < nq) gadd(g + key, v);
  }
  for (uint32_t j = threadIdx.x; j < kHash; j += kBlock) {
    const uint32_t k = D.hkey[j];
    if (k != kNoKey && D.hval[j]) gadd(g + k, D.hval[j]);
  }
}

// ---------------------------------------------------------------------------
// 1D: one particle per lane
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ uint32_t cell1d(const InstDev<T>& I, T s) {
  const T g = s * (T)I.N;
  int ic = (int)floor(g);
  if (ic > I.N - 1) ic = I.N - 1;
  return (uint32_t)ic;
}

// Wave-uniform pointers of one species' arrays.
template <class T>
struct SpPtr {
  T *s0, *s1, *v0, *v1, *v2;
  uint32_t *w, *id, *cell;
};
template <class T>
__device__ __forceinline__ SpPtr<T> species_ptrs(const InstDev<T>& I, int sp) {
  SpPtr<T> p;
  p.s0 = uniform_ptr(I.s[sp][0]);
  p.s1 = uniform_ptr(I.s[sp][1]);
  p.v0 = uniform_ptr(I.v[sp][0]);
  p.v1 = uniform_ptr(I.v[sp][1]);
  p.v2 = uniform_ptr(I.v[sp][2]);
  p.w = uniform_ptr(I.w[sp]);
  p.id = uniform_ptr(I.id[sp]);
  p.cell = uniform_ptr(I.cell[sp]);
  return p;
}

// Full batches store weight and leaf for every lane too (branch-free) when
// set, else only where they changed (absorbed / moved).
#ifndef PIC_FULL_WC
#define PIC_FULL_WC 0
#endif
constexpr bool kFullWC = PIC_FULL_WC != 0;

// Per-species constants and table pointers of the hot loop, copied into
// registers once per workgroup (the loop's compiler fences would otherwise
// make every batch reload them from the kernel arguments).
template <class T>
struct HotK {
  const T* E;
  const uint32_t* leaf_xy;
  const uint8_t* leaf_lv;
  const uint32_t* lut;
  int N, lut_level;
  bool reflect;
  bool cell_e;   // 1D energy-conserving coupling: the cell's E, no interpolation
  uint32_t nq, key0, key1;
  SpeciesK<T> k;
};
template <class T>
__device__ __forceinline__ HotK<T> hot_constants(const InstDev<T>& I, int sp) {
  HotK<T> h;
  h.E = uniform_ptr(I.E);
  h.leaf_xy = uniform_ptr(I.leaf_xy);
  h.leaf_lv = uniform_ptr(I.leaf_lv);
  h.lut = uniform_ptr(I.lut);
  h.N = I.N;
  h.lut_level = I.lut_level;
  h.reflect = I.particle_bc == PIC_REFLECT;
  h.cell_e = I.cell_e != 0;
  h.nq = I.nq;
  h.key0 = I.key0;
  h.key1 = I.key1;
  h.k = I.sk[sp];
  return h;
}

// Particle state of one lane.  A workgroup walks its contiguous range in
// batches of K particles per lane.  Vector memory operations of a wave retire
// in issue order, so a wait for any load also waits for everything issued
// before it; the batch loop therefore issues its loads in the order they are
// needed and keeps every load outside data-dependent branches (loads index
// element min(i, end - 1) and lanes past the end become holes), which keeps
// the wait counts exact:
//   1. field at the particles of batch t (leaf corners / node values);
//   2. stage A of batch t+1: weight, leaf (2D) or position (1D), id;
//   3. push and wall rule of batch t;
//   4. point location of the particles that left their leaf (lookup table);
//   5. collision candidate test; the velocity components the push does not
//      use, for the candidates (1D; the 2D collision loop takes v_z with
//      stage B);
//   6. stage B of batch t+1: the rest of the particle state;
//   7. collisions, births, stores and deposit of batch t.
// Stage B of batch t+1 thus overlaps the locate and collision round trips of
// batch t, and stage A overlaps the push.
// Compiler-only fence: loads issued above it stay above it (they are not sunk
// into the branches that use them), without waiting for their data, and no
// instruction is scheduled across it (arithmetic on a load's result hoisted
// above later loads would make those loads wait for it).
__device__ __forceinline__ void issue_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <class T>
struct PState {
  uint32_t w, cell, id;
  T s0, s1, v0, v1, v2;
};

// 2D collision loop: v_z of every particle is prefetched with the rest of
// its state (else loaded for the collision candidates only).
#ifndef PIC_VZ_PRE
#define PIC_VZ_PRE 1
#endif
constexpr bool kVzPre = PIC_VZ_PRE != 0;

template <class T, bool MCC, int DIM>
__device__ __forceinline__ void load_a(const SpPtr<T>& P, uint32_t i, uint32_t end, PState<T>& p) {
  const uint32_t ii = i < end ? i : end - 1u;
  const uint32_t w = *at(P.w, ii);
  if (DIM == 2) p.cell = *at(P.cell, ii);
  else p.s0 = *at(P.s0, ii);
  p.id = MCC ? *at(P.id, ii) : 0u;
  p.w = i < end ? w : 0u;
}
template <class T, bool MCC, int DIM>
__device__ __forceinline__ void load_b(const SpPtr<T>& P, uint32_t i, uint32_t end, PState<T>& p) {
  const uint32_t ii = i < end ? i : end - 1u;
  if (DIM == 2) {
    p.s0 = *at(P.s0, ii);
    p.s1 = *at(P.s1, ii);
    p.v1 = *at(P.v1, ii);
    if (MCC && kVzPre) p.v2 = *at(P.v2, ii);
  } else {
    p.cell = 0u;
    p.s1 = (T)0;
    p.v1 = (T)0;
  }
  p.v0 = *at(P.v0, ii);
}

// Field data at one particle: the two node values around it (1D) or the
// leaf's corner coordinates, level and corner E (2D).
template <class T, int DIM>
struct FieldAt;
template <class T>
struct FieldAt<T, 1> {
  T e0, e1;
};
template <class T>
struct FieldAt<T, 2> {
  uint32_t xy;
  int lv;
  T c[8];
};

template <class T>
__device__ __forceinline__ uint32_t cell1d_h(const HotK<T>& H, T s) {
  const T g = s * (T)H.N;
  int ic = (int)floor(g);
  if (ic > H.N - 1) ic = H.N - 1;
  return (uint32_t)ic;
}
template <class T>
__device__ __forceinline__ void fetch_field(const HotK<T>& H, const PState<T>& p, FieldAt<T, 1>& f) {
  const uint32_t ic = cell1d_h<T>(H, p.w ? p.s0 : (T)0);
  f.e0 = *at(H.E, ic);
  f.e1 = *at(H.E, ic + 1u);
}
template <class T>
__device__ __forceinline__ void fetch_leaf(const InstDev<T>& I, uint32_t leaf, FieldAt<T, 2>& f) {
  f.xy = *at(I.leaf_xy, leaf);
  f.lv = *at(I.leaf_lv, leaf);
  const gptr<const T> c = at(I.E, leaf * 8u);
#pragma unroll
  for (int q = 0; q < 8; ++q) f.c[q] = c[q];
}
template <class T>
__device__ __forceinline__ void fetch_field(const HotK<T>& H, const PState<T>& p, FieldAt<T, 2>& f) {
  const uint32_t leaf = p.w ? p.cell : 0u;
  f.xy = *at(H.leaf_xy, leaf);
  f.lv = *at(H.leaf_lv, leaf);
  const gptr<const T> c = at(H.E, leaf * 8u);
#pragma unroll
  for (int q = 0; q < 8; ++q) f.c[q] = c[q];
}

// Bilinear interpolation of the leaf's corner E (corners SW, SE, NW, NE).
template <class T>
__device__ __forceinline__ void interp2d(const FieldAt<T, 2>& f, T sx, T sy, T& ex, T& ey) {
  const int sh = kKeyBits - f.lv;
  const T sc = (T)(1u << f.lv);
  const T xi = sx * sc - (T)((f.xy >> 16) >> sh);
  const T eta = sy * sc - (T)((f.xy & 0xFFFFu) >> sh);
  const T w00 = ((T)1 - xi) * ((T)1 - eta);
  const T w10 = xi * ((T)1 - eta);
  const T w01 = ((T)1 - xi) * eta;
  const T w11 = xi * eta;
  ex = ((w00 * f.c[0] + w10 * f.c[2]) + w01 * f.c[4]) + w11 * f.c[6];
  ey = ((w00 * f.c[1] + w10 * f.c[3]) + w01 * f.c[5]) + w11 * f.c[7];
}

template <class T>
__device__ __forceinline__ void gather2d(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T& ex, T& ey) {
  FieldAt<T, 2> f;
  fetch_leaf<T>(I, leaf, f);
  interp2d<T>(f, sx, sy, ex, ey);
}

template <class T>
__device__ __forceinline__ uint32_t locate2d(const InstDev<T>& I, uint32_t X, uint32_t Y) {
  return locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, X, Y, I.lut_direct != 0);
}

// Gather, leapfrog push and wall rule of one particle, evaluated for every
// lane (holes and lanes past the end compute and discard).  An absorbed
// particle becomes a hole (w = 0; stored at once in a partial batch, with
// the other stores in a full one).  Returns true when a live
// 2D particle has left its leaf and must be located.
template <class T, int DIM, bool FULL>
__device__ __forceinline__ bool push_one(const HotK<T>& H, const SpPtr<T>& P, uint32_t i, PState<T>& p,
                                         const FieldAt<T, DIM>& f, LStat& st) {
  const SpeciesK<T>& k = H.k;
  const bool alive = p.w != 0u;
  bool ok;
  bool lost = false;
  if constexpr (DIM == 1) {
    const T g = p.s0 * (T)H.N;
    int ic = (int)floor(g);
    if (ic > H.N - 1) ic = H.N - 1;
    const T fr = g - (T)ic;
    const T E = H.cell_e ? f.e0 : f.e0 + fr * (f.e1 - f.e0);   // uniform over the launch
    p.v0 = p.v0 + k.qm_dt * E;
    p.s0 = p.s0 + p.v0 * k.dt_L;
    ok = wall_rule<T>(H.reflect, p.s0, p.v0, lost);
  } else {
    T ex, ey;
    interp2d<T>(f, p.s0, p.s1, ex, ey);
    p.v0 = p.v0 + k.qm_dt * ex;
    p.v1 = p.v1 + k.qm_dt * ey;
    p.s0 = p.s0 + p.v0 * k.dt_L;
    p.s1 = p.s1 + p.v1 * k.dt_L;
    const bool okx = wall_rule<T>(H.reflect, p.s0, p.v0, lost);
    const bool oky = wall_rule<T>(H.reflect, p.s1, p.v1, lost);
    ok = okx && oky;
  }
  const bool absorbed = alive && !ok;
  st.alive += alive ? 1u : 0u;
  st.absorbed += absorbed ? 1u : 0u;
  st.lost += (absorbed && lost) ? 1u : 0u;
  if ((!FULL || !kFullWC) && absorbed) *at(P.w, i) = 0u;   // else stored with the rest
  p.w = ok ? p.w : 0u;
  if constexpr (DIM == 1) {
    return false;
  } else {
    const uint32_t X = (uint32_t)(p.s0 * (T)65536);
    const uint32_t Y = (uint32_t)(p.s1 * (T)65536);
    const int sh = kKeyBits - f.lv;
    const bool left = (X >> sh) != ((f.xy >> 16) >> sh) || (Y >> sh) != ((f.xy & 0xFFFFu) >> sh);
    return p.w != 0u && left;
  }
}

// Candidate test result of one particle: the second word of its stream, the
// two words left in block 0, and the velocity components the push does not
// load (v_z; v_y too in 1D), fetched for candidates only.
template <class T>
struct CollIn {
  bool cand;
  uint32_t r1, wa, wb;
  T vy, vz;
};

// Ionizations and charge exchanges of a workgroup wait in an LDS queue and
// are handled densely (consecutive lanes take consecutive entries), so the
// lanes of a wave that do not take part do not pay for the long draws of the
// few that do.  The queue is drained once it holds kQDrain entries after a
// batch, and at the end of the range; a batch adds at most K x kBlock.
constexpr uint32_t kQDrain = 64;
// capacity for K particles per lane: what is left below kQDrain plus a batch
template <int K>
constexpr uint32_t q_cap() {
  return kQDrain + (uint32_t)K * kBlock;
}

// An entry holds the process, the particle's index and its draws so far;
// the drain reads the particle's state back from its arrays, where the
// batch has stored it (its position, velocity after the push, weight, id
// and leaf), so the queue stays small enough in LDS for one more workgroup
// per compute unit.
template <class T, int DIM>
struct CollQueue {
  uint32_t* n;
  uint32_t *kind, *i, *r1, *wa, *wb;
};
template <class T, int DIM, int K>
__device__ __forceinline__ CollQueue<T, DIM> coll_queue() {
  constexpr uint32_t kQCap = q_cap<K>();
  __shared__ uint32_t qn;
  __shared__ uint32_t qkind[kQCap], qi[kQCap], qr1[kQCap], qwa[kQCap], qwb[kQCap];
  CollQueue<T, DIM> q;
  q.n = &qn;
  q.kind = qkind;
  q.i = qi;
  q.r1 = qr1;
  q.wa = qwa;
  q.wb = qwb;
  return q;
}

// Run the queued ionizations and charge exchanges, one per lane: write the
// velocities, stage the births and add the newborn pairs' charge.  Empties
// the queue.  Every lane of the workgroup calls it.
template <class T, int DIM>
__device__ __forceinline__ void drain_queue(const InstDev<T>& I, const HotK<T>& H, const SpPtr<T>& P, int sp,
                                         uint32_t step, const CollQueue<T, DIM>& Q, unsigned long long* Qpar,
                                         DepCache& D, LStat& st) {
  const uint32_t n = *Q.n;
#pragma unroll 1
  for (uint32_t t0 = 0; t0 < n; t0 += kBlock) {
    const uint32_t t = t0 + threadIdx.x;
    bool birth = false;
    BirthRec<T> rec;
    uint32_t id = 0u, w = 0u, leaf = 0u;
    T s0 = (T)0, s1 = (T)0;
    if (t < n) {
      const uint32_t kind = Q.kind[t], i = Q.i[t];
      id = *at(P.id, i);
      w = *at(P.w, i);
      s0 = *at(P.s0, i);
      if constexpr (DIM == 2) {
        s1 = *at(P.s1, i);
        leaf = *at(P.cell, i);
      }
      T vx = *at(P.v0, i), vy = *at(P.v1, i), vz = *at(P.v2, i);
      WordStream ws(H.key0, H.key1, id, step, Q.wa[t], Q.wb[t]);
      if (kind == kCollIonize) {
        collide_ionize<T>(H.k, ws, vx, vy, vz, rec);
        birth = true;
        st.ionization++;
      } else {
        st.cx += collide_cx<T>(H.k, Q.r1[t], ws, vx, vy, vz, st) ? 1u : 0u;
      }
      *at(P.v0, i) = vx;
      *at(P.v1, i) = vy;
      *at(P.v2, i) = vz;
    }
    stage_birth<T>(I, birth, id, leaf, w, s0, s1, rec);
    if (birth) {   // the newborn electron and ion sit on the parent
      unsigned long long* Qs = Qpar + (size_t)sp * H.nq;
      unsigned long long* Qi = Qpar + H.nq;
      const unsigned long long ww = w;
      if constexpr (DIM == 2) {
        dep_add(D, Qs, leaf, ww);
        gadd(Qi + leaf, ww);
      } else {
        const T g = s0 * (T)H.N;
        int ic = (int)floor(g);
        if (ic > H.N - 1) ic = H.N - 1;
        const T fr = g - (T)ic;
        const unsigned long long r = (unsigned long long)(long long)rint(fr * (T)(1ull << FixedPoint<T>::F));
        const unsigned long long one = 1ull << FixedPoint<T>::F;
        dep_add(D, Qs, (uint32_t)ic, ww * (one - r));
        dep_add(D, Qs, (uint32_t)ic + 1u, ww * r);
        if (one - r) gadd(Qi + ic, ww * (one - r));
        if (r) gadd(Qi + ic + 1, ww * r);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *Q.n = 0u;
  __syncthreads();
}

// One batch of K particles per lane (stages 1-7 above).  DIRECT: the lookup
// table alone locates a point (no leaf is finer than its level).  FULL: every
// lane of the batch holds a slot of the workgroup's range, so the state is
// stored without a branch, holes included (a hole's position and velocity
// are never read; its leaf stays a valid index); the stores of a partial
// batch are masked by liveness.  Stores that depend on data (collision
// velocities, a partial batch) come after every load of the batch, so they
// do not disturb the exact wait counts of the loads.
template <class T, bool MCC, int DIM, int K, bool DIRECT, bool FULL>
__device__ __forceinline__ void process_batch(const InstDev<T>& I, const HotK<T>& H, const SpPtr<T>& P, int sp, uint32_t i0,
                                              PState<T> (&p)[K], PState<T> (&nxt)[K], uint32_t end, uint32_t step,
                                              unsigned long long* Qpar, DepCache& D, LStat& st,
                                              const CollQueue<T, DIM>& Q) {
  const SpeciesK<T>& k = H.k;
  const bool mcc = MCC && k.mcc != PIC_MCC_NONE;
  const uint32_t inext0 = i0 + (uint32_t)K * kBlock;
  // 1. field at the particles
  FieldAt<T, DIM> f[K];
#pragma unroll
  for (int j = 0; j < K; ++j) fetch_field<T>(H, p[j], f[j]);
  // 2. stage A of the next batch
#pragma unroll
  for (int j = 0; j < K; ++j) load_a<T, MCC, DIM>(P, inext0 + (uint32_t)j * kBlock, end, nxt[j]);
  issue_fence();
  // 3. push
  bool moved[K];
#pragma unroll
  for (int j = 0; j < K; ++j) moved[j] = push_one<T, DIM, FULL>(H, P, i0 + (uint32_t)j * kBlock, p[j], f[j], st);
  // 4. locate
  uint32_t leaf[K];
#pragma unroll
  for (int j = 0; j < K; ++j) leaf[j] = p[j].cell;
  if constexpr (DIM == 2) {
    if constexpr (DIRECT) {
      const int sh = kKeyBits - H.lut_level;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t X = moved[j] ? (uint32_t)(p[j].s0 * (T)65536) : 0u;
        const uint32_t Y = moved[j] ? (uint32_t)(p[j].s1 * (T)65536) : 0u;
        leaf[j] = *at(H.lut, morton2(X >> sh, Y >> sh));
      }
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (moved[j]) leaf[j] = locate2d<T>(I, (uint32_t)(p[j].s0 * (T)65536), (uint32_t)(p[j].s1 * (T)65536));
    }
  }
  // 5. collision candidates and their velocity components (a lane that is
  // not a candidate reads the wave's first element instead, so the load is
  // issued by every lane and costs no extra memory traffic)
  CollIn<T> ci[K];
  if constexpr (MCC) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      ci[j].cand = false;
      ci[j].r1 = ci[j].wa = ci[j].wb = 0u;
      if (mcc && p[j].w) {
        WordStream ws(H.key0, H.key1, p[j].id, step);
        const uint32_t r0 = ws.next();
        ci[j].r1 = ws.next();
        ci[j].wa = ws.w0;
        ci[j].wb = ws.w1;
        ci[j].cand = (r0 >> 8) < k.tcand;
      }
      if constexpr (DIM == 2 && kVzPre) {
        ci[j].vz = p[j].v2;
        ci[j].vy = (T)0;
      } else {
        const uint32_t i = i0 + (uint32_t)j * kBlock;
        const uint32_t first = i - (uint32_t)lane_id();
        const uint32_t iz = ci[j].cand ? i : (first < end ? first : end - 1u);
        ci[j].vz = *at(P.v2, iz);
        if constexpr (DIM == 1) ci[j].vy = *at(P.v1, iz);
        else ci[j].vy = (T)0;
      }
    }
    issue_fence();
  }
  // 6. stage B of the next batch
#pragma unroll
  for (int j = 0; j < K; ++j) load_b<T, MCC, DIM>(P, inext0 + (uint32_t)j * kBlock, end, nxt[j]);
  issue_fence();
  // 7. collisions, births, stores, deposit
  if constexpr (DIM == 2 && DIRECT) {
#pragma unroll
    for (int j = 0; j < K; ++j) leaf[j] = moved[j] ? leaf[j] : p[j].cell;
  }
  if constexpr (MCC) {
    if (mcc) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t i = i0 + (uint32_t)j * kBlock;
        T vy = DIM == 2 ? p[j].v1 : ci[j].vy;
        T vz = ci[j].vz;
        uint32_t kind = kCollNone;
        if (ci[j].cand) kind = collision_kind<T>(k, ci[j].r1, p[j].v0, vy, vz, st);
        // elastic scattering in place
        const bool el = kind == kCollElastic;
        st.elastic += el ? 1u : 0u;
        if (el) {
          WordStream ws(H.key0, H.key1, p[j].id, step, ci[j].wa, ci[j].wb);
          collide_elastic<T>(k, ws, p[j].v0, vy, vz);
          if constexpr (DIM == 2) p[j].v1 = vy;
          else *at(P.v1, i) = vy;
          *at(P.v2, i) = vz;
        }
        // ionization and charge exchange to the queue
        const bool qx = kind == kCollIonize || kind == kCollCx;
        const uint64_t bm = __ballot(qx);
        if (bm == 0ull) continue;
        const int lane = lane_id();
        const int leader = __ffsll((long long)bm) - 1;
        uint32_t base = 0u;
        if (lane == leader) base = atomicAdd(Q.n, (uint32_t)__popcll(bm));
        base = __shfl(base, leader);
        if (!qx) continue;
        const uint32_t t = base + (uint32_t)__popcll(bm & (lanes_le(lane) >> 1));
        Q.kind[t] = kind;
        Q.i[t] = i;
        Q.r1[t] = ci[j].r1;
        Q.wa[t] = ci[j].wa;
        Q.wb[t] = ci[j].wb;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t i = i0 + (uint32_t)j * kBlock;
    if (FULL) {
      if (kFullWC) *at(P.w, i) = p[j].w;
      *at(P.s0, i) = p[j].s0;
      *at(P.v0, i) = p[j].v0;
      if (DIM == 2) {
        *at(P.s1, i) = p[j].s1;
        *at(P.v1, i) = p[j].v1;
        if (kFullWC || moved[j]) *at(P.cell, i) = leaf[j];
      }
    } else if (p[j].w != 0u) {
      *at(P.s0, i) = p[j].s0;
      *at(P.v0, i) = p[j].v0;
      if (DIM == 2) {
        *at(P.s1, i) = p[j].s1;
        *at(P.v1, i) = p[j].v1;
        if (moved[j]) *at(P.cell, i) = leaf[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (p[j].w == 0u) continue;
    const unsigned long long w = p[j].w;
    unsigned long long* Qs = Qpar + (size_t)sp * H.nq;
    if (DIM == 2) {
      dep_add(D, Qs, leaf[j], w);
    } else {
      // CIC shares in 64-bit fixed point
      const T g = p[j].s0 * (T)H.N;
      int ic = (int)floor(g);
      if (ic > H.N - 1) ic = H.N - 1;
      const T fr = g - (T)ic;
      const unsigned long long r = (unsigned long long)(long long)rint(fr * (T)(1ull << FixedPoint<T>::F));
      const unsigned long long one = 1ull << FixedPoint<T>::F;
      dep_add(D, Qs, (uint32_t)ic, w * (one - r));
      dep_add(D, Qs, (uint32_t)ic + 1u, w * r);
    }
  }
}

// Per-workgroup counters are added into the workgroup's own row of a
// partial-stats table (no atomics); the rows are summed once per pic_step call.
__device__ __forceinline__ void add_stats_row(unsigned long long* row, const LStat& st, int sp) {
  __shared__ uint32_t red[kBlock / 64][7];
  const int lane = lane_id(), wv = threadIdx.x / 64;
  const uint32_t vals[7] = {st.alive, st.absorbed, st.elastic, st.ionization, st.cx, st.viol, st.lost};
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const uint32_t s = wave_sum(vals[q]);
    if (lane == 0) red[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    uint32_t tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) tot += red[w][threadIdx.x];
    if (tot) {
      int idx;
      switch (threadIdx.x) {
        case 0: idx = kStAlive0 + sp; break;
        case 1: idx = kStAbs0 + sp; break;
        case 2: idx = kStElastic; break;
        case 3: idx = kStIonization; break;
        case 4: idx = kStCx; break;
        case 5: idx = kStViol0 + sp; break;
        default: idx = kStLostReflect; break;
      }
      row[idx] += tot;
    }
  }
}

// Zero the deposit buffer of the other step parity (it held the previous
// step's charge, already consumed by the field solve).
__device__ __forceinline__ void zero_other_parity(unsigned long long* Q, uint32_t nq, uint32_t step, int nspecies,
                                                  uint32_t tid, uint32_t nthreads) {
  unsigned long long* Z = Q + (size_t)((step + 1u) & 1u) * 2u * nq;
  const uint32_t n = (uint32_t)nspecies * nq;
  for (uint32_t j = tid; j < n; j += nthreads) Z[j] = 0ull;
}

// Last workgroup to finish advances the step index (used when no births
// kernel or field solve follows in the same step).  No fence is needed: the
// step index is read only by later launches, and no workgroup of this launch
// reads what the others wrote.
__device__ __forceinline__ void last_block_commit(Counters* c, uint32_t step) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev = gadd32(&c->done, 1u);
    if (prev == gridDim.x - 1u) {
      c->done = 0u;
      c->step = step + 1u;
    }
  }
}

template <class T, bool MCC, int DIM, int K, bool DIRECT>
__device__ __forceinline__ void run_range(const InstDev<T>& I, int sp, uint32_t begin, uint32_t end, uint32_t step,
                                          unsigned long long* Qpar, unsigned long long* row) {
  if (begin >= end) return;   // uniform: the whole workgroup has no particles here
  const DepLds L = dep_lds();
  unsigned long long* win = L.win;
  uint32_t* hkey = L.hkey;
  unsigned long long* hval = L.hval;
  uint32_t& wbase_s = *L.wbase;
  const SpPtr<T> P = species_ptrs<T>(I, sp);
  const HotK<T> H = hot_constants<T>(I, sp);
  const bool mcc = MCC && H.k.mcc != PIC_MCC_NONE;   // uniform over the workgroup
  CollQueue<T, DIM> Q{};
  if constexpr (MCC) {
    Q = coll_queue<T, DIM, K>();
    if (threadIdx.x == 0) *Q.n = 0u;
  }
  DepCache D{win, hkey, hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) {
    // window centred on the median cell of three live particles sampled at
    // the start, middle and end of the range (particles drift from cell
    // order between sorts, and a hole's stored position or leaf carries no
    // meaning: full batches overwrite them)
    uint32_t c[3];
    int n = 0;
    const uint32_t at3[3] = {begin, begin + (end - begin) / 2u, end - 1u};
    for (int k = 0; k < 3; ++k)
      if (*at(P.w, at3[k]) != 0u) c[n++] = DIM == 2 ? *at(P.cell, at3[k]) : cell1d<T>(I, *at(P.s0, at3[k]));
    uint32_t m = 0u;
    if (n == 1) m = c[0];
    else if (n == 2) m = c[0] < c[1] ? c[0] : c[1];
    else if (n == 3) m = c[0] < c[1] ? (c[1] < c[2] ? c[1] : (c[0] < c[2] ? c[2] : c[0]))
                                     : (c[0] < c[2] ? c[0] : (c[1] < c[2] ? c[2] : c[1]));
    wbase_s = m > kWin / 2u ? m - kWin / 2u : 0u;
  }
  // first batch: stage A, then stage B, in the same order as the loop issues
  // them for later batches
  PState<T> cur[K], nxt[K];
#pragma unroll
  for (int j = 0; j < K; ++j) load_a<T, MCC, DIM>(P, begin + (uint32_t)j * kBlock + threadIdx.x, end, cur[j]);
  issue_fence();
#pragma unroll
  for (int j = 0; j < K; ++j) load_b<T, MCC, DIM>(P, begin + (uint32_t)j * kBlock + threadIdx.x, end, cur[j]);
  issue_fence();
  __syncthreads();
  D.base = wbase_s;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  // Batches with the state buffers swapping roles (cur -> nxt, then nxt ->
  // cur), so the prefetched state is never copied between registers (a copy
  // would wait for it).
  const uint32_t unit = (uint32_t)K * kBlock;
  uint32_t base = begin;
  if constexpr (!MCC) {
    // two full batches per trip, then the partial batch
    bool in_cur = true;
    while (end - base >= unit) {
      process_batch<T, MCC, DIM, K, DIRECT, true>(I, H, P, sp, base + threadIdx.x, cur, nxt, end, step, Qpar, D, st, Q);
      base += unit;
      if (end - base < unit) {
        in_cur = false;
        break;
      }
      process_batch<T, MCC, DIM, K, DIRECT, true>(I, H, P, sp, base + threadIdx.x, nxt, cur, end, step, Qpar, D, st, Q);
      base += unit;
    }
    if (base < end) {
      if (in_cur) process_batch<T, MCC, DIM, K, DIRECT, false>(I, H, P, sp, base + threadIdx.x, cur, nxt, end, step, Qpar, D, st, Q);
      else process_batch<T, MCC, DIM, K, DIRECT, false>(I, H, P, sp, base + threadIdx.x, nxt, cur, end, step, Qpar, D, st, Q);
    }
  } else {
    // collision kernels: one batch per trip; the queue of ionizations and
    // charge exchanges is drained at the top of a trip once it holds kQDrain
    // entries, and at the end.  The single drain site keeps that code in the
    // kernel once.
    bool in_cur = true;
    for (;;) {
      const bool done = base >= end;
      if (mcc) {
        __syncthreads();
        const uint32_t nq = *Q.n;
        if (nq >= kQDrain || (done && nq > 0u)) drain_queue<T, DIM>(I, H, P, sp, step, Q, Qpar, D, st);
      }
      if (done) break;
      const uint32_t i0 = base + threadIdx.x;
      if (end - base >= unit) {
        if (in_cur) process_batch<T, MCC, DIM, K, DIRECT, true>(I, H, P, sp, i0, cur, nxt, end, step, Qpar, D, st, Q);
        else process_batch<T, MCC, DIM, K, DIRECT, true>(I, H, P, sp, i0, nxt, cur, end, step, Qpar, D, st, Q);
        base += unit;
      } else {
        if (in_cur) process_batch<T, MCC, DIM, K, DIRECT, false>(I, H, P, sp, i0, cur, nxt, end, step, Qpar, D, st, Q);
        else process_batch<T, MCC, DIM, K, DIRECT, false>(I, H, P, sp, i0, nxt, cur, end, step, Qpar, D, st, Q);
        base = end;
      }
      in_cur = !in_cur;
    }
  }
  __syncthreads();
  dep_flush(D, Qpar + (size_t)sp * I.nq, I.nq);
  add_stats_row(row, st, sp);
  __syncthreads();
}

// Particles per lane per batch of the step kernels.
#ifndef PIC_BATCH_2D
#define PIC_BATCH_2D 2
#endif
#ifndef PIC_BATCH_1D
#define PIC_BATCH_1D 2
#endif
#ifndef PIC_BATCH_MCC1D
#define PIC_BATCH_MCC1D 2
#endif
#ifndef PIC_BATCH_MCC2D
#define PIC_BATCH_MCC2D 1
#endif
template <class T, int DIM, bool MCC>
constexpr int batch_k() {
  return MCC ? (DIM == 2 ? PIC_BATCH_MCC2D : PIC_BATCH_MCC1D) : DIM == 2 ? PIC_BATCH_2D : PIC_BATCH_1D;
}

// Plain launch over one instance: workgroups [0, gs) own consecutive chunks
// of species 0, [gs, grid) of species 1, gs in proportion to the live counts
// (read from the device counters, so the split follows births and losses
// without host round trips).
#ifndef PIC_STEP_WAVES
#define PIC_STEP_WAVES 0
#endif
#if PIC_STEP_WAVES > 0
#define PIC_STEP_ATTR __attribute__((amdgpu_waves_per_eu(PIC_STEP_WAVES)))
#else
#define PIC_STEP_ATTR
#endif
// Workgroup b's place when the 8 XCDs each take a contiguous share of the
// grid (workgroups are dealt to the XCDs in turn); identity when the grid
// does not divide evenly.  The octree kernel uses it: its leaves' corner E
// (96 B each, 4.5 MB on the octree workload) outgrow one XCD's L2 when
// every XCD reads every region (71.3 instead of 73.5 us per launch); on
// the quadtree (32 B per leaf) and in 1D it gained nothing.
#ifndef PIC_XCD_3D
#define PIC_XCD_3D 1
#endif
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t grid) {
  constexpr uint32_t kXcd = 8;
  if (grid % kXcd) return b;
  return (b % kXcd) * (grid / kXcd) + b / kXcd;
}

template <class T, bool MCC, int DIM, bool DIRECT>
__global__ __launch_bounds__(kBlock) PIC_STEP_ATTR void k_step(InstDev<T> I, int commit) {
  constexpr int K = batch_k<T, DIM, MCC>();
  if (step_blocked<T>(I)) {   // uniform over the launch: no room for this step's births
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
    return;
  }
  const uint32_t step = I.ctr->step;
  const uint32_t n0 = I.ctr->count[0];
  const uint32_t n1 = I.nspecies == 2 ? I.ctr->count[1] : 0u;
  const uint32_t grid = gridDim.x;
  uint32_t gs = grid;
  if (I.nspecies == 2) {
    gs = (uint32_t)(((uint64_t)grid * n0 + ((uint64_t)n0 + n1) / 2u) / ((uint64_t)n0 + n1 + 1u));
    if (gs < 1u) gs = 1u;
    if (gs > grid - 1u) gs = grid - 1u;
  }
  const int sp = blockIdx.x >= gs ? 1 : 0;
  const uint32_t b = sp == 0 ? blockIdx.x : blockIdx.x - gs;
  const uint32_t nb = sp == 0 ? gs : grid - gs;
  const uint32_t count = sp == 0 ? n0 : n1;
  constexpr int KU = K > batch_k<T, DIM, false>() ? K : batch_k<T, DIM, false>();
  const uint32_t unit = (uint32_t)KU * kBlock;
  const uint32_t chunk = ((count + nb - 1u) / nb + unit - 1u) / unit * unit;
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  const uint64_t begin64 = (uint64_t)b * chunk;
  const uint32_t begin = begin64 < count ? (uint32_t)begin64 : count;
  const uint32_t end = (uint64_t)begin + chunk < count ? begin + chunk : count;
  unsigned long long* row = I.part + (size_t)blockIdx.x * kNStat;
  if constexpr (MCC) {
    // a species without collisions takes the collisionless loop (uniform)
    if (I.sk[sp].mcc == PIC_MCC_NONE) run_range<T, false, DIM, batch_k<T, DIM, false>(), DIRECT>(I, sp, begin, end, step, Qpar, row);
    else run_range<T, true, DIM, K, DIRECT>(I, sp, begin, end, step, Qpar, row);
  } else {
    run_range<T, false, DIM, K, DIRECT>(I, sp, begin, end, step, Qpar, row);
  }
  if (commit) last_block_commit(I.ctr, step);
}

// Batched 1D launch: a persistent grid walks a list of (instance, species,
// range) work items; per-instance constants come from the descriptor table.
#ifndef PIC_BATCHED_WAVES
#define PIC_BATCHED_WAVES 0
#endif
#if PIC_BATCHED_WAVES > 0
#define PIC_BATCHED_ATTR __attribute__((amdgpu_waves_per_eu(PIC_BATCHED_WAVES)))
#else
#define PIC_BATCHED_ATTR
#endif
template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) PIC_BATCHED_ATTR void k_step1d_batched(const InstDev<T>* __restrict__ insts,
                                                           const WorkItem* __restrict__ items, uint32_t nitems,
                                                           unsigned long long* bpart) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const InstDev<T>& I = insts[wi.inst];
    const int sp = (int)wi.species;
    if (step_blocked<T>(I)) {   // the same decision for every item of the instance
      if (wi.begin == 0 && sp == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
      continue;
    }
    const uint32_t step = I.ctr->step;
    const uint32_t count = I.ctr->count[sp];
    const uint32_t end = wi.end < count ? wi.end : count;
    unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
    if (wi.begin == 0 && sp == 0) zero_other_parity(I.Q, I.nq, step, I.nspecies, threadIdx.x, kBlock);
    run_range<T, MCC, 1, batch_k<T, 1, MCC>(), false>(I, sp, wi.begin, end, step, Qpar, bpart + (size_t)it * kNStat);
  }
}

// Batched 2D launch: the same walk over (instance, species, range) work
// items of quadtree instances; each instance's leaf tables, point-location
// table and corner-E table come from its descriptor, and whether its tree
// is shallow enough for a direct lookup is decided per item (uniform over
// the workgroup).
template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) void k_step2d_batched(const InstDev<T>* __restrict__ insts,
                                                           const WorkItem* __restrict__ items, uint32_t nitems,
                                                           unsigned long long* bpart) {
  constexpr int KM = batch_k<T, 2, true>(), KF = batch_k<T, 2, false>();
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const InstDev<T>& I = insts[wi.inst];
    const int sp = (int)wi.species;
    if (step_blocked<T>(I)) {   // the same decision for every item of the instance
      if (wi.begin == 0 && sp == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
      continue;
    }
    const uint32_t step = I.ctr->step;
    const uint32_t count = I.ctr->count[sp];
    const uint32_t end = wi.end < count ? wi.end : count;
    unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
    if (wi.begin == 0 && sp == 0) zero_other_parity(I.Q, I.nq, step, I.nspecies, threadIdx.x, kBlock);
    unsigned long long* row = bpart + (size_t)it * kNStat;
    if (MCC && I.sk[sp].mcc != PIC_MCC_NONE) {
      if (I.lut_direct) run_range<T, true, 2, KM, true>(I, sp, wi.begin, end, step, Qpar, row);
      else run_range<T, true, 2, KM, false>(I, sp, wi.begin, end, step, Qpar, row);
    } else {
      if (I.lut_direct) run_range<T, false, 2, KF, true>(I, sp, wi.begin, end, step, Qpar, row);
      else run_range<T, false, 2, KF, false>(I, sp, wi.begin, end, step, Qpar, row);
    }
  }
}

// ---------------------------------------------------------------------------
// Births: rank by parent id (count of smaller staged parent ids; the ids are
// distinct), then append the electron at count[0] + r with id next_id + 2r
// and the ion at count[1] + r with id next_id + 2r + 1.
// The ranking is split into work items (key tile a, chunk c): the kRankPer x
// kBlock staged births of tile a are compared with the kRankChunk staged
// parent ids of chunk c held in LDS, and each adds its count of smaller ids
// to rank[i].  No lane walks all staged ids, so the time does not grow with
// the number of births as long as work items remain to spread.  A second
// kernel writes the newborn particles and clears rank[] for the next step.
// ---------------------------------------------------------------------------
constexpr uint32_t kRankPer = 4;
constexpr uint32_t kRankChunk = 256;
#ifndef PIC_RANK_BLOCKS
#define PIC_RANK_BLOCKS 1024
#endif
constexpr int kRankBlocks = 256;   // workgroups per instance of the batched ranking kernel
constexpr int kRankBlocksPlain = PIC_RANK_BLOCKS;   // workgroups of the single-instance ranking kernel
constexpr int kWriteBlocks = 64;   // workgroups per instance of the writing kernel

template <class T>
__device__ __forceinline__ bool births_fit(const InstDev<T>& I, uint32_t nb, bool& cap_ok, bool& id_ok) {
  cap_ok = id_ok = true;
  if (I.ctr->flags & kFlagNeedRoom) return false;   // the step was not run
  const uint32_t c0 = I.ctr->count[0], c1 = I.ctr->count[1], nid = I.ctr->next_id;
  cap_ok = (uint64_t)c0 + nb <= I.cap[0] && (uint64_t)c1 + nb <= I.cap[1] && nb <= I.birth_cap;
  id_ok = (uint64_t)nid + 2ull * nb <= 0xFFFFFFFFull;
  return cap_ok && id_ok;
}

template <class T>
__device__ void birth_rank_body(const InstDev<T>& I, uint32_t first, uint32_t nblocks) {
  __shared__ uint32_t sh[kRankChunk];
  const uint32_t nb = I.ctr->nbirths;
  bool cap_ok, id_ok;
  if (nb == 0u || !births_fit(I, nb, cap_ok, id_ok)) return;
  const uint32_t tile = kRankPer * kBlock;
  const uint32_t na = (nb + tile - 1u) / tile, nc = (nb + kRankChunk - 1u) / kRankChunk;
  for (uint32_t wi = first; wi < na * nc; wi += nblocks) {
    const uint32_t a = wi / nc, jb = (wi % nc) * kRankChunk;
    const uint32_t lim = (nb - jb) < kRankChunk ? (nb - jb) : kRankChunk;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < lim; t += kBlock) sh[t] = I.br.parent[jb + t];
    __syncthreads();
    uint32_t mine[kRankPer], cnt[kRankPer];
#pragma unroll
    for (uint32_t q = 0; q < kRankPer; ++q) {
      const uint32_t i = a * tile + q * kBlock + threadIdx.x;
      mine[q] = i < nb ? I.br.parent[i] : 0u;
      cnt[q] = 0u;
    }
    for (uint32_t j = 0; j < lim; ++j) {
      const uint32_t v = sh[j];
#pragma unroll
      for (uint32_t q = 0; q < kRankPer; ++q) cnt[q] += (v < mine[q]) ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < kRankPer; ++q) {
      const uint32_t i = a * tile + q * kBlock + threadIdx.x;
      if (i < nb && cnt[q]) atomicAdd(&I.br.rank[i], cnt[q]);
    }
  }
}

template <class T>
__device__ void birth_write_body(const InstDev<T>& I, uint32_t first, uint32_t nblocks) {
  const uint32_t nb = I.ctr->nbirths;
  if (nb == 0u) return;
  bool cap_ok, id_ok;
  if (!births_fit(I, nb, cap_ok, id_ok)) {
    if (threadIdx.x == 0 && first == 0 && !(cap_ok && id_ok))
      atomicOr(&I.ctr->flags, (!cap_ok ? kFlagBirthOverflow : 0u) | (!id_ok ? kFlagIdOverflow : 0u));
    return;
  }
  const uint32_t c0 = I.ctr->count[0], c1 = I.ctr->count[1], nid = I.ctr->next_id;
  for (uint32_t i = first * kBlock + threadIdx.x; i < nb; i += nblocks * kBlock) {
    const uint32_t r = I.br.rank[i];
    I.br.rank[i] = 0u;
    const uint32_t pe = c0 + r, pi = c1 + r;
    const uint32_t w = I.br.w[i];
    I.s[0][0][pe] = I.br.s[0][i];
    I.s[1][0][pi] = I.br.s[0][i];
    if (I.dim >= 2) {
      I.s[0][1][pe] = I.br.s[1][i];
      I.s[1][1][pi] = I.br.s[1][i];
      I.cell[0][pe] = I.br.cell[i];
      I.cell[1][pi] = I.br.cell[i];
    }
    if (I.dim == 3) {
      I.s[0][2][pe] = I.br.s[2][i];
      I.s[1][2][pi] = I.br.s[2][i];
    }
    for (int c = 0; c < 3; ++c) {
      I.v[0][c][pe] = I.br.ve[c][i];
      I.v[1][c][pi] = I.br.vi[c][i];
    }
    I.w[0][pe] = w;
    I.w[1][pi] = w;
    if (I.dipic) {   // a newborn has no filtered acceleration yet
      I.acc[0][pe] = (T)0;
      I.acc[1][pi] = (T)0;
    }
    I.id[0][pe] = nid + 2u * r;
    I.id[1][pi] = nid + 2u * r + 1u;
  }
}

// Binned ranking.  Parent ids below next_id fall into kBirthBins bins of
// 2^shift consecutive ids; a birth's rank is the number of staged parents in
// lower bins (the bin offset) plus those in its own bin with a smaller id, so
// each birth compares only with the members of its bin.
__device__ __forceinline__ uint32_t birth_bin_shift(uint32_t next_id) {
  const uint32_t top = next_id > 0u ? next_id - 1u : 0u;
  uint32_t sh = 0u;
  while (sh < 31u && (top >> sh) >= kBirthBins) ++sh;
  return sh;
}

template <class T>
__device__ void birth_bin_body(const InstDev<T>& I, uint32_t first, uint32_t nblocks) {
  __shared__ uint32_t hist[kBirthBins];
  const uint32_t nb = I.ctr->nbirths;
  bool cap_ok, id_ok;
  if (nb == 0u || !births_fit(I, nb, cap_ok, id_ok)) return;
  const uint32_t sh = birth_bin_shift(I.ctr->next_id);
  for (uint32_t b = threadIdx.x; b < kBirthBins; b += kBlock) hist[b] = 0u;
  __syncthreads();
  for (uint32_t i = first * kBlock + threadIdx.x; i < nb; i += nblocks * kBlock)
    atomicAdd(&hist[I.br.parent[i] >> sh], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < kBirthBins; b += kBlock)
    if (hist[b]) gadd32(I.br.bin + b, hist[b]);
}

// one workgroup of 1024 threads: offsets and cursors of the bins; clears the counts
template <class T>
__device__ void birth_binscan_body(const InstDev<T>& I) {
  __shared__ uint32_t part[1024];
  const uint32_t nb = I.ctr->nbirths;
  bool cap_ok, id_ok;
  if (nb == 0u || !births_fit(I, nb, cap_ok, id_ok)) return;
  constexpr uint32_t per = kBirthBins / 1024u;
  uint32_t c[per], sum = 0u;
#pragma unroll
  for (uint32_t q = 0; q < per; ++q) {
    c[q] = I.br.bin[threadIdx.x * per + q];
    sum += c[q];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < 1024u; d <<= 1) {   // inclusive scan of the thread sums
    const uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
#pragma unroll
  for (uint32_t q = 0; q < per; ++q) {
    const uint32_t b = threadIdx.x * per + q;
    I.br.bin_off[b] = run;
    I.br.cursor[b] = run;
    I.br.bin[b] = 0u;
    run += c[q];
  }
  if (threadIdx.x == 1023u) I.br.bin_off[kBirthBins] = run;
}

template <class T>
__device__ void birth_scatter_body(const InstDev<T>& I, uint32_t first, uint32_t nblocks) {
  const uint32_t nb = I.ctr->nbirths;
  bool cap_ok, id_ok;
  if (nb == 0u || !births_fit(I, nb, cap_ok, id_ok)) return;
  const uint32_t sh = birth_bin_shift(I.ctr->next_id);
  for (uint32_t i = first * kBlock + threadIdx.x; i < nb; i += nblocks * kBlock) {
    const uint32_t pid = I.br.parent[i];
    I.br.sorted[gadd32(I.br.cursor + (pid >> sh), 1u)] = pid;
  }
}

template <class T>
__device__ void birth_rank_binned_body(const InstDev<T>& I, uint32_t first, uint32_t nblocks) {
  const uint32_t nb = I.ctr->nbirths;
  bool cap_ok, id_ok;
  if (nb == 0u || !births_fit(I, nb, cap_ok, id_ok)) return;
  const uint32_t sh = birth_bin_shift(I.ctr->next_id);
  for (uint32_t i = first * kBlock + threadIdx.x; i < nb; i += nblocks * kBlock) {
    const uint32_t pid = I.br.parent[i];
    const uint32_t b = pid >> sh;
    const uint32_t lo = I.br.bin_off[b], hi = I.br.bin_off[b + 1u];
    uint32_t r = lo;
    for (uint32_t j = lo; j < hi; ++j) r += I.br.sorted[j] < pid ? 1u : 0u;
    I.br.rank[i] = r;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_bin(InstDev<T> I) { birth_bin_body<T>(I, blockIdx.x, gridDim.x); }
template <class T>
__global__ __launch_bounds__(1024) void k_birth_binscan(InstDev<T> I) { birth_binscan_body<T>(I); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_scatter(InstDev<T> I) {
  birth_scatter_body<T>(I, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_rank_binned(InstDev<T> I) {
  birth_rank_binned_body<T>(I, blockIdx.x, gridDim.x);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_rank(InstDev<T> I) { birth_rank_body<T>(I, blockIdx.x, gridDim.x); }
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_write(InstDev<T> I) { birth_write_body<T>(I, blockIdx.x, gridDim.x); }

// grid (per_inst, ninst): blockIdx.y selects the instance, blockIdx.x the
// share of its work
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_rank_batched(const InstDev<T>* insts) {
  const InstDev<T>& I = insts[blockIdx.y];
  if (!I.births_binned) birth_rank_body<T>(I, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_bin_batched(const InstDev<T>* insts) {
  const InstDev<T>& I = insts[blockIdx.y];
  if (I.births_binned) birth_bin_body<T>(I, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(1024) void k_birth_binscan_batched(const InstDev<T>* insts) {
  const InstDev<T>& I = insts[blockIdx.y];
  if (I.births_binned) birth_binscan_body<T>(I);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_scatter_batched(const InstDev<T>* insts) {
  const InstDev<T>& I = insts[blockIdx.y];
  if (I.births_binned) birth_scatter_body<T>(I, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_rank_binned_batched(const InstDev<T>* insts) {
  const InstDev<T>& I = insts[blockIdx.y];
  if (I.births_binned) birth_rank_binned_body<T>(I, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_birth_write_batched(const InstDev<T>* insts) {
  birth_write_body<T>(insts[blockIdx.y], blockIdx.x, gridDim.x);
}

// Commit a step after the births kernel: append births to the counts,
// advance the step index.  One thread.
template <class T>
__device__ void commit_body(const InstDev<T>& I) {
  if (threadIdx.x == 0) {
    Counters* c = I.ctr;
    if (c->flags & kFlagNeedRoom) return;   // the step was not run: no commit
    const uint32_t nb = c->nbirths;
    if (nb && !(c->flags & (kFlagBirthOverflow | kFlagIdOverflow))) {
      c->count[0] += nb;
      c->count[1] += nb;
      c->next_id += 2u * nb;
      c->stats[kStBirths] += nb;
    }
    c->nbirths = 0u;
    c->step += 1u;
  }
}

template <class T>
__global__ void k_commit(InstDev<T> I) { commit_body<T>(I); }

template <class T>
__global__ void k_commit_batched(const InstDev<T>* insts) { commit_body<T>(insts[blockIdx.x]); }

// Sum partial-stats rows [row_begin[b], row_begin[b+1]) into instance b's
// counters and clear them.
template <class T>
__global__ __launch_bounds__(kBlock) void k_stats_reduce(const InstDev<T>* insts, unsigned long long* rows,
                                                         const uint32_t* row_begin, uint32_t nrows_plain) {
  const InstDev<T>& I = insts[blockIdx.x];
  // row_begin: [ninst + 1] first rows followed by [ninst + 1] end rows
  const uint32_t rb = row_begin ? row_begin[blockIdx.x] : 0u;
  const uint32_t re = row_begin ? row_begin[gridDim.x + 1 + blockIdx.x] : nrows_plain;
  unsigned long long* R = rows ? rows : I.part;
  __shared__ unsigned long long acc[kBlock / 64][kNStat];
  unsigned long long loc[kNStat];
#pragma unroll
  for (int q = 0; q < kNStat; ++q) loc[q] = 0ull;
  for (uint32_t r = rb + threadIdx.x; r < re; r += kBlock) {
#pragma unroll
    for (int q = 0; q < kNStat; ++q) {
      loc[q] += R[(size_t)r * kNStat + q];
      R[(size_t)r * kNStat + q] = 0ull;
    }
  }
#pragma unroll
  for (int q = 0; q < kNStat; ++q) {
    const unsigned long long s = wave_sum(loc[q]);
    if (lane_id() == 0) acc[threadIdx.x / 64][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNStat) {
    unsigned long long t = 0ull;
    for (int w = 0; w < kBlock / 64; ++w) t += acc[w][threadIdx.x];
    I.ctr->stats[threadIdx.x] += t;
  }
}

// ---------------------------------------------------------------------------
// Standalone deposit of the current particles into the latest buffer
// Q[(step + 1) & 1] (zeroed by the caller).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void k_deposit(InstDev<T> I) {
  const uint32_t step = I.ctr->step;
  unsigned long long* Qpar = I.Q + (size_t)((step + 1u) & 1u) * 2u * I.nq;
  for (int sp = 0; sp < I.nspecies; ++sp) {
    const uint32_t count = I.ctr->count[sp];
    for (uint32_t base = blockIdx.x * kBlock; base < count; base += gridDim.x * kBlock) {
      const uint32_t i = base + threadIdx.x;
      const uint32_t w = i < count ? G(I.w[sp])[i] : 0u;
      uint32_t k0 = kNoKey, k1 = kNoKey;
      unsigned long long q0 = 0ull, q1 = 0ull;
      if (w) {
        if (I.dim == 1) {
          const T g = G(I.s[sp][0])[i] * (T)I.N;
          int ic = (int)floor(g);
          if (ic > I.N - 1) ic = I.N - 1;
          const T f = g - (T)ic;
          const unsigned long long r = (unsigned long long)(long long)rint(f * (T)(1ull << FixedPoint<T>::F));
          const unsigned long long one = 1ull << FixedPoint<T>::F;
          k0 = (uint32_t)ic;
          k1 = (uint32_t)ic + 1u;
          q0 = (unsigned long long)w * (one - r);
          q1 = (unsigned long long)w * r;
        } else {
          k0 = G(I.cell[sp])[i];
          q0 = w;
        }
      }
      seg_atomic_add(Qpar + (size_t)sp * I.nq, k0, q0);
      seg_atomic_add(Qpar + (size_t)sp * I.nq, k1, q1);
    }
  }
}

// ---------------------------------------------------------------------------
// Octree (3D, Sec. 3.1 quad/octree with cubic cells).  The gather is the
// trilinear interpolation of the leaf's corner E (corner c = a + 2b + 4e
// along x, y, z), weights ((x factor)(y factor))(z factor), summed over the
// corners in order; the deposit is NGP to the leaf.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void gather3d(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T sz, T e[3]) {
  const uint32_t p = G(I.leaf_xy)[leaf];
  const int L = (int)G(I.leaf_lv)[leaf];
  const int sh = 10 - L;
  const T sc = (T)(1u << L);
  const T f0 = sx * sc - (T)((p & 0x3FFu) >> sh);
  const T f1 = sy * sc - (T)(((p >> 10) & 0x3FFu) >> sh);
  const T f2 = sz * sc - (T)(((p >> 20) & 0x3FFu) >> sh);
  const T* ce = I.E + (size_t)leaf * 24u;
  e[0] = e[1] = e[2] = (T)0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const T wx = (c & 1) ? f0 : (T)1 - f0;
    const T wy = ((c >> 1) & 1) ? f1 : (T)1 - f1;
    const T wz = (c >> 2) ? f2 : (T)1 - f2;
    const T w = (wx * wy) * wz;
#pragma unroll
    for (int a = 0; a < 3; ++a) e[a] = e[a] + w * G(ce)[c * 3 + a];
  }
}

// The particle loop of an octree slot: one particle per lane, in place
// (gather, push, walls, locate, MCC with births, NGP deposit).  Workgroups
// take contiguous ranges of a species as k_step does.
template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) void k_step3d(InstDev<T> I, int commit) {
  if (step_blocked<T>(I)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
    return;
  }
  const uint32_t step = I.ctr->step;
  const uint32_t n0 = I.ctr->count[0];
  const uint32_t n1 = I.nspecies == 2 ? I.ctr->count[1] : 0u;
  const uint32_t grid = gridDim.x;
  uint32_t gs = grid;
  if (I.nspecies == 2) {
    gs = (uint32_t)(((uint64_t)grid * n0 + ((uint64_t)n0 + n1) / 2u) / ((uint64_t)n0 + n1 + 1u));
    if (gs < 1u) gs = 1u;
    if (gs > grid - 1u) gs = grid - 1u;
  }
  // the workgroups one XCD receives (the dispatcher deals them out in turn)
  // take consecutive ranges of the cell-ordered particles, so each leaf's
  // corner E is read into one XCD's L2
  const uint32_t vb = PIC_XCD_3D ? xcd_contiguous(blockIdx.x, grid) : blockIdx.x;
  const int sp = vb >= gs ? 1 : 0;
  const uint32_t b = sp == 0 ? vb : vb - gs;
  const uint32_t nb = sp == 0 ? gs : grid - gs;
  const uint32_t count = sp == 0 ? n0 : n1;
  const uint32_t chunk = ((count + nb - 1u) / nb + kBlock - 1u) / kBlock * kBlock;
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  const uint64_t begin64 = (uint64_t)b * chunk;
  const uint32_t begin = begin64 < count ? (uint32_t)begin64 : count;
  const uint32_t end = (uint64_t)begin + chunk < count ? begin + chunk : count;
  unsigned long long* row = I.part + (size_t)blockIdx.x * kNStat;
  unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
  unsigned long long* Qi = Qpar + I.nq;
  const DepLds Ld = dep_lds();
  DepCache D{Ld.win, Ld.hkey, Ld.hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) {
    const uint32_t c0 = begin < end && G(I.w[sp])[begin] ? G(I.cell[sp])[begin] : 0u;
    *Ld.wbase = c0 > kWin / 2u ? c0 - kWin / 2u : 0u;
  }
  __syncthreads();
  D.base = *Ld.wbase;
  const SpeciesK<T> k = I.sk[sp];
  const bool mcc = MCC && k.mcc != PIC_MCC_NONE;
  const bool reflect = I.particle_bc == PIC_REFLECT;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t base = begin; base < end; base += kBlock) {
    const uint32_t i = base + threadIdx.x;
    uint32_t w = i < end ? G(I.w[sp])[i] : 0u;
    bool live = w != 0u;
    T s[3] = {(T)0, (T)0, (T)0}, v[3] = {(T)0, (T)0, (T)0};
    uint32_t id = 0u, leaf = 0u;
    bool birth = false;
    BirthRec<T> rec;
    if (live) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a] = G(I.s[sp][a])[i];
        v[a] = G(I.v[sp][a])[i];
      }
      id = G(I.id[sp])[i];
      leaf = G(I.cell[sp])[i];
      st.alive++;
      T e[3];
      gather3d<T>(I, leaf, s[0], s[1], s[2], e);
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a] = v[a] + k.qm_dt * e[a];
#pragma unroll
      for (int a = 0; a < 3; ++a) s[a] = s[a] + v[a] * k.dt_L;
      bool lost = false;
      const bool okx = wall_rule<T>(reflect, s[0], v[0], lost);
      const bool oky = okx && wall_rule<T>(reflect, s[1], v[1], lost);
      const bool okz = oky && wall_rule<T>(reflect, s[2], v[2], lost);
      if (!okz) {
        live = false;
        st.absorbed++;
        st.lost += lost ? 1u : 0u;
        G(I.w[sp])[i] = 0u;
      } else {
        leaf = locate_leaf3(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, (uint32_t)(s[0] * (T)1024),
                            (uint32_t)(s[1] * (T)1024), (uint32_t)(s[2] * (T)1024), I.lut_direct != 0);
        if (mcc) {
          WordStream ws(I.key0, I.key1, id, step);
          const uint32_t r0 = ws.next();
          const uint32_t r1 = ws.next();
          if ((r0 >> 8) < k.tcand) {
            const uint32_t kind = collision_kind<T>(k, r1, v[0], v[1], v[2], st);
            if (kind == kCollElastic) {
              collide_elastic<T>(k, ws, v[0], v[1], v[2]);
              st.elastic++;
            } else if (kind == kCollIonize) {
              collide_ionize<T>(k, ws, v[0], v[1], v[2], rec);
              birth = true;
              st.ionization++;
            } else if (kind == kCollCx) {
              st.cx += collide_cx<T>(k, r1, ws, v[0], v[1], v[2], st) ? 1u : 0u;
            }
          }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          G(I.s[sp][a])[i] = s[a];
          G(I.v[sp][a])[i] = v[a];
        }
        G(I.cell[sp])[i] = leaf;
      }
    }
    stage_birth<T>(I, birth, id, leaf, w, s[0], s[1], rec, s[2]);
    if (live) dep_add(D, Qs, leaf, (unsigned long long)w);
    if (birth) {   // the newborn electron and ion sit on the parent
      dep_add(D, Qs, leaf, (unsigned long long)w);
      gadd(Qi + leaf, (unsigned long long)w);
    }
  }
  __syncthreads();
  dep_flush(D, Qs, I.nq);
  add_stats_row(row, st, sp);
  if (commit) last_block_commit(I.ctr, step);
}

// ---------------------------------------------------------------------------
// 1D direct implicit step (Sec. 3, the D1 scheme).  acc holds b = (dt/2)
// abar, abar the time-filtered acceleration.  The predictor moves every
// particle with v~ = v + b, x~ = x + dt v~ (wall rule) and deposits the CIC
// charge of x~ into Qp; the field kernel then solves the Poisson equation
// with the implicit susceptibility of that charge for E_n+1; the corrector
// adds dv = (q dt / 2m) E_n+1(x~) to v and dt dv to x, sets b = (b + dv)/2,
// applies the wall rule, the collisions and births, and deposits the step's
// charge.  One lane per particle; the species split of the workgroups is
// the explicit step's, so both kernels add their counts to the same
// partial-stats rows.
struct BlockRange {
  int sp;
  uint32_t begin, end;
};
template <class T>
__device__ __forceinline__ BlockRange dipic_range(const InstDev<T>& I) {
  const uint32_t n0 = I.ctr->count[0];
  const uint32_t n1 = I.nspecies == 2 ? I.ctr->count[1] : 0u;
  const uint32_t grid = gridDim.x;
  uint32_t gs = grid;
  if (I.nspecies == 2) {
    gs = (uint32_t)(((uint64_t)grid * n0 + ((uint64_t)n0 + n1) / 2u) / ((uint64_t)n0 + n1 + 1u));
    if (gs < 1u) gs = 1u;
    if (gs > grid - 1u) gs = grid - 1u;
  }
  BlockRange r;
  r.sp = blockIdx.x >= gs ? 1 : 0;
  const uint32_t b = r.sp == 0 ? blockIdx.x : blockIdx.x - gs;
  const uint32_t nb = r.sp == 0 ? gs : grid - gs;
  const uint32_t count = r.sp == 0 ? n0 : n1;
  const uint32_t chunk = ((count + nb - 1u) / nb + kBlock - 1u) / kBlock * kBlock;
  const uint64_t begin64 = (uint64_t)b * chunk;
  r.begin = begin64 < count ? (uint32_t)begin64 : count;
  r.end = (uint64_t)r.begin + chunk < count ? r.begin + chunk : count;
  return r;
}

// CIC shares of a 1D position in 64-bit fixed point: node ic gets w (1 - f),
// node ic + 1 gets w f.
template <class T>
__device__ __forceinline__ void cic1d_shares(int N, T s, uint32_t w, uint32_t& ic_out, unsigned long long& q0,
                                             unsigned long long& q1) {
  const T g = s * (T)N;
  int ic = (int)floor(g);
  if (ic > N - 1) ic = N - 1;
  const T fr = g - (T)ic;
  const unsigned long long one = 1ull << FixedPoint<T>::F;
  const unsigned long long r = (unsigned long long)(long long)rint(fr * (T)(1ull << FixedPoint<T>::F));
  ic_out = (uint32_t)ic;
  q0 = (unsigned long long)w * (one - r);
  q1 = (unsigned long long)w * r;
}

// Wave-level pre-aggregation in front of the LDS deposit cache: runs of
// equal consecutive keys are summed by shuffles and their last lane adds the
// run (cell-ordered particles make long runs).  Every lane of the wave calls
// it; kNoKey lanes add nothing.
__device__ __forceinline__ void seg_dep_add(DepCache& D, unsigned long long* g, uint32_t key,
                                            unsigned long long val) {
  const int lane = lane_id();
  const int start = run_start(key, lane);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long o = __shfl_up(val, (unsigned)off);
    if (lane - off >= start) val += o;
  }
  if (run_tail(key, lane)) dep_add(D, g, key, val);
}

// Deposit window of a workgroup's range: centred on the median cell of
// three live particles sampled at its start, middle and end.
template <class T>
__device__ __forceinline__ uint32_t dipic_window_base(const InstDev<T>& I, const T* S, const uint32_t* W,
                                                      uint32_t begin, uint32_t end) {
  if (begin >= end || I.nq <= kWin) return 0u;   // the window holds every node
  uint32_t c[3];
  int n = 0;
  const uint32_t at3[3] = {begin, begin + (end - begin) / 2u, end - 1u};
  for (int k = 0; k < 3; ++k)
    if (W[at3[k]] != 0u) c[n++] = cell1d<T>(I, S[at3[k]]);
  uint32_t m = 0u;
  if (n == 1) m = c[0];
  else if (n == 2) m = c[0] < c[1] ? c[0] : c[1];
  else if (n == 3) m = c[0] < c[1] ? (c[1] < c[2] ? c[1] : (c[0] < c[2] ? c[2] : c[0]))
                                   : (c[0] < c[2] ? c[0] : (c[1] < c[2] ? c[2] : c[1]));
  return m > kWin / 2u ? m - kWin / 2u : 0u;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_dipic_predict(InstDev<T> I) {
  if (step_blocked<T>(I)) {   // uniform over the launch: no room for this step's births
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
    return;
  }
  const BlockRange R = dipic_range<T>(I);
  const int sp = R.sp;
  const T dt_L = I.sk[sp].dt_L;
  const bool reflect = I.particle_bc == PIC_REFLECT;
  T* S = I.s[sp][0];
  T* V = I.v[sp][0];
  const T* A = I.acc[sp];
  uint32_t* W = I.w[sp];
  unsigned long long* Qs = I.Qp + (size_t)sp * I.nq;
  const DepLds L = dep_lds();
  DepCache D{L.win, L.hkey, L.hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) *L.wbase = dipic_window_base<T>(I, S, W, R.begin, R.end);
  __syncthreads();
  D.base = *L.wbase;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  // one particle per lane and trip, its loads issued together (a lane past
  // the end reads the range's first particle and drops it); the trip count
  // is uniform over the workgroup (the deposit shuffles across the wave)
  for (uint32_t t = R.begin; t < R.end; t += kBlock) {
    const uint32_t i = t + threadIdx.x;
    const uint32_t ii = i < R.end ? i : R.begin;
    const uint32_t w = i < R.end ? W[ii] : 0u;
    const T v0 = V[ii], s0 = S[ii], b = A[ii];
    uint32_t key = kNoKey;
    unsigned long long q0 = 0ull, q1 = 0ull;
    if (w) {
      T v = v0 + b;
      T s = s0 + v * dt_L;
      bool lost = false;
      const bool ok = wall_rule<T>(reflect, s, v, lost);
      st.alive++;
      if (!ok) {
        st.absorbed++;
        st.lost += lost ? 1u : 0u;
        W[i] = 0u;
      } else {
        S[i] = s;
        V[i] = v;
        cic1d_shares<T>(I.N, s, w, key, q0, q1);
      }
    }
    seg_dep_add(D, Qs, key, q0);
    seg_dep_add(D, Qs, key == kNoKey ? kNoKey : key + 1u, q1);
  }
  __syncthreads();
  dep_flush(D, Qs, I.nq);
  add_stats_row(I.part + (size_t)blockIdx.x * kNStat, st, sp);
}

template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) void k_dipic_correct(InstDev<T> I) {
  if (I.ctr->flags & kFlagNeedRoom) return;   // the predictor did not run this step
  const uint32_t step = I.ctr->step;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  const BlockRange R = dipic_range<T>(I);
  const int sp = R.sp;
  const SpeciesK<T> k = I.sk[sp];
  const bool mcc = MCC && k.mcc != PIC_MCC_NONE;          // uniform
  const bool births = mcc && k.mcc == PIC_MCC_ELECTRON;   // uniform: newborns only from electron impact
  const bool reflect = I.particle_bc == PIC_REFLECT;
  const int N = I.N;
  const T* E = I.E;
  T* S = I.s[sp][0];
  T* V0 = I.v[sp][0];
  T* V1 = I.v[sp][1];
  T* V2 = I.v[sp][2];
  T* A = I.acc[sp];
  uint32_t* W = I.w[sp];
  const uint32_t* ID = I.id[sp];
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
  const DepLds L = dep_lds();
  DepCache D{L.win, L.hkey, L.hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) *L.wbase = dipic_window_base<T>(I, S, W, R.begin, R.end);
  __syncthreads();
  D.base = *L.wbase;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t t = R.begin; t < R.end; t += kBlock) {
    // the particle's loads together (as in the predictor), then the field
    // at its predicted position (the E table is cache resident)
    const uint32_t i = t + threadIdx.x;
    const uint32_t ii = i < R.end ? i : R.begin;
    uint32_t w = i < R.end ? W[ii] : 0u;
    const T s0 = S[ii], v0 = V0[ii], b = A[ii];
    const uint32_t pid = mcc ? ID[ii] : 0u;
    const T g = (w ? s0 : (T)0) * (T)N;
    int ic = (int)floor(g);
    if (ic > N - 1) ic = N - 1;
    const T e0 = E[ic], e1 = E[ic + 1];
    bool birth = false;
    BirthRec<T> rec = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
    uint32_t id = 0u;
    T s = (T)0;
    uint32_t key = kNoKey;
    unsigned long long q0 = 0ull, q1 = 0ull;
    if (w) {
      s = s0;
      T v = v0;
      // E_n+1 at the predicted position, linear between the cell's nodes
      const T fr = g - (T)ic;
      const T dv = k.hqm_dt * (e0 + fr * (e1 - e0));
      v = v + dv;
      s = s + dv * k.dt_L;
      A[i] = (b + dv) * (T)0.5;
      bool lost = false;
      if (!wall_rule<T>(reflect, s, v, lost)) {
        st.absorbed++;
        st.lost += lost ? 1u : 0u;
        W[i] = 0u;
        w = 0u;
      } else {
        if (mcc) {
          id = pid;
          WordStream ws(I.key0, I.key1, id, step);
          const uint32_t r0 = ws.next();
          const uint32_t r1 = ws.next();
          if ((r0 >> 8) < k.tcand) {
            T vy = V1[i], vz = V2[i];
            const uint32_t kind = collision_kind<T>(k, r1, v, vy, vz, st);
            if (kind == kCollElastic) {
              st.elastic++;
              collide_elastic<T>(k, ws, v, vy, vz);
            } else if (kind == kCollIonize) {
              st.ionization++;
              collide_ionize<T>(k, ws, v, vy, vz, rec);
              birth = true;
            } else if (kind == kCollCx) {
              st.cx += collide_cx<T>(k, r1, ws, v, vy, vz, st) ? 1u : 0u;
            }
            if (kind != kCollNone) {
              V1[i] = vy;
              V2[i] = vz;
            }
          }
        }
        S[i] = s;
        V0[i] = v;
        cic1d_shares<T>(N, s, w, key, q0, q1);
      }
    }
    if (births) stage_birth<T>(I, birth, id, 0u, w, s, (T)0, rec);
    seg_dep_add(D, Qs, key, q0);
    seg_dep_add(D, Qs, key == kNoKey ? kNoKey : key + 1u, q1);
    // a newborn pair sits on its parent with the parent's weight (rare:
    // straight to global memory)
    if (births && __ballot(birth) != 0ull) {
      const uint32_t kb = birth ? key : kNoKey;
      const uint32_t kb1 = birth ? key + 1u : kNoKey;
      seg_atomic_add(Qpar, kb, q0);
      seg_atomic_add(Qpar, kb1, q1);
      seg_atomic_add(Qpar + I.nq, kb, q0);
      seg_atomic_add(Qpar + I.nq, kb1, q1);
    }
  }
  __syncthreads();
  dep_flush(D, Qs, I.nq);
  add_stats_row(I.part + (size_t)blockIdx.x * kNStat, st, sp);
}

// v <- v - (q dt / 2m) E(x) with the current field table.
template <class T>
__global__ __launch_bounds__(kBlock) void k_leapfrog_start(InstDev<T> I) {
  for (int sp = 0; sp < I.nspecies; ++sp) {
    const uint32_t count = I.ctr->count[sp];
    const T h = I.sk[sp].hqm_dt;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
      if (!G(I.w[sp])[i]) continue;
      if (I.dim == 1) {
        const T g = G(I.s[sp][0])[i] * (T)I.N;
        int ic = (int)floor(g);
        if (ic > I.N - 1) ic = I.N - 1;
        const T f = g - (T)ic;
        // the step loop's gather: the cell's E (energy-conserving) or linear between nodes
        const T E = I.cell_e ? G(I.E)[ic] : G(I.E)[ic] + f * (G(I.E)[ic + 1] - G(I.E)[ic]);
        G(I.v[sp][0])[i] = G(I.v[sp][0])[i] - h * E;
        if (I.dipic) G(I.acc[sp])[i] = h * E;   // b = (dt/2) a(x_0)
      } else if (I.dim == 3) {
        T e[3];
        gather3d<T>(I, G(I.cell[sp])[i], G(I.s[sp][0])[i], G(I.s[sp][1])[i], G(I.s[sp][2])[i], e);
        for (int a = 0; a < 3; ++a) G(I.v[sp][a])[i] = G(I.v[sp][a])[i] - h * e[a];
      } else {
        T ex, ey;
        if (I.cic_amr) gather_cic<T>(I, G(I.cell[sp])[i], G(I.s[sp][0])[i], G(I.s[sp][1])[i], ex, ey);
        else gather2d<T>(I, G(I.cell[sp])[i], G(I.s[sp][0])[i], G(I.s[sp][1])[i], ex, ey);
        G(I.v[sp][0])[i] = G(I.v[sp][0])[i] - h * ex;
        G(I.v[sp][1])[i] = G(I.v[sp][1])[i] - h * ey;
      }
    }
  }
}

// cell <- leaf containing s (2D), for all live particles of one species.
template <class T>
__global__ __launch_bounds__(kBlock) void k_relocate(InstDev<T> I, int sp) {
  const uint32_t count = I.ctr->count[sp];
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    if (!G(I.w[sp])[i]) continue;
    if (I.dim == 3) {
      G(I.cell[sp])[i] = locate_leaf3(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, (uint32_t)(G(I.s[sp][0])[i] * (T)1024),
                                      (uint32_t)(G(I.s[sp][1])[i] * (T)1024), (uint32_t)(G(I.s[sp][2])[i] * (T)1024),
                                      I.lut_direct != 0);
      continue;
    }
    const uint32_t X = (uint32_t)(G(I.s[sp][0])[i] * (T)65536);
    const uint32_t Y = (uint32_t)(G(I.s[sp][1])[i] * (T)65536);
    G(I.cell[sp])[i] = locate2d<T>(I, X, Y);
  }
}

// ---------------------------------------------------------------------------
// Cloud-in-cell on the quadtree (Sec. 3.1, Fig. 2).  A particle in leaf l
// (level L, side h) is a square cloud of side h centred on it, covering l and
// up to three level-L cells beside it (the direct neighbours on the
// particle's side of l's centre in x and in y, and the diagonal one), with
// the bilinear area fractions in fixed point, F/2 bits per axis.  Where the
// tree is not uniform those cells are ghost cells (ghost cells at +-1 level
// in direct and diagonal neighbours, Sec. 3.1): inside a coarser leaf a ghost
// cell belongs to it; over finer leaves (which follow each other in Morton
// order) it is shared among them by area.  A ghost cell outside the domain is
// folded back across the wall.  The same fractions scatter the charge and
// gather the cell-centred field (the same shape function both ways).
// ---------------------------------------------------------------------------
template <class T>
struct Cloud {
  int32_t cx[4], cy[4];        // centres of own, x-, y- and diagonal cells (16-bit units)
  unsigned long long share[4]; // in units of 2^-F of the particle
  T wt[4];                     // the same fractions in T
  int level;
};

template <class T>
__device__ __forceinline__ Cloud<T> cloud_at(const InstDev<T>& I, uint32_t leaf, T sx, T sy) {
  constexpr int H = FixedPoint<T>::F / 2;
  const uint32_t xy = G(I.leaf_xy)[leaf];
  const int L = (int)G(I.leaf_lv)[leaf];
  const int32_t S = 1 << (16 - L);
  const uint32_t X0 = xy >> 16, Y0 = xy & 0xFFFFu;
  const T sc = (T)(1u << L);
  const T gx = (sx * sc - (T)(X0 >> (16 - L))) - (T)0.5;
  const T gy = (sy * sc - (T)(Y0 >> (16 - L))) - (T)0.5;
  const T ax = gx < (T)0 ? -gx : gx, ay = gy < (T)0 ? -gy : gy;
  const T one = (T)(1u << H);
  const unsigned long long rx = (unsigned long long)rint(ax * one), ry = (unsigned long long)rint(ay * one);
  const unsigned long long o = 1ull << H;
  Cloud<T> c;
  c.level = L;
  const int32_t X = (int32_t)X0 + S / 2, Y = (int32_t)Y0 + S / 2;
  const int32_t Xn = X + (gx >= (T)0 ? S : -S), Yn = Y + (gy >= (T)0 ? S : -S);
  const int32_t xs = (Xn >= 0 && Xn < 65536) ? Xn : X;   // folded back at the walls
  const int32_t ys = (Yn >= 0 && Yn < 65536) ? Yn : Y;
  c.cx[0] = X;  c.cy[0] = Y;
  c.cx[1] = xs; c.cy[1] = Y;
  c.cx[2] = X;  c.cy[2] = ys;
  c.cx[3] = xs; c.cy[3] = ys;
  c.share[0] = (o - rx) * (o - ry);
  c.share[1] = rx * (o - ry);
  c.share[2] = (o - rx) * ry;
  c.share[3] = rx * ry;
  const T fx = (T)rx / one, fy = (T)ry / one;
  c.wt[0] = ((T)1 - fx) * ((T)1 - fy);
  c.wt[1] = fx * ((T)1 - fy);
  c.wt[2] = ((T)1 - fx) * fy;
  c.wt[3] = fx * fy;
  return c;
}

// First leaf of the level-L cell centred at (X, Y): the leaf holding its low
// corner.  If that leaf is at level L or coarser it holds the whole cell
// (coarse = true); else the cell is tiled by it and the leaves after it
// whose keys stay below the cell's end.
template <class T>
__device__ __forceinline__ uint32_t cell_first(const InstDev<T>& I, int32_t X, int32_t Y, int L, bool& coarse,
                                               uint64_t& key_end) {
  const uint32_t S = 1u << (16 - L);
  const uint32_t X0 = (uint32_t)X - S / 2, Y0 = (uint32_t)Y - S / 2;
  const uint32_t f = locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, X0, Y0, I.lut_direct != 0);
  coarse = (int)G(I.leaf_lv)[f] <= L;
  key_end = (uint64_t)morton2(X0, Y0) + ((uint64_t)S * (uint64_t)S);
  return f;
}

template <class T>
__device__ __forceinline__ void gather_cell(const InstDev<T>& I, int32_t X, int32_t Y, int L, T& ex, T& ey) {
  bool coarse;
  uint64_t kend;
  uint32_t l = cell_first(I, X, Y, L, coarse, kend);
  ex = (T)0;
  ey = (T)0;
  if (coarse) {
    ex = ex + G(I.cellE)[2 * l];
    ey = ey + G(I.cellE)[2 * l + 1];
    return;
  }
  for (; l < I.nleaves && (uint64_t)G(I.leaf_key)[l] < kend; ++l) {
    const T f = (T)ldexp(1.0, -2 * ((int)G(I.leaf_lv)[l] - L));
    ex = ex + G(I.cellE)[2 * l] * f;
    ey = ey + G(I.cellE)[2 * l + 1] * f;
  }
}

template <class T>
__device__ __forceinline__ void gather_cic(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T& ex, T& ey) {
  const Cloud<T> c = cloud_at<T>(I, leaf, sx, sy);
  T e0[4], e1[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) gather_cell<T>(I, c.cx[k], c.cy[k], c.level, e0[k], e1[k]);
  ex = ((c.wt[0] * e0[0] + c.wt[1] * e0[1]) + c.wt[2] * e0[2]) + c.wt[3] * e0[3];
  ey = ((c.wt[0] * e1[0] + c.wt[1] * e1[1]) + c.wt[2] * e1[2]) + c.wt[3] * e1[3];
}

// units of charge into the level-L cell centred at (X, Y): to its leaf, or by
// area to the finer leaves tiling it (rounded down; the rest to the first)
template <class T, class Add>
__device__ __forceinline__ void scatter_cell(const InstDev<T>& I, int32_t X, int32_t Y, int L,
                                             unsigned long long units, Add add) {
  bool coarse;
  uint64_t kend;
  const uint32_t f = cell_first(I, X, Y, L, coarse, kend);
  if (coarse) {
    add(f, units);
    return;
  }
  unsigned long long given = 0ull;
  for (uint32_t l = f; l < I.nleaves && (uint64_t)G(I.leaf_key)[l] < kend; ++l) {
    const unsigned long long part = units >> (2 * ((int)G(I.leaf_lv)[l] - L));
    add(l, part);
    given += part;
  }
  add(f, units - given);
}

template <class T, class Add>
__device__ __forceinline__ void scatter_cic(const InstDev<T>& I, uint32_t leaf, T sx, T sy, uint32_t w, Add add) {
  const Cloud<T> c = cloud_at<T>(I, leaf, sx, sy);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (c.share[k]) scatter_cell<T>(I, c.cx[k], c.cy[k], c.level, (unsigned long long)w * c.share[k], add);
}

// The particle loop of a quadtree slot with the cloud-in-cell coupling: one
// particle per lane, in place (gather from the cell-centred field table,
// push, walls, locate, MCC with births, deposit of the cloud).  Workgroups
// take contiguous ranges of a species as k_step does.
template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) void k_step2d_cic(InstDev<T> I, int commit) {
  if (step_blocked<T>(I)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&I.ctr->flags, kFlagNeedRoom);
    return;
  }
  const uint32_t step = I.ctr->step;
  const uint32_t n0 = I.ctr->count[0];
  const uint32_t n1 = I.nspecies == 2 ? I.ctr->count[1] : 0u;
  const uint32_t grid = gridDim.x;
  uint32_t gs = grid;
  if (I.nspecies == 2) {
    gs = (uint32_t)(((uint64_t)grid * n0 + ((uint64_t)n0 + n1) / 2u) / ((uint64_t)n0 + n1 + 1u));
    if (gs < 1u) gs = 1u;
    if (gs > grid - 1u) gs = grid - 1u;
  }
  const int sp = blockIdx.x >= gs ? 1 : 0;
  const uint32_t b = sp == 0 ? blockIdx.x : blockIdx.x - gs;
  const uint32_t nb = sp == 0 ? gs : grid - gs;
  const uint32_t count = sp == 0 ? n0 : n1;
  const uint32_t chunk = ((count + nb - 1u) / nb + kBlock - 1u) / kBlock * kBlock;
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  const uint64_t begin64 = (uint64_t)b * chunk;
  const uint32_t begin = begin64 < count ? (uint32_t)begin64 : count;
  const uint32_t end = (uint64_t)begin + chunk < count ? begin + chunk : count;
  unsigned long long* row = I.part + (size_t)blockIdx.x * kNStat;
  unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
  unsigned long long* Qi = Qpar + I.nq;
  const DepLds Ld = dep_lds();
  DepCache D{Ld.win, Ld.hkey, Ld.hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) {
    const uint32_t c0 = begin < end && G(I.w[sp])[begin] ? G(I.cell[sp])[begin] : 0u;
    *Ld.wbase = c0 > kWin / 2u ? c0 - kWin / 2u : 0u;
  }
  __syncthreads();
  D.base = *Ld.wbase;
  const SpeciesK<T> k = I.sk[sp];
  const bool mcc = MCC && k.mcc != PIC_MCC_NONE;
  const bool reflect = I.particle_bc == PIC_REFLECT;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  auto add_own = [&](uint32_t l, unsigned long long v) { dep_add(D, Qs, l, v); };
  auto add_ion = [&](uint32_t l, unsigned long long v) {
    if (v) gadd(Qi + l, v);
  };
  for (uint32_t base = begin; base < end; base += kBlock) {
    const uint32_t i = base + threadIdx.x;
    uint32_t w = i < end ? G(I.w[sp])[i] : 0u;
    bool live = w != 0u;
    T sx = (T)0, sy = (T)0, vx = (T)0, vy = (T)0, vz = (T)0;
    uint32_t id = 0u, leaf = 0u;
    bool birth = false;
    BirthRec<T> rec;
    if (live) {
      sx = G(I.s[sp][0])[i];
      sy = G(I.s[sp][1])[i];
      vx = G(I.v[sp][0])[i];
      vy = G(I.v[sp][1])[i];
      vz = G(I.v[sp][2])[i];
      id = G(I.id[sp])[i];
      leaf = G(I.cell[sp])[i];
      st.alive++;
      T ex, ey;
      gather_cic<T>(I, leaf, sx, sy, ex, ey);
      vx = vx + k.qm_dt * ex;
      vy = vy + k.qm_dt * ey;
      sx = sx + vx * k.dt_L;
      sy = sy + vy * k.dt_L;
      bool lost = false;
      const bool okx = wall_rule<T>(reflect, sx, vx, lost);
      const bool oky = okx && wall_rule<T>(reflect, sy, vy, lost);
      if (!(okx && oky)) {
        live = false;
        st.absorbed++;
        st.lost += lost ? 1u : 0u;
        G(I.w[sp])[i] = 0u;
      } else {
        leaf = locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, (uint32_t)(sx * (T)65536),
                           (uint32_t)(sy * (T)65536), I.lut_direct != 0);
        if (mcc) {
          WordStream ws(I.key0, I.key1, id, step);
          const uint32_t r0 = ws.next();
          const uint32_t r1 = ws.next();
          if ((r0 >> 8) < k.tcand) {
            const uint32_t kind = collision_kind<T>(k, r1, vx, vy, vz, st);
            if (kind == kCollElastic) {
              collide_elastic<T>(k, ws, vx, vy, vz);
              st.elastic++;
            } else if (kind == kCollIonize) {
              collide_ionize<T>(k, ws, vx, vy, vz, rec);
              birth = true;
              st.ionization++;
            } else if (kind == kCollCx) {
              st.cx += collide_cx<T>(k, r1, ws, vx, vy, vz, st) ? 1u : 0u;
            }
          }
        }
        G(I.s[sp][0])[i] = sx;
        G(I.s[sp][1])[i] = sy;
        G(I.v[sp][0])[i] = vx;
        G(I.v[sp][1])[i] = vy;
        G(I.v[sp][2])[i] = vz;
        G(I.cell[sp])[i] = leaf;
      }
    }
    stage_birth<T>(I, birth, id, leaf, w, sx, sy, rec);
    if (live) scatter_cic<T>(I, leaf, sx, sy, w, add_own);
    if (birth) {   // the newborn electron and ion sit on the parent
      scatter_cic<T>(I, leaf, sx, sy, w, add_own);
      scatter_cic<T>(I, leaf, sx, sy, w, add_ion);
    }
  }
  __syncthreads();
  dep_flush(D, Qs, I.nq);
  add_stats_row(row, st, sp);
  if (commit) last_block_commit(I.ctr, step);
}

// Standalone cloud deposit of the current particles into Q[(step + 1) & 1].
template <class T>
__global__ __launch_bounds__(kBlock) void k_deposit_cic(InstDev<T> I) {
  const uint32_t step = I.ctr->step;
  unsigned long long* Qpar = I.Q + (size_t)((step + 1u) & 1u) * 2u * I.nq;
  for (int sp = 0; sp < I.nspecies; ++sp) {
    unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
    const uint32_t count = I.ctr->count[sp];
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
      const uint32_t w = G(I.w[sp])[i];
      if (!w) continue;
      scatter_cic<T>(I, G(I.cell[sp])[i], G(I.s[sp][0])[i], G(I.s[sp][1])[i], w,
                     [&](uint32_t l, unsigned long long v) {
                       if (v) gadd(Qs + l, v);
                     });
    }
  }
}

// Cell-centred E of each leaf: the mean of its four nodal E values.
template <class T>
__global__ void k_cell_e(const double* corner_e64, uint32_t nleaves, T* cellE) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaves) return;
  const double* c = corner_e64 + (size_t)8 * l;
#pragma unroll
  for (int k = 0; k < 2; ++k) cellE[2 * l + k] = (T)(0.25 * ((c[0 + k] + c[2 + k]) + (c[4 + k] + c[6 + k])));
}

// The field the step's gather gives at n points (test helper).
template <class T>
__global__ void k_gather_points(InstDev<T> I, const double* s, int64_t n, double* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (I.dim == 1) {
    const T x = (T)s[j];
    const T g = x * (T)I.N;
    int ic = (int)floor(g);
    if (ic > I.N - 1) ic = I.N - 1;
    const T f = g - (T)ic;
    out[j] = (double)(I.cell_e ? G(I.E)[ic] : G(I.E)[ic] + f * (G(I.E)[ic + 1] - G(I.E)[ic]));
    return;
  }
  if (I.dim == 3) {
    const T p[3] = {(T)s[3 * j], (T)s[3 * j + 1], (T)s[3 * j + 2]};
    const uint32_t leaf = locate_leaf3(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, (uint32_t)(p[0] * (T)1024),
                                       (uint32_t)(p[1] * (T)1024), (uint32_t)(p[2] * (T)1024), I.lut_direct != 0);
    T e[3];
    gather3d<T>(I, leaf, p[0], p[1], p[2], e);
    for (int a = 0; a < 3; ++a) out[3 * j + a] = (double)e[a];
    return;
  }
  const T sx = (T)s[2 * j], sy = (T)s[2 * j + 1];
  const uint32_t leaf = locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, (uint32_t)(sx * (T)65536),
                                    (uint32_t)(sy * (T)65536), I.lut_direct != 0);
  T ex, ey;
  if (I.cic_amr) gather_cic<T>(I, leaf, sx, sy, ex, ey);
  else gather2d<T>(I, leaf, sx, sy, ex, ey);
  out[2 * j] = (double)ex;
  out[2 * j + 1] = (double)ey;
}

// ---- launchers ----
// A launch whose start and end the runtime writes into t0 / t1 (the
// dispatch's own timestamps) when they are given.
template <typename F, typename... A>
void launch_timed(F kernel, dim3 g, dim3 b, hipStream_t s, hipEvent_t t0, hipEvent_t t1, A... args) {
  if (t0 || t1) hipExtLaunchKernelGGL(kernel, g, b, 0, s, t0, t1, 0, args...);
  else hipLaunchKernelGGL(kernel, g, b, 0, s, args...);
}

template <class T>
hipError_t launch_step(const InstDev<T>& I, hipStream_t s, int grid, bool mcc, int commit, hipEvent_t t0,
                       hipEvent_t t1) {
  if (I.nspecies == 2 && grid < 2) return hipErrorInvalidValue;   // the species split needs two workgroups
  const dim3 g(grid), b(kBlock);
  if (I.dim == 3) {
    if (mcc) launch_timed(k_step3d<T, true>, g, b, s, t0, t1, I, commit);
    else launch_timed(k_step3d<T, false>, g, b, s, t0, t1, I, commit);
  } else if (I.cic_amr) {
    if (mcc) launch_timed(k_step2d_cic<T, true>, g, b, s, t0, t1, I, commit);
    else launch_timed(k_step2d_cic<T, false>, g, b, s, t0, t1, I, commit);
  } else if (I.dim == 1) {
    if (mcc) launch_timed(k_step<T, true, 1, false>, g, b, s, t0, t1, I, commit);
    else launch_timed(k_step<T, false, 1, false>, g, b, s, t0, t1, I, commit);
  } else if (I.lut_direct) {
    if (mcc) launch_timed(k_step<T, true, 2, true>, g, b, s, t0, t1, I, commit);
    else launch_timed(k_step<T, false, 2, true>, g, b, s, t0, t1, I, commit);
  } else {
    if (mcc) launch_timed(k_step<T, true, 2, false>, g, b, s, t0, t1, I, commit);
    else launch_timed(k_step<T, false, 2, false>, g, b, s, t0, t1, I, commit);
  }
  return hipGetLastError();
}
// Workgroups of the step kernel variant that fit on the device at once
// (occupancy per compute unit x compute units), cached per variant (contexts
// driven from several threads may fill the cache at once: same value).
template <class T>
int step_resident_grid(int dim, bool mcc, bool direct) {
  static std::atomic<int> cache[3][2][2] = {};
  std::atomic<int>& slot = cache[dim - 1][mcc ? 1 : 0][direct ? 1 : 0];
  int c = slot.load(std::memory_order_relaxed);
  if (c == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    const void* fn;
    if (dim == 3) fn = mcc ? (const void*)k_step3d<T, true> : (const void*)k_step3d<T, false>;
    else if (dim == 1) fn = mcc ? (const void*)k_step<T, true, 1, false> : (const void*)k_step<T, false, 1, false>;
    else if (direct) fn = mcc ? (const void*)k_step<T, true, 2, true> : (const void*)k_step<T, false, 2, true>;
    else fn = mcc ? (const void*)k_step<T, true, 2, false> : (const void*)k_step<T, false, 2, false>;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess)
      return 2048;
    c = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    slot.store(c, std::memory_order_relaxed);
  }
  return c;
}

template <class T>
hipError_t launch_step1d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                 unsigned long long* bpart, hipStream_t s, int grid, bool mcc) {
  if (mcc) hipLaunchKernelGGL((k_step1d_batched<T, true>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  else hipLaunchKernelGGL((k_step1d_batched<T, false>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  return hipGetLastError();
}
template <class T>
hipError_t launch_step2d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                 unsigned long long* bpart, hipStream_t s, int grid, bool mcc) {
  if (mcc) hipLaunchKernelGGL((k_step2d_batched<T, true>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  else hipLaunchKernelGGL((k_step2d_batched<T, false>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births(const InstDev<T>& I, hipStream_t s, bool binned) {
  if (binned) {
    hipLaunchKernelGGL(k_birth_bin<T>, dim3(256), dim3(kBlock), 0, s, I);
    hipLaunchKernelGGL(k_birth_binscan<T>, dim3(1), dim3(1024), 0, s, I);
    hipLaunchKernelGGL(k_birth_scatter<T>, dim3(512), dim3(kBlock), 0, s, I);
    hipLaunchKernelGGL(k_birth_rank_binned<T>, dim3(1024), dim3(kBlock), 0, s, I);
  } else {
    hipLaunchKernelGGL(k_birth_rank<T>, dim3(kRankBlocksPlain), dim3(kBlock), 0, s, I);
  }
  hipLaunchKernelGGL(k_birth_write<T>, dim3(kWriteBlocks), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births_batched(const InstDev<T>* I, int ninst, hipStream_t s, double pair_births,
                                 double bin_births) {
  // workgroups per instance from the births expected per step (the kernels
  // loop over their work, so any count is correct; idle workgroups only cost
  // dispatch time): pairwise ranking work items are (births / 1024) x
  // (births / 256)
  if (pair_births >= 0.0) {
    const double nb = pair_births;
    const double items = (nb / (kRankPer * kBlock) + 1.0) * (nb / kRankChunk + 1.0);
    const int rank_blocks = (int)std::min<double>(kRankBlocks, std::max(4.0, items / 2.0));
    hipLaunchKernelGGL(k_birth_rank_batched<T>, dim3(rank_blocks, ninst), dim3(kBlock), 0, s, I);
  }
  if (bin_births >= 0.0) {
    const double nb = bin_births;
    const int hist_blocks = (int)std::min<double>(64.0, nb / 4096.0 + 1.0);   // LDS histogram per 4096 births
    const int per = (int)std::min<double>(512.0, std::max(8.0, nb / kBlock + 1.0));
    hipLaunchKernelGGL(k_birth_bin_batched<T>, dim3(hist_blocks, ninst), dim3(kBlock), 0, s, I);
    hipLaunchKernelGGL(k_birth_binscan_batched<T>, dim3(1, ninst), dim3(1024), 0, s, I);
    hipLaunchKernelGGL(k_birth_scatter_batched<T>, dim3(per, ninst), dim3(kBlock), 0, s, I);
    hipLaunchKernelGGL(k_birth_rank_binned_batched<T>, dim3(per, ninst), dim3(kBlock), 0, s, I);
  }
  const double nb = std::max(pair_births, bin_births);
  const int write_blocks = (int)std::min<double>(kWriteBlocks, std::max(1.0, nb / kBlock + 1.0));
  hipLaunchKernelGGL(k_birth_write_batched<T>, dim3(write_blocks, ninst), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_commit(const InstDev<T>& I, hipStream_t s) {
  hipLaunchKernelGGL(k_commit<T>, dim3(1), dim3(64), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_commit_batched(const InstDev<T>* I, int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_batched<T>, dim3(ninst), dim3(64), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_stats_reduce(const InstDev<T>* I, int ninst, unsigned long long* rows, const uint32_t* row_begin,
                               uint32_t nrows_plain, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce<T>, dim3(ninst), dim3(kBlock), 0, s, I, rows, row_begin, nrows_plain);
  return hipGetLastError();
}
template <class T>
hipError_t launch_deposit(const InstDev<T>& I, hipStream_t s, int grid) {
  if (I.cic_amr) hipLaunchKernelGGL(k_deposit_cic<T>, dim3(grid), dim3(kBlock), 0, s, I);
  else hipLaunchKernelGGL(k_deposit<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cell_e(const double* corner_e64, uint32_t nleaves, T* cellE, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_e<T>, dim3(ceil_div(nleaves, kBlock)), dim3(kBlock), 0, s, corner_e64, nleaves, cellE);
  return hipGetLastError();
}
template <class T>
hipError_t launch_gather_points(const InstDev<T>& I, const double* pts, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_points<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, I, pts, n, out);
  return hipGetLastError();
}
template <class T>
hipError_t launch_leapfrog_start(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_leapfrog_start<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_dipic_predict(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_dipic_predict<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_dipic_correct(const InstDev<T>& I, hipStream_t s, int grid, bool mcc) {
  if (mcc) hipLaunchKernelGGL((k_dipic_correct<T, true>), dim3(grid), dim3(kBlock), 0, s, I);
  else hipLaunchKernelGGL((k_dipic_correct<T, false>), dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_relocate(const InstDev<T>& I, int species, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_relocate<T>, dim3(grid), dim3(kBlock), 0, s, I, species);
  return hipGetLastError();
}

#define PIC_INSTANTIATE(T)                                                                                 \
  template hipError_t launch_step<T>(const InstDev<T>&, hipStream_t, int, bool, int, hipEvent_t, hipEvent_t);                                                     \
  template int step_resident_grid<T>(int, bool, bool);                      \
  template hipError_t launch_step1d_batched<T>(const InstDev<T>*, const WorkItem*, uint32_t,               \
                                               unsigned long long*, hipStream_t, int, bool);               \
  template hipError_t launch_step2d_batched<T>(const InstDev<T>*, const WorkItem*, uint32_t,               \
                                               unsigned long long*, hipStream_t, int, bool);               \
  template hipError_t launch_births<T>(const InstDev<T>&, hipStream_t, bool);                              \
  template hipError_t launch_births_batched<T>(const InstDev<T>*, int, hipStream_t, double, double);       \
  template hipError_t launch_commit<T>(const InstDev<T>&, hipStream_t);                                    \
  template hipError_t launch_commit_batched<T>(const InstDev<T>*, int, hipStream_t);                       \
  template hipError_t launch_stats_reduce<T>(const InstDev<T>*, int, unsigned long long*, const uint32_t*, \
                                             uint32_t, hipStream_t);                                       \
  template hipError_t launch_deposit<T>(const InstDev<T>&, hipStream_t, int);                              \
  template hipError_t launch_cell_e<T>(const double*, uint32_t, T*, hipStream_t);                          \
  template hipError_t launch_gather_points<T>(const InstDev<T>&, const double*, int64_t, double*, hipStream_t); \
  template hipError_t launch_leapfrog_start<T>(const InstDev<T>&, hipStream_t, int);                       \
  template hipError_t launch_relocate<T>(const InstDev<T>&, int, hipStream_t, int);                        \
  template hipError_t launch_dipic_predict<T>(const InstDev<T>&, hipStream_t, int);                        \
  template hipError_t launch_dipic_correct<T>(const InstDev<T>&, hipStream_t, int, bool);
PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

}  // namespace pic
