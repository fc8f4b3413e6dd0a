// Particle-loop kernels of the ES-PIC step (arXiv:1604.07713, Sec. 3, 3.1, 4.3):
// gather E at the particle, leapfrog push, wall rule, locate the cell,
// null-collision MCC with ionization births, charge deposit.
//
// One lane per particle.  Particles of a species are stored as structure of
// arrays; when they are ordered by cell, neighbouring lanes read the same
// field-table entries and deposit into the same cell, so a wave's run of
// equal cells becomes a single 64-bit integer atomic (seg_atomic_add).  The
// deposit is integer (64-bit fixed point), hence exact and independent of the
// order in which lanes and waves add.
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
// leaves the domain (absorbed, or reflected but still outside).
template <class T>
__device__ __forceinline__ bool wall_rule(int bc, T& s, T& v, bool& lost) {
  if (s >= (T)0 && s < (T)1) return true;
  if (bc == PIC_ABSORB) return false;
  if (s < (T)0) {
    s = -s;
    v = -v;
  } else if (s >= (T)1) {
    s = (T)2 - s;
    v = -v;
    if (s == (T)1) s = (T)1 - (T)(sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16);
  }
  if (s >= (T)0 && s < (T)1) return true;
  lost = true;
  return false;
}

// Null-collision MCC for one particle (v in registers; vy/vz already loaded).
// Returns true if an ionization produced a birth (rec filled).
template <class T>
__device__ __forceinline__ bool collide(const InstDev<T>& I, const SpeciesK<T>& k, uint32_t pid, uint32_t step,
                                        uint32_t r1, WordStream& ws, T& vx, T& vy, T& vz, LStat& st,
                                        BirthRec<T>& rec) {
  const T u1 = unit_uniform<T>(r1);
  if (k.mcc == PIC_MCC_ELECTRON) {
    const T v2 = (vx * vx + vy * vy) + vz * vz;
    st.viol += (v2 > k.vmax2) ? 1u : 0u;
    const T vmag = sqrt(v2);
    const T x_el = k.a_el * vmag;
    if (u1 < x_el) {
      T dx, dy, dz;
      isotropic<T>(ws, dx, dy, dz);
      const T vd = (vx * dx + vy * dy) + vz * dz;
      T vp2 = v2 - k.mu2 * (v2 - vmag * vd);
      if (vp2 < (T)0) vp2 = (T)0;
      const T vpm = sqrt(vp2);
      vx = vpm * dx;
      vy = vpm * dy;
      vz = vpm * dz;
      st.elastic++;
      return false;
    }
    if (v2 >= k.v_iz2 && u1 < x_el + k.a_iz * vmag) {
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
      st.ionization++;
      return true;
    }
    return false;
  }
  // ion charge exchange with a gas atom drawn from the gas Maxwellian
  const T n0 = k.v_thg * normal12<T>(ws);
  const T n1 = k.v_thg * normal12<T>(ws);
  const T n2 = k.v_thg * normal12<T>(ws);
  const T dx = vx - n0, dy = vy - n1, dz = vz - n2;
  const T g = sqrt((dx * dx + dy * dy) + dz * dz);
  st.viol += (g > k.gmax) ? 1u : 0u;
  if (u1 < k.a_cx * g) {
    vx = n0;
    vy = n1;
    vz = n2;
    st.cx++;
  }
  return false;
}

// Stage a birth: slot from one atomic per wave.
template <class T>
__device__ __forceinline__ void stage_birth(const InstDev<T>& I, bool birth, uint32_t pid, uint32_t cell, uint32_t w,
                                            T s0, T s1, const BirthRec<T>& rec) {
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
  if (I.dim == 2) G(I.br.s[1])[slot] = s1;
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

// ---------------------------------------------------------------------------
// Deposit pre-aggregation: each workgroup owns a window of kWin consecutive
// cells in LDS (its particles are a contiguous, cell-ordered range, so their
// cells cluster); deposits inside the window are LDS atomics, the rest go
// straight to global memory, and the window is flushed once per workgroup.
// ---------------------------------------------------------------------------
constexpr uint32_t kWin = 1024;
constexpr uint32_t kWinMargin = 128;
constexpr uint32_t kHash = 512;      // open-addressed LDS table for cells outside the window
constexpr uint32_t kHashProbe = 8;

struct DepCache {
  unsigned long long* win;     // [kWin]
  uint32_t* hkey;              // [kHash], kNoKey = empty
  unsigned long long* hval;    // [kHash]
  uint32_t base;
};

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
    if (v && D.base + j < nq) gadd(g + D.base + j, v);
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

// Particle state loaded for one lane.  Loads are issued unconditionally and
// one tile ahead (software pipelining), so the latency of the particle
// arrays overlaps the work on the previous tile.
template <class T>
struct PState {
  uint32_t w, cell;
  T s0, s1, v0, v1;
};

template <class T, int DIM>
__device__ __forceinline__ PState<T> load_particle(const SpPtr<T>& P, uint32_t i, bool valid) {
  PState<T> p;
  p.w = 0u;
  p.cell = 0u;
  p.s0 = p.s1 = p.v0 = p.v1 = (T)0;
  if (valid) {
    p.w = *at(P.w, i);
    p.s0 = *at(P.s0, i);
    p.v0 = *at(P.v0, i);
    if (DIM == 2) {
      p.cell = *at(P.cell, i);
      p.s1 = *at(P.s1, i);
      p.v1 = *at(P.v1, i);
    }
  }
  return p;
}

template <class T, bool MCC>
__device__ __forceinline__ void particle1d(const InstDev<T>& I, const SpPtr<T>& P, int sp, uint32_t i, PState<T> p,
                                           uint32_t step,
                                           unsigned long long* Qpar, DepCache& D,
                                           LStat& st) {
  const SpeciesK<T>& k = I.sk[sp];
  const int N = I.N;
  const T Nt = (T)N;
  uint32_t w = p.w;
  bool birth = false;
  BirthRec<T> rec;
  T s = p.s0;
  uint32_t pid = 0;
  if (w != 0u) {
    st.alive++;
    T vx = p.v0;
    {
      const T g = s * Nt;
      int ic = (int)floor(g);
      if (ic > N - 1) ic = N - 1;
      const T f = g - (T)ic;
      const T e0 = *at(I.E, (uint32_t)ic), e1 = *at(I.E, (uint32_t)ic + 1u);
      const T E = e0 + f * (e1 - e0);
      vx = vx + k.qm_dt * E;
      s = s + vx * k.dt_L;
    }
    bool lost = false;
    if (!wall_rule<T>(I.particle_bc, s, vx, lost)) {
      st.absorbed++;
      st.lost += lost ? 1u : 0u;
      *at(P.w, i) = 0u;
      w = 0u;
    } else {
      if (MCC && k.mcc != PIC_MCC_NONE) {
        pid = *at(P.id, i);
        WordStream ws(I.key0, I.key1, pid, step);
        const uint32_t r0 = ws.next();
        const uint32_t r1 = ws.next();
        if ((r0 >> 8) < k.tcand) {
          T vy = *at(P.v1, i), vz = *at(P.v2, i);
          birth = collide<T>(I, k, pid, step, r1, ws, vx, vy, vz, st, rec);
          *at(P.v1, i) = vy;
          *at(P.v2, i) = vz;
        }
      }
      *at(P.s0, i) = s;
      *at(P.v0, i) = vx;
      // CIC shares in 64-bit fixed point
      const T g = s * Nt;
      int ic = (int)floor(g);
      if (ic > N - 1) ic = N - 1;
      const T f = g - (T)ic;
      const unsigned long long r = (unsigned long long)(long long)rint(f * (T)(1ull << FixedPoint<T>::F));
      const unsigned long long one = 1ull << FixedPoint<T>::F;
      const unsigned long long mult = birth ? 2ull : 1ull;
      unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
      dep_add(D, Qs, (uint32_t)ic, mult * (unsigned long long)w * (one - r));
      dep_add(D, Qs, (uint32_t)ic + 1u, mult * (unsigned long long)w * r);
      if (MCC && birth) {   // the newborn ion sits on the parent
        unsigned long long* Qi = Qpar + I.nq;
        if (one - r) gadd(Qi + ic, (unsigned long long)w * (one - r));
        if (r) gadd(Qi + ic + 1, (unsigned long long)w * r);
      }
    }
  }
  if (MCC) stage_birth<T>(I, birth, pid, 0u, w, s, (T)0, rec);
}

// ---------------------------------------------------------------------------
// 2D quadtree: one particle per lane
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ uint32_t locate2d(const InstDev<T>& I, uint32_t X, uint32_t Y) {
  return locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, X, Y, I.lut_direct != 0);
}

template <class T>
__device__ __forceinline__ void gather2d(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T& ex, T& ey) {
  const uint32_t xy = *at(I.leaf_xy, leaf);
  const int lv = *at(I.leaf_lv, leaf);
  const int sh = kKeyBits - lv;
  const T sc = (T)(1u << lv);
  const T xi = sx * sc - (T)((xy >> 16) >> sh);
  const T eta = sy * sc - (T)((xy & 0xFFFFu) >> sh);
  const T w00 = ((T)1 - xi) * ((T)1 - eta);
  const T w10 = xi * ((T)1 - eta);
  const T w01 = ((T)1 - xi) * eta;
  const T w11 = xi * eta;
  const gptr<const T> c = at(I.E, leaf * 8u);
  ex = ((w00 * c[0] + w10 * c[2]) + w01 * c[4]) + w11 * c[6];
  ey = ((w00 * c[1] + w10 * c[3]) + w01 * c[5]) + w11 * c[7];
}

template <class T, bool MCC>
__device__ __forceinline__ void particle2d(const InstDev<T>& I, const SpPtr<T>& P, int sp, uint32_t i, PState<T> p,
                                           uint32_t step,
                                           unsigned long long* Qpar, DepCache& D,
                                           LStat& st) {
  const SpeciesK<T>& k = I.sk[sp];
  uint32_t w = p.w;
  bool birth = false;
  BirthRec<T> rec;
  T sx = p.s0, sy = p.s1;
  uint32_t pid = 0, leaf = p.cell;
  if (w != 0u) {
    st.alive++;
    T vx = p.v0;
    T vy = p.v1;
    T ex, ey;
    gather2d<T>(I, leaf, sx, sy, ex, ey);
    vx = vx + k.qm_dt * ex;
    vy = vy + k.qm_dt * ey;
    sx = sx + vx * k.dt_L;
    sy = sy + vy * k.dt_L;
    bool lost = false;
    const bool okx = wall_rule<T>(I.particle_bc, sx, vx, lost);
    const bool ok = okx && wall_rule<T>(I.particle_bc, sy, vy, lost);
    if (!ok) {
      st.absorbed++;
      st.lost += lost ? 1u : 0u;
      *at(P.w, i) = 0u;
      w = 0u;
    } else {
      const uint32_t X = (uint32_t)(sx * (T)65536);
      const uint32_t Y = (uint32_t)(sy * (T)65536);
      const uint32_t xy = *at(I.leaf_xy, leaf);
      const int sh = kKeyBits - (int)*at(I.leaf_lv, leaf);
      if ((X >> sh) != ((xy >> 16) >> sh) || (Y >> sh) != ((xy & 0xFFFFu) >> sh)) leaf = locate2d<T>(I, X, Y);
      if (MCC && k.mcc != PIC_MCC_NONE) {
        pid = *at(P.id, i);
        WordStream ws(I.key0, I.key1, pid, step);
        const uint32_t r0 = ws.next();
        const uint32_t r1 = ws.next();
        if ((r0 >> 8) < k.tcand) {
          T vz = *at(P.v2, i);
          birth = collide<T>(I, k, pid, step, r1, ws, vx, vy, vz, st, rec);
          *at(P.v2, i) = vz;
        }
      }
      *at(P.s0, i) = sx;
      *at(P.s1, i) = sy;
      *at(P.v0, i) = vx;
      *at(P.v1, i) = vy;
      if (leaf != p.cell) *at(P.cell, i) = leaf;
      dep_add(D, Qpar + (size_t)sp * I.nq, leaf, (birth ? 2ull : 1ull) * (unsigned long long)w);
      if (MCC && birth) gadd(Qpar + I.nq + leaf, (unsigned long long)w);
    }
  }
  if (MCC) stage_birth<T>(I, birth, pid, leaf, w, sx, sy, rec);
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

template <class T, bool MCC, int DIM>
__device__ __forceinline__ void run_range(const InstDev<T>& I, int sp, uint32_t begin, uint32_t end, uint32_t step,
                                          unsigned long long* Qpar, unsigned long long* row) {
  if (begin >= end) return;   // uniform: the whole workgroup has no particles here
  __shared__ unsigned long long win[kWin];
  __shared__ uint32_t hkey[kHash];
  __shared__ unsigned long long hval[kHash];
  __shared__ uint32_t wbase_s;
  const SpPtr<T> P = species_ptrs<T>(I, sp);
  DepCache D{win, hkey, hval, 0u};
  dep_zero(D);
  if (threadIdx.x == 0) {
    uint32_t c0 = 0;
    if (begin < end) c0 = DIM == 2 ? *at(P.cell, begin) : cell1d<T>(I, *at(P.s0, begin));
    wbase_s = c0 > kWinMargin ? c0 - kWinMargin : 0u;
  }
  __syncthreads();
  D.base = wbase_s;
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  uint32_t i = begin + threadIdx.x;
  PState<T> cur = load_particle<T, DIM>(P, i, i < end);
  for (uint32_t base = begin; base < end; base += kBlock) {
    const uint32_t inext = i + kBlock;
    const PState<T> nxt = load_particle<T, DIM>(P, inext, inext < end);
    if (DIM == 2) particle2d<T, MCC>(I, P, sp, i, cur, step, Qpar, D, st);
    else particle1d<T, MCC>(I, P, sp, i, cur, step, Qpar, D, st);
    cur = nxt;
    i = inext;
  }
  __syncthreads();
  dep_flush(D, Qpar + (size_t)sp * I.nq, I.nq);
  add_stats_row(row, st, sp);
  __syncthreads();
}

// Plain launch over one instance: workgroups [0, gs) own consecutive chunks
// of species 0, [gs, grid) of species 1.
template <class T, bool MCC, int DIM>
__global__ __launch_bounds__(kBlock) void k_step(InstDev<T> I, int gs, uint32_t chunk0, uint32_t chunk1, int commit) {
  const int sp = (I.nspecies == 2 && (int)blockIdx.x >= gs) ? 1 : 0;
  const uint32_t b = sp == 0 ? blockIdx.x : blockIdx.x - (uint32_t)gs;
  const uint32_t chunk = sp == 0 ? chunk0 : chunk1;
  const uint32_t step = I.ctr->step;
  const uint32_t count = I.ctr->count[sp];
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  const uint32_t begin = b * chunk;
  const uint32_t end = begin + chunk < count ? begin + chunk : count;
  run_range<T, MCC, DIM>(I, sp, begin, end, step, Qpar, I.part + (size_t)blockIdx.x * kNStat);
  if (commit) last_block_commit(I.ctr, step);
}

// Batched 1D launch: a persistent grid walks a list of (instance, species,
// range) work items; per-instance constants come from the descriptor table.
template <class T, bool MCC>
__global__ __launch_bounds__(kBlock) void k_step1d_batched(const InstDev<T>* __restrict__ insts,
                                                           const WorkItem* __restrict__ items, uint32_t nitems,
                                                           unsigned long long* bpart) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const InstDev<T>& I = insts[wi.inst];
    const int sp = (int)wi.species;
    const uint32_t step = I.ctr->step;
    const uint32_t count = I.ctr->count[sp];
    const uint32_t end = wi.end < count ? wi.end : count;
    unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
    if (wi.begin == 0 && sp == 0) zero_other_parity(I.Q, I.nq, step, I.nspecies, threadIdx.x, kBlock);
    run_range<T, MCC, 1>(I, sp, wi.begin, end, step, Qpar, bpart + (size_t)it * kNStat);
  }
}

// ---------------------------------------------------------------------------
// Births: rank by parent id (count of smaller staged parent ids), then append
// the electron at count[0] + r with id next_id + 2r and the ion at
// count[1] + r with id next_id + 2r + 1.
// ---------------------------------------------------------------------------
template <class T>
__device__ void births_body(const InstDev<T>& I, uint32_t first_block, uint32_t nblocks) {
  __shared__ uint32_t sh[1024];
  const uint32_t nb = I.ctr->nbirths;
  if (nb == 0u) return;
  const uint32_t c0 = I.ctr->count[0], c1 = I.ctr->count[1], nid = I.ctr->next_id;
  const bool cap_ok = (uint64_t)c0 + nb <= I.cap[0] && (uint64_t)c1 + nb <= I.cap[1] && nb <= I.birth_cap;
  const bool id_ok = (uint64_t)nid + 2ull * nb <= 0xFFFFFFFFull;
  if (!cap_ok || !id_ok) {
    if (threadIdx.x == 0 && first_block == 0)
      atomicOr(&I.ctr->flags, (!cap_ok ? kFlagBirthOverflow : 0u) | (!id_ok ? kFlagIdOverflow : 0u));
    return;
  }
  for (uint32_t ib = first_block * kBlock; ib < nb; ib += nblocks * kBlock) {
    const uint32_t i = ib + threadIdx.x;
    const uint32_t mine = i < nb ? I.br.parent[i] : 0xFFFFFFFFu;
    uint32_t r = 0;
    for (uint32_t jb = 0; jb < nb; jb += 1024u) {
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < 1024u && jb + t < nb; t += kBlock) sh[t] = I.br.parent[jb + t];
      __syncthreads();
      const uint32_t lim = (nb - jb) < 1024u ? (nb - jb) : 1024u;
      for (uint32_t j = 0; j < lim; ++j) r += (sh[j] < mine) ? 1u : 0u;
    }
    if (i < nb) {
      const uint32_t pe = c0 + r, pi = c1 + r;
      const uint32_t w = I.br.w[i];
      I.s[0][0][pe] = I.br.s[0][i];
      I.s[1][0][pi] = I.br.s[0][i];
      if (I.dim == 2) {
        I.s[0][1][pe] = I.br.s[1][i];
        I.s[1][1][pi] = I.br.s[1][i];
        I.cell[0][pe] = I.br.cell[i];
        I.cell[1][pi] = I.br.cell[i];
      }
      for (int c = 0; c < 3; ++c) {
        I.v[0][c][pe] = I.br.ve[c][i];
        I.v[1][c][pi] = I.br.vi[c][i];
      }
      I.w[0][pe] = w;
      I.w[1][pi] = w;
      I.id[0][pe] = nid + 2u * r;
      I.id[1][pi] = nid + 2u * r + 1u;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_births(InstDev<T> I) { births_body<T>(I, blockIdx.x, gridDim.x); }

// grid (per_inst, ninst): blockIdx.y selects the instance, blockIdx.x the
// share of its births
template <class T>
__global__ __launch_bounds__(kBlock) void k_births_batched(const InstDev<T>* insts) {
  births_body<T>(insts[blockIdx.y], blockIdx.x, gridDim.x);
}

// Commit a step after the births kernel: append births to the counts,
// advance the step index.  One thread.
template <class T>
__device__ void commit_body(const InstDev<T>& I) {
  if (threadIdx.x == 0) {
    Counters* c = I.ctr;
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
        const T E = G(I.E)[ic] + f * (G(I.E)[ic + 1] - G(I.E)[ic]);
        G(I.v[sp][0])[i] = G(I.v[sp][0])[i] - h * E;
      } else {
        T ex, ey;
        gather2d<T>(I, G(I.cell[sp])[i], G(I.s[sp][0])[i], G(I.s[sp][1])[i], ex, ey);
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
    const uint32_t X = (uint32_t)(G(I.s[sp][0])[i] * (T)65536);
    const uint32_t Y = (uint32_t)(G(I.s[sp][1])[i] * (T)65536);
    G(I.cell[sp])[i] = locate2d<T>(I, X, Y);
  }
}

// ---- launchers ----
template <class T>
static int species_split(const InstDev<T>& I, int grid) {
  if (I.nspecies < 2) return grid;
  const double f = (double)I.cap[0] / ((double)I.cap[0] + (double)I.cap[1] + 1.0);
  int gs = (int)(grid * f + 0.5);
  if (gs < 1) gs = 1;
  if (gs > grid - 1) gs = grid - 1;
  return gs;
}

template <class T>
hipError_t launch_step(const InstDev<T>& I, hipStream_t s, int grid, bool mcc, int commit) {
  const int gs = species_split(I, grid);
  const int g0 = gs, g1 = I.nspecies == 2 ? grid - gs : 1;
  uint32_t c0 = (ceil_div(I.cap[0], (uint32_t)g0) + kBlock - 1) / kBlock * kBlock;
  uint32_t c1 = (ceil_div(I.cap[1] ? I.cap[1] : 1u, (uint32_t)g1) + kBlock - 1) / kBlock * kBlock;
  if (c0 < kBlock) c0 = kBlock;
  if (c1 < kBlock) c1 = kBlock;
  if (I.dim == 1) {
    if (mcc) hipLaunchKernelGGL((k_step<T, true, 1>), dim3(grid), dim3(kBlock), 0, s, I, gs, c0, c1, commit);
    else hipLaunchKernelGGL((k_step<T, false, 1>), dim3(grid), dim3(kBlock), 0, s, I, gs, c0, c1, commit);
  } else {
    if (mcc) hipLaunchKernelGGL((k_step<T, true, 2>), dim3(grid), dim3(kBlock), 0, s, I, gs, c0, c1, commit);
    else hipLaunchKernelGGL((k_step<T, false, 2>), dim3(grid), dim3(kBlock), 0, s, I, gs, c0, c1, commit);
  }
  return hipGetLastError();
}
template <class T>
hipError_t launch_step1d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                 unsigned long long* bpart, hipStream_t s, int grid, bool mcc) {
  if (mcc) hipLaunchKernelGGL((k_step1d_batched<T, true>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  else hipLaunchKernelGGL((k_step1d_batched<T, false>), dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_births<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births_batched(const InstDev<T>* I, int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_births_batched<T>, dim3(32, ninst), dim3(kBlock), 0, s, I);
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
  hipLaunchKernelGGL(k_deposit<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_leapfrog_start(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_leapfrog_start<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_relocate(const InstDev<T>& I, int species, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_relocate<T>, dim3(grid), dim3(kBlock), 0, s, I, species);
  return hipGetLastError();
}

#define PIC_INSTANTIATE(T)                                                                                 \
  template hipError_t launch_step<T>(const InstDev<T>&, hipStream_t, int, bool, int);                      \
  template hipError_t launch_step1d_batched<T>(const InstDev<T>*, const WorkItem*, uint32_t,               \
                                               unsigned long long*, hipStream_t, int, bool);               \
  template hipError_t launch_births<T>(const InstDev<T>&, hipStream_t, int);                               \
  template hipError_t launch_births_batched<T>(const InstDev<T>*, int, hipStream_t);                       \
  template hipError_t launch_commit<T>(const InstDev<T>&, hipStream_t);                                    \
  template hipError_t launch_commit_batched<T>(const InstDev<T>*, int, hipStream_t);                       \
  template hipError_t launch_stats_reduce<T>(const InstDev<T>*, int, unsigned long long*, const uint32_t*, \
                                             uint32_t, hipStream_t);                                       \
  template hipError_t launch_deposit<T>(const InstDev<T>&, hipStream_t, int);                              \
  template hipError_t launch_leapfrog_start<T>(const InstDev<T>&, hipStream_t, int);                       \
  template hipError_t launch_relocate<T>(const InstDev<T>&, int, hipStream_t, int);
PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

}  // namespace pic
