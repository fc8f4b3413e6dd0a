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
  I.br.parent[slot] = pid;
  I.br.cell[slot] = cell;
  I.br.w[slot] = w;
  I.br.s[0][slot] = s0;
  if (I.dim == 2) I.br.s[1][slot] = s1;
  I.br.ve[0][slot] = rec.ve0;
  I.br.ve[1][slot] = rec.ve1;
  I.br.ve[2][slot] = rec.ve2;
  I.br.vi[0][slot] = rec.vi0;
  I.br.vi[1][slot] = rec.vi1;
  I.br.vi[2][slot] = rec.vi2;
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
// 1D: one tile of kBlock particles of species sp.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void tile1d(const InstDev<T>& I, int sp, uint32_t i, uint32_t limit, uint32_t step,
                                       unsigned long long* Qpar, LStat& st) {
  const SpeciesK<T>& k = I.sk[sp];
  const int N = I.N;
  const T Nt = (T)N;
  const bool valid = i < limit;
  uint32_t w = valid ? I.w[sp][i] : 0u;
  uint32_t key0 = kNoKey, key1 = kNoKey;
  unsigned long long q0 = 0ull, q1 = 0ull;
  bool birth = false;
  BirthRec<T> rec;
  T s = (T)0;
  uint32_t pid = 0;
  if (w != 0u) {
    st.alive++;
    s = I.s[sp][0][i];
    T vx = I.v[sp][0][i];
    {
      const T g = s * Nt;
      int ic = (int)floor(g);
      if (ic > N - 1) ic = N - 1;
      const T f = g - (T)ic;
      const T e0 = I.E[ic], e1 = I.E[ic + 1];
      const T E = e0 + f * (e1 - e0);
      vx = vx + k.qm_dt * E;
      s = s + vx * k.dt_L;
    }
    bool lost = false;
    if (!wall_rule<T>(I.particle_bc, s, vx, lost)) {
      st.absorbed++;
      st.lost += lost ? 1u : 0u;
      I.w[sp][i] = 0u;
      w = 0u;
    } else {
      if (k.mcc != PIC_MCC_NONE) {
        pid = I.id[sp][i];
        WordStream ws(I.key0, I.key1, pid, step);
        const uint32_t r0 = ws.next();
        const uint32_t r1 = ws.next();
        if ((r0 >> 8) < k.tcand) {
          T vy = I.v[sp][1][i], vz = I.v[sp][2][i];
          birth = collide<T>(I, k, pid, step, r1, ws, vx, vy, vz, st, rec);
          I.v[sp][1][i] = vy;
          I.v[sp][2][i] = vz;
        }
      }
      I.s[sp][0][i] = s;
      I.v[sp][0][i] = vx;
      // CIC shares in 64-bit fixed point
      const T g = s * Nt;
      int ic = (int)floor(g);
      if (ic > N - 1) ic = N - 1;
      const T f = g - (T)ic;
      const unsigned long long r = (unsigned long long)(long long)rint(f * (T)(1ull << FixedPoint<T>::F));
      const unsigned long long one = 1ull << FixedPoint<T>::F;
      const unsigned long long mult = birth ? 2ull : 1ull;
      key0 = (uint32_t)ic;
      key1 = (uint32_t)ic + 1u;
      q0 = mult * (unsigned long long)w * (one - r);
      q1 = mult * (unsigned long long)w * r;
      if (birth) {   // the newborn ion sits on the parent
        unsigned long long* Qi = Qpar + I.nq;
        if (one - r) atomicAdd(Qi + ic, (unsigned long long)w * (one - r));
        if (r) atomicAdd(Qi + ic + 1, (unsigned long long)w * r);
      }
    }
  }
  stage_birth<T>(I, birth, pid, 0u, w, s, (T)0, rec);
  unsigned long long* Qs = Qpar + (size_t)sp * I.nq;
  seg_atomic_add(Qs, key0, q0);
  seg_atomic_add(Qs, key1, q1);
}

// Per-block sum of the per-lane counters into one row of a partial-stats
// table (plain writes, no atomics; the commit kernel adds the rows up).
__device__ __forceinline__ void write_stats_row(unsigned long long* row, const LStat& st, int sp) {
  __shared__ uint32_t red[kBlock / 64][7];
  const int lane = lane_id(), wv = threadIdx.x / 64;
  const uint32_t vals[7] = {st.alive, st.absorbed, st.elastic, st.ionization, st.cx, st.viol, st.lost};
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const uint32_t s = wave_sum(vals[q]);
    if (lane == 0) red[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNStat) {
    uint32_t tot[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int w = 0; w < kBlock / 64; ++w)
      for (int q = 0; q < 7; ++q) tot[q] += red[w][q];
    unsigned long long v = 0ull;
    switch (threadIdx.x) {
      case kStAlive0: v = sp == 0 ? tot[0] : 0u; break;
      case kStAlive1: v = sp == 1 ? tot[0] : 0u; break;
      case kStAbs0: v = sp == 0 ? tot[1] : 0u; break;
      case kStAbs1: v = sp == 1 ? tot[1] : 0u; break;
      case kStElastic: v = tot[2]; break;
      case kStIonization: v = tot[3]; break;
      case kStCx: v = tot[4]; break;
      case kStViol0: v = sp == 0 ? tot[5] : 0u; break;
      case kStViol1: v = sp == 1 ? tot[5] : 0u; break;
      case kStLostReflect: v = tot[6]; break;
      default: v = 0ull; break;
    }
    row[threadIdx.x] = v;
  }
  __syncthreads();
}

// Zero the deposit buffer of the other step parity (it held the previous
// step's charge, already consumed by the field solve).
__device__ __forceinline__ void zero_other_parity(unsigned long long* Q, uint32_t nq, uint32_t step, int nspecies,
                                                  uint32_t tid, uint32_t nthreads) {
  unsigned long long* Z = Q + (size_t)((step + 1u) & 1u) * 2u * nq;
  const uint32_t n = (uint32_t)nspecies * nq;
  for (uint32_t j = tid; j < n; j += nthreads) Z[j] = 0ull;
}

// Plain 1D launch: blocks [0, gs) advance species 0, [gs, grid) species 1.
template <class T>
__global__ __launch_bounds__(kBlock) void k_step1d(InstDev<T> I, int gs) {
  const int sp = (I.nspecies == 2 && (int)blockIdx.x >= gs) ? 1 : 0;
  const int b0 = sp == 0 ? 0 : gs;
  const int nb = sp == 0 ? (I.nspecies == 2 ? gs : (int)gridDim.x) : (int)gridDim.x - gs;
  const uint32_t step = I.ctr->step;
  const uint32_t count = I.ctr->count[sp];
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t base = (uint32_t)((int)blockIdx.x - b0) * kBlock; base < count; base += (uint32_t)nb * kBlock)
    tile1d<T>(I, sp, base + threadIdx.x, count, step, Qpar, st);
  write_stats_row(I.part + (size_t)blockIdx.x * kNStat, st, sp);
}

// Batched 1D launch: a persistent grid walks a list of (instance, species,
// range) work items; per-instance constants come from the descriptor table.
template <class T>
__global__ __launch_bounds__(kBlock) void k_step1d_batched(const InstDev<T>* __restrict__ insts,
                                                           const WorkItem* __restrict__ items, uint32_t nitems,
                                                           unsigned long long* bpart) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const InstDev<T>& I = insts[wi.inst];
    const int sp = (int)wi.species;
    const uint32_t step = I.ctr->step;
    const uint32_t count = I.ctr->count[sp];
    const uint32_t limit = wi.end < count ? wi.end : count;
    unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
    if (wi.begin == 0 && sp == 0) zero_other_parity(I.Q, I.nq, step, I.nspecies, threadIdx.x, kBlock);
    LStat st = {0, 0, 0, 0, 0, 0, 0};
    for (uint32_t base = wi.begin; base < limit; base += kBlock) tile1d<T>(I, sp, base + threadIdx.x, limit, step, Qpar, st);
    write_stats_row(bpart + (size_t)it * kNStat, st, sp);
  }
}

// ---------------------------------------------------------------------------
// 2D quadtree
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ uint32_t locate2d(const InstDev<T>& I, uint32_t X, uint32_t Y) {
  return locate_leaf(I.leaf_key, I.leaf_lv, I.lut, I.lut_level, X, Y);
}

template <class T>
__device__ __forceinline__ void gather2d(const InstDev<T>& I, uint32_t leaf, T sx, T sy, T& ex, T& ey) {
  const uint32_t xy = I.leaf_xy[leaf];
  const int lv = I.leaf_lv[leaf];
  const int sh = kKeyBits - lv;
  const T sc = (T)(1u << lv);
  const T xi = sx * sc - (T)((xy >> 16) >> sh);
  const T eta = sy * sc - (T)((xy & 0xFFFFu) >> sh);
  const T w00 = ((T)1 - xi) * ((T)1 - eta);
  const T w10 = xi * ((T)1 - eta);
  const T w01 = ((T)1 - xi) * eta;
  const T w11 = xi * eta;
  const T* c = I.E + (size_t)leaf * 8u;
  ex = ((w00 * c[0] + w10 * c[2]) + w01 * c[4]) + w11 * c[6];
  ey = ((w00 * c[1] + w10 * c[3]) + w01 * c[5]) + w11 * c[7];
}

template <class T>
__device__ __forceinline__ void tile2d(const InstDev<T>& I, int sp, uint32_t i, uint32_t limit, uint32_t step,
                                       unsigned long long* Qpar, LStat& st) {
  const SpeciesK<T>& k = I.sk[sp];
  const bool valid = i < limit;
  uint32_t w = valid ? I.w[sp][i] : 0u;
  uint32_t key = kNoKey;
  unsigned long long q = 0ull;
  bool birth = false;
  BirthRec<T> rec;
  T sx = (T)0, sy = (T)0;
  uint32_t pid = 0, leaf = 0;
  if (w != 0u) {
    st.alive++;
    leaf = I.cell[sp][i];
    sx = I.s[sp][0][i];
    sy = I.s[sp][1][i];
    T vx = I.v[sp][0][i];
    T vy = I.v[sp][1][i];
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
      I.w[sp][i] = 0u;
      w = 0u;
    } else {
      const uint32_t X = (uint32_t)(sx * (T)65536);
      const uint32_t Y = (uint32_t)(sy * (T)65536);
      const uint32_t xy = I.leaf_xy[leaf];
      const int sh = kKeyBits - (int)I.leaf_lv[leaf];
      if ((X >> sh) != ((xy >> 16) >> sh) || (Y >> sh) != ((xy & 0xFFFFu) >> sh)) leaf = locate2d<T>(I, X, Y);
      if (k.mcc != PIC_MCC_NONE) {
        pid = I.id[sp][i];
        WordStream ws(I.key0, I.key1, pid, step);
        const uint32_t r0 = ws.next();
        const uint32_t r1 = ws.next();
        if ((r0 >> 8) < k.tcand) {
          T vz = I.v[sp][2][i];
          birth = collide<T>(I, k, pid, step, r1, ws, vx, vy, vz, st, rec);
          I.v[sp][2][i] = vz;
        }
      }
      I.s[sp][0][i] = sx;
      I.s[sp][1][i] = sy;
      I.v[sp][0][i] = vx;
      I.v[sp][1][i] = vy;
      I.cell[sp][i] = leaf;
      key = leaf;
      q = (birth ? 2ull : 1ull) * (unsigned long long)w;
      if (birth) atomicAdd(Qpar + I.nq + leaf, (unsigned long long)w);
    }
  }
  stage_birth<T>(I, birth, pid, leaf, w, sx, sy, rec);
  seg_atomic_add(Qpar + (size_t)sp * I.nq, key, q);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_step2d(InstDev<T> I, int gs) {
  const int sp = (I.nspecies == 2 && (int)blockIdx.x >= gs) ? 1 : 0;
  const int b0 = sp == 0 ? 0 : gs;
  const int nb = sp == 0 ? (I.nspecies == 2 ? gs : (int)gridDim.x) : (int)gridDim.x - gs;
  const uint32_t step = I.ctr->step;
  const uint32_t count = I.ctr->count[sp];
  unsigned long long* Qpar = I.Q + (size_t)(step & 1u) * 2u * I.nq;
  zero_other_parity(I.Q, I.nq, step, I.nspecies, blockIdx.x * kBlock + threadIdx.x, gridDim.x * kBlock);
  LStat st = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t base = (uint32_t)((int)blockIdx.x - b0) * kBlock; base < count; base += (uint32_t)nb * kBlock)
    tile2d<T>(I, sp, base + threadIdx.x, count, step, Qpar, st);
  write_stats_row(I.part + (size_t)blockIdx.x * kNStat, st, sp);
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

template <class T>
__global__ __launch_bounds__(kBlock) void k_births_batched(const InstDev<T>* insts) {
  births_body<T>(insts[blockIdx.x], 0u, 1u);
}

// Commit a step: sum the partial-stats rows, append births to the counts,
// advance the step index.  One block.
template <class T>
__device__ void commit_body(const InstDev<T>& I, const unsigned long long* rows, uint32_t nrows) {
  __shared__ unsigned long long acc[kNStat];
  if (threadIdx.x < kNStat) acc[threadIdx.x] = 0ull;
  __syncthreads();
  for (uint32_t r = threadIdx.x / kNStat; r < nrows; r += kBlock / kNStat) {
    if (threadIdx.x < (kBlock / kNStat) * kNStat) atomicAdd(&acc[threadIdx.x % kNStat], rows[(size_t)r * kNStat + threadIdx.x % kNStat]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Counters* c = I.ctr;
    for (int q = 0; q < kNStat; ++q) c->stats[q] += acc[q];
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
__global__ __launch_bounds__(kBlock) void k_commit(InstDev<T> I, uint32_t nrows) { commit_body<T>(I, I.part, nrows); }

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
      const uint32_t w = i < count ? I.w[sp][i] : 0u;
      uint32_t k0 = kNoKey, k1 = kNoKey;
      unsigned long long q0 = 0ull, q1 = 0ull;
      if (w) {
        if (I.dim == 1) {
          const T g = I.s[sp][0][i] * (T)I.N;
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
          k0 = I.cell[sp][i];
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
      if (!I.w[sp][i]) continue;
      if (I.dim == 1) {
        const T g = I.s[sp][0][i] * (T)I.N;
        int ic = (int)floor(g);
        if (ic > I.N - 1) ic = I.N - 1;
        const T f = g - (T)ic;
        const T E = I.E[ic] + f * (I.E[ic + 1] - I.E[ic]);
        I.v[sp][0][i] = I.v[sp][0][i] - h * E;
      } else {
        T ex, ey;
        gather2d<T>(I, I.cell[sp][i], I.s[sp][0][i], I.s[sp][1][i], ex, ey);
        I.v[sp][0][i] = I.v[sp][0][i] - h * ex;
        I.v[sp][1][i] = I.v[sp][1][i] - h * ey;
      }
    }
  }
}

// cell <- leaf containing s (2D), for all live particles of one species.
template <class T>
__global__ __launch_bounds__(kBlock) void k_relocate(InstDev<T> I, int sp) {
  const uint32_t count = I.ctr->count[sp];
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    if (!I.w[sp][i]) continue;
    const uint32_t X = (uint32_t)(I.s[sp][0][i] * (T)65536);
    const uint32_t Y = (uint32_t)(I.s[sp][1][i] * (T)65536);
    I.cell[sp][i] = locate2d<T>(I, X, Y);
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
hipError_t launch_step1d(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_step1d<T>, dim3(grid), dim3(kBlock), 0, s, I, species_split(I, grid));
  return hipGetLastError();
}
template <class T>
hipError_t launch_step2d(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_step2d<T>, dim3(grid), dim3(kBlock), 0, s, I, species_split(I, grid));
  return hipGetLastError();
}
template <class T>
hipError_t launch_step1d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                 unsigned long long* bpart, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_step1d_batched<T>, dim3(grid), dim3(kBlock), 0, s, I, items, nitems, bpart);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births(const InstDev<T>& I, hipStream_t s, int grid) {
  hipLaunchKernelGGL(k_births<T>, dim3(grid), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_births_batched(const InstDev<T>* I, int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_births_batched<T>, dim3(ninst), dim3(kBlock), 0, s, I);
  return hipGetLastError();
}
template <class T>
hipError_t launch_commit(const InstDev<T>& I, uint32_t nrows, hipStream_t s) {
  hipLaunchKernelGGL(k_commit<T>, dim3(1), dim3(kBlock), 0, s, I, nrows);
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
  template hipError_t launch_step1d<T>(const InstDev<T>&, hipStream_t, int);                               \
  template hipError_t launch_step2d<T>(const InstDev<T>&, hipStream_t, int);                               \
  template hipError_t launch_step1d_batched<T>(const InstDev<T>*, const WorkItem*, uint32_t,               \
                                               unsigned long long*, hipStream_t, int);                     \
  template hipError_t launch_births<T>(const InstDev<T>&, hipStream_t, int);                               \
  template hipError_t launch_births_batched<T>(const InstDev<T>*, int, hipStream_t);                       \
  template hipError_t launch_commit<T>(const InstDev<T>&, uint32_t, hipStream_t);                          \
  template hipError_t launch_deposit<T>(const InstDev<T>&, hipStream_t, int);                              \
  template hipError_t launch_leapfrog_start<T>(const InstDev<T>&, hipStream_t, int);                       \
  template hipError_t launch_relocate<T>(const InstDev<T>&, int, hipStream_t, int);
PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

// commit entry for the batched 1D path without a field solve (one block per slot)
template <class T>
__global__ __launch_bounds__(kBlock) void k_commit_batched(const InstDev<T>* insts, const unsigned long long* bpart,
                                                           const uint32_t* item_begin) {
  const uint32_t b = item_begin[blockIdx.x], e = item_begin[blockIdx.x + 1];
  commit_body<T>(insts[blockIdx.x], bpart + (size_t)b * kNStat, e - b);
}
template <class T>
hipError_t launch_commit_batched(const InstDev<T>* I, const unsigned long long* bpart, const uint32_t* item_begin,
                                 int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_batched<T>, dim3(ninst), dim3(kBlock), 0, s, I, bpart, item_begin);
  return hipGetLastError();
}
template hipError_t launch_commit_batched<float>(const InstDev<float>*, const unsigned long long*, const uint32_t*,
                                                 int, hipStream_t);
template hipError_t launch_commit_batched<double>(const InstDev<double>*, const unsigned long long*, const uint32_t*,
                                                  int, hipStream_t);

}  // namespace pic
