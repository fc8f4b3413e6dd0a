// Host orchestration of pic_adapt: the launch sequence of the quadtree
// adaptation and particle split/merge kernels (k_adapt.hip).  The host only
// reads back small counters that decide whether another pass is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "k_adapt.hpp"
#include "k_mesh.hpp"
#include "pic_internal.hpp"

namespace pic {

namespace {

// scoped device scratch, freed after the stream has drained
// Scratch of one adaptation pass, from the context's device cache (blocks
// are reusable after the context's next stream synchronization).
struct Scratch {
  DevPool& pool;
  std::vector<std::pair<size_t, void*>> blocks;
  explicit Scratch(Ctx& C) : pool(C.pool) {}
  template <class T>
  T* get(size_t n) {
    const size_t cls = DevPool::class_of(std::max<size_t>(n, 1) * sizeof(T));
    void* p = nullptr;
    if (pool.pooled(cls)) {
      p = pool.get(cls);
    } else {
      hip_check(hipMalloc(&p, cls), "hipMalloc scratch");
    }
    blocks.emplace_back(cls, p);
    return (T*)p;
  }
  ~Scratch() {
    for (auto& b : blocks) {
      if (pool.pooled(b.first)) {
        pool.put(b.second, b.first);
      } else {
        (void)hipDeviceSynchronize();
        (void)hipFree(b.second);
      }
    }
  }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
};

TreeView view(const Slot& sl) {
  if (launch_checks()) check_tables(sl);
  TreeView t;
  t.key = sl.key;
  t.lv = sl.lv;
  t.lut = sl.lut;
  t.lut_level = sl.lut_level;
  t.n = sl.nleaves;
  t.min_level = sl.d.min_level;
  t.max_level = sl.d.max_level;
  return t;
}

template <class V>
V read1(Ctx& C, const V* d) {
  V h;
  hip_check(hipMemcpyAsync(&h, d, sizeof(V), hipMemcpyDeviceToHost, C.stream), "read");
  C.sync();
  return h;
}

template <class T>
void relocate_all(Ctx& C, Slot& sl) {
  const InstDev<T> I = make_dev<T>(sl);
  for (int sp = 0; sp < sl.d.nspecies; ++sp)
    if (sl.pb[sp][sl.cur[sp]].base)
      hip_check(launch_relocate<T>(I, sp, C.stream, grid_for(sl.cap[sp])), "relocate");
}

template <class T>
uint32_t* count_all(Ctx& C, Slot& sl, Scratch& S) {
  uint32_t* cnt = S.get<uint32_t>(2 * (size_t)sl.nleaves);
  hip_check(hipMemsetAsync(cnt, 0, 8 * (size_t)sl.nleaves, C.stream), "memset");
  const InstDev<T> I = make_dev<T>(sl);
  for (int sp = 0; sp < sl.d.nspecies; ++sp)
    if (sl.pb[sp][sl.cur[sp]].base) hip_check(launch_count<T>(I, sp, cnt, grid_for(sl.cap[sp]), C.stream), "count");
  return cnt;
}

// Rebuild the leaf array from per-leaf emit counts; returns false if nothing changed.
bool rebuild(Ctx& C, Slot& sl, Scratch& S, uint32_t* emit, const uint32_t* cflag) {
  const uint32_t n = sl.nleaves;
  uint32_t* tmp = S.get<uint32_t>(scan_tmp_words(n));
  hip_check(launch_scan_u32(emit, n, tmp, C.stream), "scan");
  const uint32_t total = read1(C, emit + n);
  uint32_t* maxlv = S.get<uint32_t>(1);
  hip_check(hipMemsetAsync(maxlv, 0, 4, C.stream), "memset");
  uint32_t* nkey = (uint32_t*)sl.alloc(4 * (size_t)total);
  uint8_t* nlv = (uint8_t*)sl.alloc((size_t)total);
  hip_check(launch_tree_emit(view(sl), emit, cflag, nkey, nlv, maxlv, C.stream), "emit");
  // the finest level present matters only when the tree may go below the
  // point-location table; else the table is direct whatever it is
  const uint32_t mx = sl.d.max_level <= kLutMaxLevel ? (uint32_t)sl.d.max_level : read1(C, maxlv);
  set_mesh2d_device(C, sl, nkey, nlv, total, (int)mx);
  return true;
}

// Per-leaf counts of the present tree and particles, kept until either
// changes (a rebuild, a relocation or new particles), so a pass that finds
// nothing to do leaves its counts to the next pass.
template <class T>
struct Counts {
  Ctx& C;
  Slot& sl;
  Scratch keep;
  uint32_t* cnt = nullptr;
  Counts(Ctx& c, Slot& s) : C(c), sl(s), keep(c) {}
  uint32_t* get() {
    if (!cnt) cnt = count_all<T>(C, sl, keep);
    return cnt;
  }
  void stale() { cnt = nullptr; }
};

template <class T>
void adapt_impl(Ctx& C, Slot& sl, int n_lo, int n_hi, pic_adapt_stats* out) {
  pic_adapt_stats st;
  std::memset(&st, 0, sizeof(st));
  const int ns = sl.d.nspecies;
  // a capacity limit met while splitting or merging stops that part only;
  // it is raised once the adaptation is complete
  std::string deferred;
  relocate_all<T>(C, sl);
  Counts<T> counts(C, sl);
  // ---- coarsen and refine decided on the current tree ----
  {
    Scratch S(C);
    uint32_t* cnt = counts.get();
    const uint32_t n = sl.nleaves;
    uint32_t* cflag = S.get<uint32_t>(n);
    uint32_t* emit = S.get<uint32_t>(n + 1);
    uint32_t* nch = S.get<uint32_t>(3);
    hip_check(hipMemsetAsync(nch, 0, 12, C.stream), "memset");
    hip_check(launch_coarsen_flags(view(sl), cnt, ns, n_lo, n_hi, cflag, C.stream), "coarsen flags");
    hip_check(launch_tree_flags(view(sl), cnt, ns, n_hi, 0, nullptr, cflag, emit, nch, C.stream), "flags");
    uint32_t h[3];
    hip_check(hipMemcpyAsync(h, nch, 12, hipMemcpyDeviceToHost, C.stream), "read");
    C.sync();
    st.coarsened += h[1];
    st.refined += h[2];
    if (h[0]) {
      rebuild(C, sl, S, emit, cflag);
      relocate_all<T>(C, sl);
      counts.stale();
    }
  }
  // ---- refine again while a leaf is over the upper bound ----
  for (;;) {
    Scratch S(C);
    uint32_t* cnt = counts.get();
    const uint32_t n = sl.nleaves;
    uint32_t* emit = S.get<uint32_t>(n + 1);
    uint32_t* nch = S.get<uint32_t>(3);
    hip_check(hipMemsetAsync(nch, 0, 12, C.stream), "memset");
    hip_check(launch_tree_flags(view(sl), cnt, ns, n_hi, 1, nullptr, nullptr, emit, nch, C.stream), "flags");
    uint32_t h[3];
    hip_check(hipMemcpyAsync(h, nch, 12, hipMemcpyDeviceToHost, C.stream), "read");
    C.sync();
    if (!h[0]) break;
    st.refined += h[2];
    rebuild(C, sl, S, emit, nullptr);
    relocate_all<T>(C, sl);
    counts.stale();
  }
  // ---- 2:1 balance by refinement ----
  bool balanced = false;
  for (;;) {
    Scratch S(C);
    const uint32_t n = sl.nleaves;
    uint32_t* mark = S.get<uint32_t>(n);
    uint32_t* nmark = S.get<uint32_t>(1);
    hip_check(hipMemsetAsync(mark, 0, 4 * (size_t)n, C.stream), "memset");
    hip_check(hipMemsetAsync(nmark, 0, 4, C.stream), "memset");
    hip_check(launch_balance_mark(view(sl), mark, nmark, C.stream), "balance");
    const uint32_t nm = read1(C, nmark);
    if (!nm) break;
    st.balance_refined += nm;
    uint32_t* emit = S.get<uint32_t>(n + 1);
    uint32_t* nch = S.get<uint32_t>(3);
    hip_check(hipMemsetAsync(nch, 0, 12, C.stream), "memset");
    hip_check(launch_tree_flags(view(sl), nullptr, ns, n_hi, 2, mark, nullptr, emit, nch, C.stream), "flags");
    rebuild(C, sl, S, emit, nullptr);
    balanced = true;
  }
  if (balanced) {
    relocate_all<T>(C, sl);
    counts.stale();
  }
  // ---- split rounds ----
  for (;;) {
    Scratch S(C);
    uint32_t* cnt = counts.get();
    Counters cn = read_counters(C, sl);
    const uint32_t nw = cn.next_id / 32u + 1u;
    uint32_t* bitmap = S.get<uint32_t>(nw);
    uint32_t* np = S.get<uint32_t>(2);
    hip_check(hipMemsetAsync(bitmap, 0, 4 * (size_t)nw, C.stream), "memset");
    hip_check(hipMemsetAsync(np, 0, 8, C.stream), "memset");
    {
      const InstDev<T> I = make_dev<T>(sl);
      for (int sp = 0; sp < ns; ++sp)
        hip_check(launch_split_mark<T>(I, sp, cnt, n_lo, bitmap, np, grid_for(sl.cap[sp]), C.stream), "split mark");
    }
    uint32_t h[2] = {0, 0};
    hip_check(hipMemcpyAsync(h, np, 8, hipMemcpyDeviceToHost, C.stream), "read");
    C.sync();
    const uint64_t tot = (uint64_t)h[0] + h[1];
    if (!tot) break;
    if ((uint64_t)cn.next_id + 3ull * tot > 0xFFFFFFFFull) {
      deferred = "particle ids exhausted by splitting";
      break;
    }
    bool room = true;
    for (int sp = 0; sp < ns && room; ++sp) {
      const int64_t need = (int64_t)cn.count[sp] + 3 * (int64_t)h[sp];
      if (need <= sl.cap[sp]) continue;
      try {
        grow(C, sl, sp, need + need / 2 + 1024, cn.count[sp]);
      } catch (const Err& e) {   // the per-array limit: no split this round (growth leaves the slot whole)
        if (e.code != PIC_E_CAPACITY) throw;
        deferred = e.msg;
        room = false;
      }
    }
    if (!room) break;
    upload_dev(C, sl);
    uint32_t* prefix = S.get<uint32_t>(nw + 1);
    uint32_t* tmp = S.get<uint32_t>(scan_tmp_words(nw));
    uint32_t* cursor = S.get<uint32_t>(2);
    hip_check(launch_popc(bitmap, nw, prefix, C.stream), "popc");
    hip_check(launch_scan_u32(prefix, nw, tmp, C.stream), "scan");
    hip_check(hipMemsetAsync(cursor, 0, 8, C.stream), "memset");
    {
      const InstDev<T> I = make_dev<T>(sl);
      for (int sp = 0; sp < ns; ++sp)
        hip_check(launch_split_emit<T>(I, sp, cnt, n_lo, bitmap, prefix, cursor, grid_for(sl.cap[sp]), C.stream),
                  "split emit");
    }
    hip_check(launch_split_commit(sl.ctr, np, ns, C.stream), "split commit");
    counts.stale();
    st.split_parents += (int64_t)tot;
  }
  // ---- merge (leaves at the finest level over the upper bound) ----
  // One count serves both species (merging one leaves the other's counts as
  // they are); the merge kernel runs every round of a leaf, so one launch
  // per species finishes it.
  {
    Scratch S(C);
    uint32_t* cnt = counts.get();
    const uint32_t n = sl.nleaves;
    uint32_t* groups = S.get<uint32_t>(n);
    uint32_t* ng = S.get<uint32_t>(1);
    uint32_t* flags = S.get<uint32_t>(1);
    uint32_t* npairs = S.get<uint32_t>(1);
    double* energy = S.get<double>(1);
    for (int sp = 0; sp < ns; ++sp) {
      hip_check(hipMemsetAsync(ng, 0, 4, C.stream), "memset");
      hip_check(launch_merge_groups(cnt, n, sp, n_hi, groups, ng, C.stream), "merge groups");
      const uint32_t ngroups = read1(C, ng);
      if (!ngroups) continue;
      hip_check(hipMemsetAsync(flags, 0, 4, C.stream), "memset");
      hip_check(hipMemsetAsync(npairs, 0, 4, C.stream), "memset");
      hip_check(hipMemsetAsync(energy, 0, 8, C.stream), "memset");
      // order this species by leaf: its particles of a leaf become contiguous and
      // sl.off holds the end offset of each leaf
      {
        const InstDev<T> I = make_dev<T>(sl);
        const int other = 1 - sl.cur[sp];
        check_sort_target(sl, sp);
        PBuf& d = sl.pb[sp][other];
        SortDst<T> dst{(T*)d.s[0], (T*)d.s[1], (T*)d.v[0], (T*)d.v[1], (T*)d.v[2], d.w, d.id, d.cell};
        hip_check(launch_sort<T>(I, sp, n, sl.off, sl.scan_tmp, dst, grid_for(sl.cap[sp]), C.stream), "sort");
        sl.cur[sp] = other;
      }
      upload_dev(C, sl);
      {
        const InstDev<T> I = make_dev<T>(sl);
        hip_check(launch_merge<T>(I, sp, groups, ngroups, cnt, sl.off, n_hi, flags, energy, npairs, C.stream), "merge");
      }
      const uint32_t fl = read1(C, flags);
      const uint32_t pairs = read1(C, npairs);
      st.merge_energy_change += read1(C, energy);
      if (fl) deferred = "a leaf holds more particles than a merge round can sort";   // such leaves are left as they are
      st.merged_pairs += pairs;
    }
  }
  // ---- drop merged-away particles, order by leaf, fresh deposit ----
  sort_slot(C, sl);
  hip_check(hipMemsetAsync(sl.Q, 0, 32 * (size_t)sl.nq, C.stream), "memset");
  hip_check(launch_deposit<T>(make_dev<T>(sl), C.stream, grid_for(std::max(sl.cap[0], sl.cap[1]))), "deposit");
  C.sync();
  st.nleaves = sl.nleaves;
  if (out) *out = st;
  if (!deferred.empty()) throw Err(PIC_E_CAPACITY, deferred);
}

}  // namespace

void adapt_slot(Ctx& C, Slot& sl, int n_lo, int n_hi, pic_adapt_stats* out) {
  if (sl.d.dim != 2) throw Err(PIC_E_ARG, "adapt needs a quadtree slot");
  if (sl.error_state) throw Err(PIC_E_STATE, "slot is in an error state");
  if (n_lo < 0 || n_hi < 1 || n_lo > n_hi) throw Err(PIC_E_ARG, "need 0 <= n_lo <= n_hi");
  // An adaptation that fails part-way (device memory, a runtime error) leaves
  // the tree and the particles in between two states: the slot is then
  // marked failed, and every later call on it but pic_retire and the counter
  // reads returns PIC_E_STATE.  A capacity limit leaves a complete
  // adaptation (particles not split, or an over-full leaf not merged).
  try {
    if (sl.prec == 32) adapt_impl<float>(C, sl, n_lo, n_hi, out);
    else adapt_impl<double>(C, sl, n_lo, n_hi, out);
  } catch (const Err& e) {
    if (e.code != PIC_E_CAPACITY) {
      sl.error_state = true;
      throw;
    }
    try {
      upload_dev(C, sl);
      C.sync();
    } catch (...) {
      sl.error_state = true;
    }
    throw;
  } catch (...) {
    sl.error_state = true;
    throw;
  }
  upload_dev(C, sl);
  C.sync();
}

}  // namespace pic
