// Host-side state of the library (slots, context) shared by api.hip and abi.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <map>
#include <vector>

#include "pic_internal.hpp"

namespace pic {

constexpr int kMaxGrid = 2048;       // default upper bound on helper-kernel grids
constexpr int kLutMaxLevel = 11;   // finest level of the point-location table (4^11 + 1 entries)
constexpr int kMaxStepGrid = 8192;   // upper bound on the per-slot step-kernel grid (stats rows)

struct Err {
  int code;
  std::string msg;
  Err(int c, std::string m) : code(c), msg(std::move(m)) {}
};
void hip_check(hipError_t e, const char* what);

struct HostK {
  double qm_dt = 0, dt_L = 0, a_el = 0, a_iz = 0, v_iz2 = 0, mu2 = 0, vmax2 = 0, v_thg = 0, a_cx = 0, gmax = 0;
  uint32_t tcand = 0;
  int mcc = 0;
};

struct HostLeaf {
  uint32_t key;
  uint8_t lv;
};

struct PBuf {
  void* base = nullptr;
  void* s[3] = {nullptr, nullptr, nullptr};
  void* v[3] = {nullptr, nullptr, nullptr};
  uint32_t* w = nullptr;
  uint32_t* id = nullptr;
  uint32_t* cell = nullptr;
  void* acc = nullptr;   // direct implicit: (dt/2) x the filtered acceleration per particle
};

// Device memory cache of a context.  Blocks of up to kMaxBlock bytes are
// kept after release and handed out again (sizes rounded up to a class of at
// most 25 % slack), so the tree rebuilds and the scratch of adaptation do not
// call hipMalloc / hipFree (whose free synchronizes the device).  A released
// block becomes reusable only after the context's next stream
// synchronization, when no queued work can still read or write it.
struct DevPool {
  static constexpr size_t kMaxBlock = size_t(256) << 20;
  // cached bytes beyond a quarter of what the context's slots hold (at least
  // 64 MiB, at most 4 GiB) are freed: many small contexts do not hoard memory
  static constexpr size_t kMinFree = size_t(64) << 20;
  static constexpr size_t kMaxFree = size_t(4) << 30;
  std::multimap<size_t, void*> free_;
  std::vector<std::pair<size_t, void*>> pending_;
  size_t free_bytes = 0;
  // caller's allocator (pic_set_allocator): every block comes from it and
  // goes back to it at the next synchronization; nothing is cached here
  pic_allocator ext{};
  bool has_ext = false;
  hipStream_t stream = nullptr;
  static size_t class_of(size_t bytes);
  bool pooled(size_t cls) const { return has_ext || cls <= kMaxBlock; }
  void* get(size_t cls);   // cls from class_of; throws PIC_E_NOMEM
  void put(void* p, size_t cls);
  void synced(size_t held);   // held: bytes the context's slots hold
  void clear();
};

struct Slot {
  bool live = false;
  DevPool* pool = nullptr;   // the context's cache (set when the slot is built)
  pic_instance_desc d{};
  int prec = 64;
  size_t esz = 8;
  bool ionizing = false;
  HostK hk[2];
  double kappa[2] = {0, 0};
  double inv2dx = 0;
  double chi[2] = {0, 0};                  // direct implicit: charge sum -> susceptibility per species
  uint32_t sort_shift = 0;                 // 1D: order kept by bins of 2^sort_shift cells (sort_bins_1d bins)
  unsigned long long* Qp = nullptr;        // direct implicit: charge at the predicted positions [2][N+1]
  double* dws = nullptr;                   // direct implicit solve scratch [3][N+1]
  // particles: [species][buffer]; cur = live buffer, the other is the sort target
  PBuf pb[2][2];
  int cur[2] = {0, 0};
  int64_t cap[2] = {0, 0};
  // births staging
  void* birth_base = nullptr;
  uint32_t* scan_tmp = nullptr;   // 2D: scratch of the sort's multi-block scan (after off)
  uint32_t *br_parent = nullptr, *br_rank = nullptr, *br_cell = nullptr, *br_w = nullptr;
  uint32_t *br_bin = nullptr, *br_bin_off = nullptr, *br_cursor = nullptr, *br_sorted = nullptr;
  // births ranking: 0 by the births of recent steps, 1 pairwise, 2 binned
  int births_method = 0;
  double births_rate = 0.0;           // births per step over the previous chunk of steps
  uint64_t rate_births_mark = 0;
  uint32_t rate_step_mark = 0;
  void* br_s[3] = {nullptr, nullptr, nullptr};
  void* br_ve[3] = {nullptr, nullptr, nullptr};
  void* br_vi[3] = {nullptr, nullptr, nullptr};
  uint32_t birth_cap = 0;
  // field tables
  void* E = nullptr;
  void* cellE = nullptr;   // 2D cloud-in-cell: cell-centred E [nleaves][2] in the particle precision
  double *e64 = nullptr, *phi64 = nullptr, *cphi = nullptr, *grad = nullptr;
  // 2D mesh
  uint32_t *key = nullptr, *xy = nullptr, *lut = nullptr;
  uint8_t* lv = nullptr;
  int lut_level = 0;
  bool lut_direct = false;
  uint32_t nleaves = 0;
  Stencil2D st{nullptr, nullptr, nullptr, nullptr};
  double* cg_ws = nullptr;
  bool stencil_ok = false;
  uint32_t cg_iters_prev = 0;   // iterations of the slot's last CG solve
  // deposit, counters, stats rows, order scratch
  unsigned long long* Q = nullptr;
  uint32_t nq = 0;
  Counters* ctr = nullptr;
  unsigned long long* part = nullptr;
  uint32_t* off = nullptr;
  double* v_table = nullptr;
  uint32_t v_len = 0, v_cap = 0;
  void* devI = nullptr;    // device copy of InstDev<T>
  uint32_t max_id_loaded[2] = {0, 0};
  bool error_state = false;
  size_t byte_limit = 0;   // device bytes the slot may hold after growth (0: no limit)
  // allocations
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  std::vector<char> alloc_pooled;   // the block came from (and goes back to) the pool
  size_t bytes_held = 0;
  void* alloc(size_t bytes);
  void release(void* p);
  void release_all();
};

// 1D order upkeep sorts by bins of consecutive cells, at most kSortBins1D of
// them: a bin keeps a workgroup's particles within the step kernel's deposit
// window, and a sort pass over 1024 particles then writes runs of about 16
// particles per bin instead of one particle per cell (the electrons of a
// discharge mix over the whole mesh between sorts).
#ifndef PIC_SORT_BINS_1D
#define PIC_SORT_BINS_1D 64
#endif
constexpr uint32_t kSortBins1D = PIC_SORT_BINS_1D;
inline uint32_t sort_shift_1d(int ncells) {
  uint32_t s = 0;
  while ((((uint32_t)ncells - 1u) >> s) + 1u > kSortBins1D) ++s;
  return s;
}
inline uint32_t sort_bins_1d(const Slot& sl) { return (((uint32_t)sl.d.ncells - 1u) >> sl.sort_shift) + 1u; }

// Births of the slot ranked through id bins (else pairwise): by request, or
// once its births per step are many.
inline bool slot_births_binned(const Slot& sl) {
  return sl.births_method == 2 || (sl.births_method == 0 && sl.births_rate > kBinnedBirthsPerStep);
}

// One small host -> device (or device -> device) copy of a gathered batch:
// a copy kernel moves 'bytes' (a multiple of 4) from src to dst.
struct Blob {
  void* dst;
  const void* src;
  uint32_t bytes, pad;
};

struct Ctx {
  std::vector<Slot> slots;
  hipStream_t stream = nullptr;
  DevPool pool;
  std::string err;
  void* arena = nullptr;
  size_t arena_size = 0, arena_off = 0;
  std::vector<hipEvent_t> ev;
  // batched launch resources
  void* b_insts = nullptr;
  size_t b_insts_bytes = 0;
  void* b_items = nullptr;
  size_t b_items_bytes = 0;
  unsigned long long* b_part = nullptr;
  size_t b_part_bytes = 0;
  uint32_t* b_rowbeg = nullptr;
  size_t b_rowbeg_bytes = 0;
  void* b_jobs = nullptr;   // batched sort jobs, two per slot
  size_t b_jobs_bytes = 0;
  // graph capture stream (default priority) and the events joining it to the caller's stream
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  // set during a no-allocation step: synchronizations keep released blocks
  // pending instead of freeing them (they are freed at a later sync)
  bool hold_pool = false;
  // Small uploads (counters, instance views) of many slots gathered into one
  // transfer and one copy kernel while defer_uploads is set; flushed by
  // flush_uploads (and before any read of counters).
  bool defer_uploads = false;
  std::vector<Blob> pend;        // src holds the offset into pend_data
  std::vector<char> pend_data;
  void* b_blob = nullptr;        // device side of a gathered batch: table, then payload
  size_t b_blob_bytes = 0;
  void upload(void* dst, const void* src, size_t bytes);
  void flush_uploads();
  void* blob_buffer(size_t bytes);
  void* stage(const void* src, size_t bytes);
  void* pinned(size_t bytes);   // pinned host scratch from the staging arena
  void sync();
  void release_tables();        // batched launch tables back to the pool
};

void derive(Slot& sl);
void build_slot(Ctx& C, Slot& sl, const pic_instance_desc& d);
void set_mesh2d(Ctx& C, Slot& sl, const std::vector<HostLeaf>& L);
void set_mesh2d_device(Ctx& C, Slot& sl, uint32_t* key, uint8_t* lv, uint32_t n, int maxlv);
void adapt_slot(Ctx& C, Slot& sl, int n_lo, int n_hi, pic_adapt_stats* out);
void alloc_particles(Slot& sl, int sp, int64_t cap);
size_t pbuf_bytes(const Slot& sl, int64_t cap);
size_t births_bytes(const Slot& sl, int64_t cap);
void alloc_births(Ctx& C, Slot& sl, int64_t cap);
template <class T> InstDev<T> make_dev(const Slot& sl);   // checked when launch checks are on
bool launch_checks();                        // PIC_CHECK_LAUNCHES set in the environment
void check_tables(const Slot& sl);           // mesh, field and deposit tables against the slot's blocks
void check_sort_target(const Slot& sl, int sp);   // no-op unless launch checks are on
void upload_dev(Ctx& C, Slot& sl);
Counters read_counters(Ctx& C, Slot& sl);
std::vector<Counters> read_counters_many(Ctx& C, const std::vector<Slot*>& sel);
void write_counters(Ctx& C, Slot& sl, const Counters& c);
int grid_for(int64_t n);
void ensure_capacity(Ctx& C, Slot& sl, const Counters& c, int64_t steps_ahead);
void check_capacity(const Slot& sl, const Counters& c);
void sort_slot(Ctx& C, Slot& sl);
void grow(Ctx& C, Slot& sl, int sp, int64_t newcap, uint32_t count);
uint32_t morton_host(uint32_t x, uint32_t y);
void unmorton_host(uint32_t k, uint32_t& x, uint32_t& y);
size_t host_locate(const std::vector<HostLeaf>& L, uint32_t X, uint32_t Y);
std::vector<HostLeaf> host_build_tree(const pic_instance_desc& d);
template <class T> SpeciesK<T> to_dev(const HostK& h);

}  // namespace pic
