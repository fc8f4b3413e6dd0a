// extern "C" entry points of include/pic.h.  Argument checking, marshalling
// between host arrays and device state, and the launch sequences; every
// step of the particle loop and of the field solves runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "k_mesh.hpp"
#include "device_util.hpp"
#include "pic_internal.hpp"

using namespace pic;

struct pic_ctx_s : public Ctx {};

// Device memory of the no-allocation step (pic_step_noalloc): its launch
// tables live in this file-scope array, one copy per device, held until the
// process ends.  Host code must not pass the array's name to a kernel (on
// the host it is only a stand-in); scratch_device_ptr() gives the device
// address, looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of 'scratch' on the current device (looked up on the first
// call per device, with that device current).
void* scratch_device_ptr() {
  int dev = -1;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) throw Err(PIC_E_ARG, "device index out of range for the no-allocation workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Err(PIC_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Launch tables carved from the no-allocation workspace.
struct Workspace {
  char* base;
  size_t size, off;
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (off + bytes > size)
      throw Err(PIC_E_ARG, "the launch tables need more than the " + std::to_string(size >> 20) +
                               " MiB no-allocation workspace (fewer slots, larger work items or fewer steps per call)");
    void* p = base + off;
    off += bytes;
    return p;
  }
};

__global__ void k_zero_u64(unsigned long long* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0ull;
}

#define PIC_GUARD_BEGIN try {
#define PIC_GUARD_END(ctx)                                   \
  }                                                          \
  catch (const Err& e) {                                     \
    if (ctx) (ctx)->err = e.msg;                             \
    g_last_error = e.msg;                                    \
    return e.code;                                           \
  }                                                          \
  catch (const std::exception& e) {                          \
    if (ctx) (ctx)->err = e.what();                          \
    g_last_error = e.what();                                 \
    return PIC_E_ARG;                                        \
  }

Slot& get_slot(pic_ctx c, int slot) {
  if (!c) throw Err(PIC_E_ARG, "null context");
  if (slot < 0 || slot >= (int)c->slots.size() || !c->slots[slot].live) throw Err(PIC_E_ARG, "no such slot");
  return c->slots[slot];
}

// A slot whose device data may be used: not marked failed (a device-side
// overflow, or a call that failed part-way through changing its tables).
// A failed slot answers only the counter reads and pic_retire.
Slot& usable_slot(pic_ctx c, int slot) {
  Slot& sl = get_slot(c, slot);
  if (sl.error_state) throw Err(PIC_E_STATE, "slot is in an error state (retire it)");
  return sl;
}

Mesh2D mesh_of(const Slot& sl) {
  if (launch_checks()) check_tables(sl);
  Mesh2D m;
  m.key = sl.key;
  m.xy = sl.xy;
  m.lv = sl.lv;
  m.lut = sl.lut;
  m.lut_level = sl.lut_level;
  m.nleaves = sl.nleaves;
  m.length = sl.d.length;
  for (int i = 0; i < 4; ++i) {
    m.field_bc[i] = sl.d.field_bc[i];
    m.wall_phi[i] = sl.d.wall_phi[i];
  }
  return m;
}

// The cell-centred E table of a cloud-in-cell slot from its FP64 corner
// table (after every change of the corner table).
void refresh_cell_e(Ctx& C, Slot& sl) {
  if (sl.d.dim != 2 || sl.d.field_scheme != PIC_FIELD_CIC_AMR || !sl.cellE) return;
  if (sl.prec == 32) hip_check(launch_cell_e<float>(sl.e64, sl.nleaves, (float*)sl.cellE, C.stream), "cell_e");
  else hip_check(launch_cell_e<double>(sl.e64, sl.nleaves, (double*)sl.cellE, C.stream), "cell_e");
}

void* dev_upload(Ctx& C, Slot& sl, const void* host, size_t bytes) {
  void* d = sl.alloc(bytes);
  hip_check(hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, C.stream), "upload");
  C.sync();
  return d;
}

bool slot_has_mcc(const Slot& sl);

// Grid of the per-slot step kernel: by default one workgroup per 256
// particles of capacity, at most as many as are resident on the device at
// once (each workgroup walks its chunk in one pass); or the caller's choice.
int step_grid(const Slot& sl, int requested) {
  int g;
  if (requested > 0) {
    g = std::min(requested, kMaxStepGrid);
  } else {
    const int res = sl.prec == 32 ? step_resident_grid<float>(sl.d.dim, slot_has_mcc(sl), sl.lut_direct)
                                  : step_resident_grid<double>(sl.d.dim, slot_has_mcc(sl), sl.lut_direct);
    g = std::min(grid_for(sl.cap[0] + sl.cap[1]), std::min(res, kMaxStepGrid));
  }
  return sl.d.nspecies == 2 ? std::max(g, 2) : g;   // one workgroup per species at least
}

__global__ void k_locate_points(const uint32_t* key, const uint8_t* lv, const uint32_t* lut, int L, const double* s,
                                int64_t n, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t X = (uint32_t)(s[2 * i] * 65536.0), Y = (uint32_t)(s[2 * i + 1] * 65536.0);
  out[i] = locate_leaf(key, lv, lut, L, X, Y);
}

__global__ void k_locate_points3(const uint32_t* key, const uint8_t* lv, const uint32_t* lut, int L, const double* s,
                                 int64_t n, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = locate_leaf3(key, lv, lut, L, (uint32_t)(s[3 * i] * 1024.0), (uint32_t)(s[3 * i + 1] * 1024.0),
                        (uint32_t)(s[3 * i + 2] * 1024.0));
}

// A coordinate inside [0, 1) once rounded to the particle precision (a
// double just below 1 rounds to 1 in FP32).
bool in_unit(double x, int prec) {
  const double r = prec == 32 ? (double)(float)x : x;
  return r >= 0.0 && r < 1.0;
}

__global__ void k_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x0 = ctr[4 * i], x1 = ctr[4 * i + 1], x2 = ctr[4 * i + 2], x3 = ctr[4 * i + 3];
  philox4x32_10(x0, x1, x2, x3, k0, k1);
  out[4 * i] = x0;
  out[4 * i + 1] = x1;
  out[4 * i + 2] = x2;
  out[4 * i + 3] = x3;
}

// ---- one plain step of one slot ----
bool slot_has_mcc(const Slot& sl) {
  for (int sp = 0; sp < sl.d.nspecies; ++sp)
    if (sl.d.species[sp].mcc != PIC_MCC_NONE) return true;
  return false;
}

template <class T>
void plain_step(Ctx& C, Slot& sl, bool solve, int g, hipEvent_t e0, hipEvent_t e1) {
  InstDev<T> I = make_dev<T>(sl);
  if (I.dipic) {   // predictor, implicit field, corrector; then births and the commit
    if (e0) hip_check(hipEventRecord(e0, C.stream), "event");
    hip_check(launch_dipic_predict<T>(I, C.stream, g), "dipic predict");
    hip_check(launch_dipic_field<T>(I, C.stream), "dipic field");
    hip_check(launch_dipic_correct<T>(I, C.stream, g, slot_has_mcc(sl)), "dipic correct");
    if (sl.ionizing) hip_check(launch_births<T>(I, C.stream, I.births_binned != 0), "births");
    if (e1) hip_check(hipEventRecord(e1, C.stream), "event");
    hip_check(launch_commit<T>(I, C.stream), "commit");
    return;
  }
  const bool field = sl.d.dim == 1 && solve;
  const int commit = (!sl.ionizing && !field) ? 1 : 0;
  // a timed step: from the step kernel's own start to its end, or to after
  // the births kernels
  hip_check(launch_step<T>(I, C.stream, g, slot_has_mcc(sl), commit, e0, sl.ionizing ? nullptr : e1), "step");
  if (sl.ionizing) {
    // binned ranking once births per step are many (pairwise work grows as their square)
    hip_check(launch_births<T>(I, C.stream, I.births_binned != 0), "births");
    if (e1) hip_check(hipEventRecord(e1, C.stream), "event");
  }
  if (field)
    hip_check(launch_field1d<T>((const InstDev<T>*)sl.devI, 1, sl.d.ncells, 1, nullptr, C.stream), "field1d");
  else if (!commit)
    hip_check(launch_commit<T>(I, C.stream), "commit");
}

template <class T>
void reduce_plain_stats(Ctx& C, Slot& sl, int g) {
  hip_check(launch_stats_reduce<T>((const InstDev<T>*)sl.devI, 1, nullptr, nullptr, (uint32_t)g,
                                   C.stream),
            "stats_reduce");
}

// Before a run of 'nsteps' steps of one slot: births rate (ranking method),
// drive table v_next[k * nsel + j] for k < nsteps, capacity, device view.
// The slot continues from its own step index.
void prepare_slot(Ctx& C, Slot& sl, const pic_step_args* a, const double* v_next, int j, int nsel, int64_t nsteps,
                  Counters cn, bool noalloc = false) {
  if (sl.error_state) throw Err(PIC_E_STATE, "slot is in an error state (retire it)");
  if (!sl.pb[0][sl.cur[0]].base) throw Err(PIC_E_STATE, "no particles loaded");
  if (sl.ionizing) {   // births per step since the previous chunk picks the ranking method
    const uint64_t b = cn.stats[kStBirths];
    if (cn.step > sl.rate_step_mark && b >= sl.rate_births_mark)
      sl.births_rate = (double)(b - sl.rate_births_mark) / (double)(cn.step - sl.rate_step_mark);
    sl.rate_births_mark = b;
    sl.rate_step_mark = cn.step;
  }
  cn.vstep0 = cn.step + 1u;
  cn.flags &= ~kFlagNeedRoom;
  if (noalloc) {   // the drive table goes to the workspace; no growth
    if (sl.d.dim == 1 && a->solve_field && !v_next) throw Err(PIC_E_ARG, "solve_field needs v_next");
    check_capacity(sl, cn);
    write_counters(C, sl, cn);
    upload_dev(C, sl);
    return;
  }
  if (sl.d.dim == 1 && a->solve_field) {
    if (!v_next) throw Err(PIC_E_ARG, "solve_field needs v_next");
    if (sl.v_cap < (uint32_t)nsteps) {
      double* nt = (double*)sl.alloc(8 * (size_t)std::max<int64_t>(nsteps, 64));
      sl.release(sl.v_table);
      sl.v_table = nt;
      sl.v_cap = (uint32_t)std::max<int64_t>(nsteps, 64);
    }
    std::vector<double> vt(nsteps);
    for (int64_t k = 0; k < nsteps; ++k) vt[k] = v_next[(size_t)k * nsel + j];
    hip_check(hipMemcpyAsync(sl.v_table, C.stage(vt.data(), 8 * vt.size()), 8 * vt.size(), hipMemcpyHostToDevice,
                             C.stream),
              "v table");
    sl.v_len = (uint32_t)nsteps;
  }
  ensure_capacity(C, sl, cn, nsteps);
  write_counters(C, sl, cn);
  upload_dev(C, sl);
}

// now: the counters after the last launch of the call (read after it).
void finish_stats(Ctx& C, std::vector<Slot*>& sel, std::vector<Counters>& before, const std::vector<Counters>& now,
                  pic_step_stats* st) {
  pic_step_stats out;
  std::memset(&out, 0, sizeof(out));
  std::string err;
  for (size_t j = 0; j < sel.size(); ++j) {
    const Counters& c = now[j];
    const Counters& b = before[j];
    out.alive_start[0] += (int64_t)(c.stats[kStAlive0] - b.stats[kStAlive0]);
    out.alive_start[1] += (int64_t)(c.stats[kStAlive1] - b.stats[kStAlive1]);
    out.absorbed[0] += (int64_t)(c.stats[kStAbs0] - b.stats[kStAbs0]);
    out.absorbed[1] += (int64_t)(c.stats[kStAbs1] - b.stats[kStAbs1]);
    out.elastic += (int64_t)(c.stats[kStElastic] - b.stats[kStElastic]);
    out.ionization += (int64_t)(c.stats[kStIonization] - b.stats[kStIonization]);
    out.cx += (int64_t)(c.stats[kStCx] - b.stats[kStCx]);
    out.births += (int64_t)(c.stats[kStBirths] - b.stats[kStBirths]);
    out.numax_violations[0] += (int64_t)(c.stats[kStViol0] - b.stats[kStViol0]);
    out.numax_violations[1] += (int64_t)(c.stats[kStViol1] - b.stats[kStViol1]);
    out.lost_reflect += (int64_t)(c.stats[kStLostReflect] - b.stats[kStLostReflect]);
    if (c.flags & ~kFlagNeedRoom) {
      sel[j]->error_state = true;
      err = "capacity exceeded on the device (flags " + std::to_string(c.flags) + ")";
    }
  }
  if (st) {
    const double lm = st->loop_ms, sm = st->step_ms;
    const int64_t ll = st->loop_launches;
    *st = out;
    st->loop_ms = lm;
    st->step_ms = sm;
    st->loop_launches = ll;
  }
  if (!err.empty()) throw Err(PIC_E_CAPACITY, err);
}

std::vector<Slot*> selection(pic_ctx c, const pic_step_args* a) {
  std::vector<Slot*> sel;
  if (a->slots) {
    for (int j = 0; j < a->nslots; ++j) sel.push_back(&get_slot(c, a->slots[j]));
  } else {
    for (Slot& s : c->slots)
      if (s.live) sel.push_back(&s);
  }
  if (sel.empty()) throw Err(PIC_E_ARG, "no slots selected");
  return sel;
}

hipEvent_t get_event(Ctx& C, size_t i) {
  while (C.ev.size() <= i) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    C.ev.push_back(e);
  }
  return C.ev[i];
}

// One persistent launch per step over all selected slots (all 1D, or all
// quadtree slots with the corner-field coupling): the work items
// (slot, species, particle range) are listed largest slot first; per-slot
// constants come from a device table of InstDev.  With graph_steps > 0 the
// step sequence (particle loop, births, field solve + commit) is captured
// once into a HIP graph on the context's capture stream and replayed.
template <class T>
void batched_steps(Ctx& C, std::vector<Slot*>& sel, const pic_step_args* a, int64_t kbeg, int64_t kend,
                   double* loop_ms, Workspace* ws = nullptr) {
  const int nsel = (int)sel.size();
  const uint32_t tile = (uint32_t)(a->batched > 1 ? a->batched : 4096);
  if (tile % kBlock) throw Err(PIC_E_ARG, "batched tile must be a multiple of 256");
  bool ionizing = false, any_mcc = false;
  const bool dim2 = sel[0]->d.dim == 2;
  int maxn = 0;
  // the busiest ionizing slot of each ranking method (-1: none ranks that way)
  double pair_rate = -1.0, bin_rate = -1.0;
  for (Slot* s : sel) {
    if (!s->ionizing) continue;
    double& r = slot_births_binned(*s) ? bin_rate : pair_rate;
    r = std::max(r, s->births_rate);
  }
  std::vector<int> order(nsel);
  for (int j = 0; j < nsel; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return sel[x]->cap[0] + sel[x]->cap[1] > sel[y]->cap[0] + sel[y]->cap[1];
  });
  // work items grouped per slot, largest slot first; item k owns stats row k
  std::vector<WorkItem> issued;
  std::vector<uint32_t> rb(2 * (nsel + 1), 0);   // [row begin per slot][row end per slot]
  for (int j : order) {
    Slot& sl = *sel[j];
    ionizing = ionizing || sl.ionizing;
    any_mcc = any_mcc || slot_has_mcc(sl);
    maxn = std::max(maxn, sl.d.ncells);
    rb[j] = (uint32_t)issued.size();
    for (int sp = 0; sp < sl.d.nspecies; ++sp)
      for (int64_t b = 0; b < sl.cap[sp]; b += tile)
        issued.push_back(WorkItem{(uint32_t)j, (uint32_t)sp, (uint32_t)b,
                                  (uint32_t)std::min<int64_t>(b + tile, sl.cap[sp])});
    rb[nsel + 1 + j] = (uint32_t)issued.size();
  }
  // launch tables from the context's device memory source; a replaced table
  // is reusable after the next synchronization
  auto ensure = [&](void*& p, size_t& have, size_t need) {
    if (have >= need) return;
    if (p) C.pool.put(p, have);
    p = nullptr;
    have = 0;
    const size_t cls = DevPool::class_of(need);
    p = C.pool.get(cls);
    have = cls;
  };
  // the tables: the context's (pooled, kept between calls) or, without
  // allocation, carved from the workspace (the caller's drive tables sit
  // there already)
  void *t_items, *t_insts, *t_rowbeg, *t_jobs;
  unsigned long long* t_part;
  if (ws) {
    t_items = ws->take(sizeof(WorkItem) * issued.size());
    t_insts = ws->take(sizeof(InstDev<T>) * nsel);
    t_part = (unsigned long long*)ws->take(sizeof(unsigned long long) * kNStat * issued.size());
    t_rowbeg = ws->take(sizeof(uint32_t) * rb.size());
    t_jobs = ws->take(sizeof(SortJob<T>) * 2 * (size_t)nsel);
    // partial-stats rows start at zero (the workspace keeps the last call's contents)
    const size_t nrow = (size_t)kNStat * issued.size();
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<size_t>((nrow + 255) / 256, 1024)), dim3(256), 0,
                       C.stream, t_part, nrow);
    hip_check(hipGetLastError(), "zero rows");
  } else {
    ensure(C.b_items, C.b_items_bytes, sizeof(WorkItem) * issued.size());
    ensure(C.b_insts, C.b_insts_bytes, sizeof(InstDev<T>) * nsel);
    if (C.b_part_bytes < sizeof(unsigned long long) * kNStat * issued.size()) {
      ensure(*(void**)&C.b_part, C.b_part_bytes, sizeof(unsigned long long) * kNStat * issued.size());
      hip_check(hipMemsetAsync(C.b_part, 0, C.b_part_bytes, C.stream), "memset");
    }
    ensure(*(void**)&C.b_rowbeg, C.b_rowbeg_bytes, sizeof(uint32_t) * rb.size());
    ensure(C.b_jobs, C.b_jobs_bytes, sizeof(SortJob<T>) * 2 * (size_t)nsel);
    t_items = C.b_items;
    t_insts = C.b_insts;
    t_part = C.b_part;
    t_rowbeg = C.b_rowbeg;
    t_jobs = C.b_jobs;
  }
  hip_check(hipMemcpyAsync(t_items, C.stage(issued.data(), sizeof(WorkItem) * issued.size()),
                           sizeof(WorkItem) * issued.size(), hipMemcpyHostToDevice, C.stream),
            "items");
  hip_check(hipMemcpyAsync(t_rowbeg, C.stage(rb.data(), 4 * rb.size()), 4 * rb.size(), hipMemcpyHostToDevice,
                           C.stream),
            "rowbeg");
  // Batched sort of every selected slot (both species at once), replacing
  // per-slot sorts; the slots' own device descriptors are refreshed once at
  // the end of the call.
  bool sorted_any = false;
  auto sort_all = [&]() {
    std::vector<SortJob<T>> jobs(2 * (size_t)nsel);
    uint32_t max_ncell = 0;
    for (int j = 0; j < nsel; ++j) {
      Slot& sl = *sel[j];
      const uint32_t N = dim2 ? sl.nq : sort_bins_1d(sl);
      for (int sp = 0; sp < 2; ++sp) {
        SortJob<T>& J = jobs[2 * (size_t)j + sp];
        J.off = nullptr;   // no job for an absent species (every sort kernel skips it)
        J.ncell = 0;
        if (sp >= sl.d.nspecies || !sl.pb[sp][0].base) continue;
        J.ncell = N;
        check_sort_target(sl, sp);
        PBuf& d = sl.pb[sp][1 - sl.cur[sp]];
        J.off = sl.off + (size_t)sp * (N + 1);
        J.dst = SortDst<T>{(T*)d.s[0], (T*)d.s[1], (T*)d.v[0], (T*)d.v[1], (T*)d.v[2], d.w, d.id, d.cell,
                           (T*)d.s[2], (T*)d.acc};
        max_ncell = std::max(max_ncell, N);
      }
    }
    hip_check(hipMemcpyAsync(t_jobs, C.stage(jobs.data(), sizeof(SortJob<T>) * jobs.size()),
                             sizeof(SortJob<T>) * jobs.size(), hipMemcpyHostToDevice, C.stream),
              "sort jobs");
    hip_check(launch_sort_batched<T>((const InstDev<T>*)t_insts, (const SortJob<T>*)t_jobs, 2 * nsel, max_ncell,
                                     (const WorkItem*)t_items, (uint32_t)issued.size(),
                                     (int)std::min<size_t>(issued.size(), 2048), C.stream),
              "sort batched");
    for (int j = 0; j < nsel; ++j)
      for (int sp = 0; sp < sel[j]->d.nspecies; ++sp)
        if (jobs[2 * (size_t)j + sp].off) sel[j]->cur[sp] = 1 - sel[j]->cur[sp];
    sorted_any = true;
  };
  auto upload_insts = [&]() {
    std::vector<InstDev<T>> v(nsel);
    for (int j = 0; j < nsel; ++j) {
      v[j] = make_dev<T>(*sel[j]);
      if (ws && a->solve_field) {   // drive tables in the workspace: [slot][step] from its start
        v[j].v_table = (const double*)ws->base + (size_t)j * (size_t)(kend - kbeg);
        v[j].v_len = (uint32_t)(kend - kbeg);
      }
    }
    hip_check(hipMemcpyAsync(t_insts, C.stage(v.data(), sizeof(InstDev<T>) * nsel), sizeof(InstDev<T>) * nsel,
                             hipMemcpyHostToDevice, C.stream),
              "insts");
  };
  upload_insts();
  const int grid = (int)std::min<size_t>(issued.size(), (size_t)(a->grid > 0 ? a->grid : 2048));
  const InstDev<T>* dI = (const InstDev<T>*)t_insts;
  auto one_step = [&](hipStream_t st) {
    if (dim2)
      hip_check(launch_step2d_batched<T>(dI, (const WorkItem*)t_items, (uint32_t)issued.size(), t_part, st, grid,
                                         any_mcc),
                "step2d_batched");
    else
      hip_check(launch_step1d_batched<T>(dI, (const WorkItem*)t_items, (uint32_t)issued.size(), t_part, st, grid,
                                         any_mcc),
                "step1d_batched");
    if (ionizing)
      hip_check(launch_births_batched<T>(dI, nsel, st, pair_rate < 0 ? -1.0 : 2.0 * pair_rate,
                                         bin_rate < 0 ? -1.0 : 2.0 * bin_rate),
                "births_batched");
  };
  auto one_commit = [&](hipStream_t st) {
    if (a->solve_field && !dim2) hip_check(launch_field1d<T>(dI, nsel, maxn, 1, nullptr, st), "field1d batched");
    else hip_check(launch_commit_batched<T>(dI, nsel, st), "commit batched");
  };
  const int gsteps = a->graph_steps;
  if (gsteps > 0) {
    if (loop_ms) throw Err(PIC_E_ARG, "timing is not available with graph replay");
    // capture gsteps steps once; replay between sorts
    if (!C.cap_stream) hip_check(hipStreamCreateWithFlags(&C.cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!C.ev_a) hip_check(hipEventCreateWithFlags(&C.ev_a, hipEventDisableTiming), "event");
    if (!C.ev_b) hip_check(hipEventCreateWithFlags(&C.ev_b, hipEventDisableTiming), "event");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    C.sync();
    hip_check(hipStreamBeginCapture(C.cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    for (int k = 0; k < gsteps; ++k) {
      one_step(C.cap_stream);
      one_commit(C.cap_stream);
    }
    hip_check(hipStreamEndCapture(C.cap_stream, &graph), "end capture");
    hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
    int64_t k = kbeg, since_sort = 0;
    while (k < kend) {
      const int64_t k_prev = k;
      if (kend - k >= gsteps) {
        hip_check(hipEventRecord(C.ev_a, C.stream), "event");
        hip_check(hipStreamWaitEvent(C.cap_stream, C.ev_a, 0), "wait");
        hip_check(hipGraphLaunch(exec, C.cap_stream), "graph launch");
        hip_check(hipEventRecord(C.ev_b, C.cap_stream), "event");
        hip_check(hipStreamWaitEvent(C.stream, C.ev_b, 0), "wait");
        k += gsteps;
      } else {
        one_step(C.stream);
        one_commit(C.stream);
        ++k;
      }
      since_sort += k - k_prev;
      if (a->sort_every > 0 && k < kend && since_sort >= a->sort_every) {
        sort_all();
        upload_insts();
        since_sort = 0;
      }
    }
    C.sync();
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
  } else {
    for (int64_t k = kbeg; k < kend; ++k) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (loop_ms) {
        e0 = get_event(C, 2 + 2 * (k - kbeg));
        e1 = get_event(C, 3 + 2 * (k - kbeg));
        hip_check(hipEventRecord(e0, C.stream), "event");
      }
      one_step(C.stream);
      if (e1) hip_check(hipEventRecord(e1, C.stream), "event");
      one_commit(C.stream);
      if (a->sort_every > 0 && (k + 1) % a->sort_every == 0 && k + 1 < kend) {
        sort_all();
        upload_insts();
      }
    }
  }
  hip_check(launch_stats_reduce<T>(dI, nsel, t_part, (const uint32_t*)t_rowbeg, 0u, C.stream), "stats_reduce batched");
  if (sorted_any)
    for (Slot* s : sel) upload_dev(C, *s);
  if (loop_ms) {
    C.sync();
    for (int64_t k = kbeg; k < kend; ++k) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, C.ev[2 + 2 * (k - kbeg)], C.ev[3 + 2 * (k - kbeg)]), "elapsed");
      *loop_ms += ms;
    }
  }
}

}  // namespace

extern "C" {

int pic_abi_version(void) { return PIC_ABI_VERSION; }

const char* pic_last_error(pic_ctx c) { return c ? c->err.c_str() : g_last_error.c_str(); }

int pic_mesh_build(const pic_instance_desc* descs, int ninst, void* stream, pic_ctx* out) {
  pic_ctx c = nullptr;
  PIC_GUARD_BEGIN
  if (ninst < 0 || (ninst > 0 && !descs) || !out) throw Err(PIC_E_ARG, "need descriptors and an output handle");
  c = new pic_ctx_s();
  c->stream = (hipStream_t)stream;
  c->arena_size = 8u << 20;
  hip_check(hipHostMalloc(&c->arena, c->arena_size, hipHostMallocDefault), "hipHostMalloc");
  c->slots.resize(ninst);
  for (int i = 0; i < ninst; ++i) build_slot(*c, c->slots[i], descs[i]);
  for (int i = 0; i < ninst; ++i) upload_dev(*c, c->slots[i]);
  c->sync();
  *out = c;
  return PIC_OK;
  }
  catch (const Err& e) {
    g_last_error = e.msg;
    if (c) pic_destroy(c);
    return e.code;
  }
}

void pic_destroy(pic_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (Slot& s : c->slots) s.release_all();
  c->release_tables();
  c->pool.clear();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->ev_a) (void)hipEventDestroy(c->ev_a);
  if (c->ev_b) (void)hipEventDestroy(c->ev_b);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->arena) (void)hipHostFree(c->arena);
  delete c;
}

int pic_set_stream(pic_ctx c, void* stream) {
  PIC_GUARD_BEGIN
  if (!c) throw Err(PIC_E_ARG, "null context");
  c->sync();
  c->stream = (hipStream_t)stream;
  c->pool.stream = c->stream;
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_set_allocator(pic_ctx c, const pic_allocator* a) {
  PIC_GUARD_BEGIN
  if (!c) throw Err(PIC_E_ARG, "null context");
  if (a && (!a->alloc || !a->free)) throw Err(PIC_E_ARG, "allocator needs alloc and free");
  for (const Slot& s : c->slots)
    if (s.live || !s.allocs.empty()) throw Err(PIC_E_STATE, "the context already holds instances");
  c->sync();
  c->release_tables();
  c->pool.clear();   // blocks of the previous source go back to it
  c->pool.has_ext = a != nullptr;
  c->pool.ext = a ? *a : pic_allocator{};
  c->pool.stream = c->stream;
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_sync(pic_ctx c) {
  PIC_GUARD_BEGIN
  if (!c) throw Err(PIC_E_ARG, "null context");
  c->sync();
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_num_slots(pic_ctx c) { return c ? (int)c->slots.size() : 0; }

int pic_particles_load(pic_ctx c, int slot, int species, int64_t n, const double* s, const double* v,
                       const uint32_t* w, const uint32_t* id) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (species < 0 || species >= sl.d.nspecies) throw Err(PIC_E_ARG, "bad species");
  if (n < 0 || n > 0x7FFFFFFF || (n > 0 && (!s || !v))) throw Err(PIC_E_ARG, "bad particle arrays");
  const int dim = sl.d.dim;
  for (int64_t i = 0; i < n * dim; ++i)
    if (!in_unit(s[i], sl.prec)) throw Err(PIC_E_ARG, "position outside [0,1) in the particle precision");
  std::vector<uint32_t> ww(n), ii(n);
  uint32_t mx = 0;
  for (int64_t i = 0; i < n; ++i) {
    ww[i] = w ? w[i] : 65536u;
    ii[i] = id ? id[i] : (uint32_t)i;
    if (ww[i] == 0u) throw Err(PIC_E_ARG, "particle weight must be positive");
    mx = std::max(mx, ii[i]);
  }
  int64_t cap = sl.d.capacity[species] > 0 ? std::max<int64_t>(sl.d.capacity[species], n)
                                            : (sl.ionizing ? 3 * n + 4096 : n);
  cap = std::max<int64_t>(cap, 256);
  cap = (cap + 255) & ~(int64_t)255;
  Counters cn = read_counters(*c, sl);
  // Room first: births staging, then the particle buffers, each whole or not
  // done, so a failed allocation leaves the slot as it was.  A failure after
  // the old particles are overwritten marks the slot failed.
  const bool fresh = cap > sl.cap[species] || !sl.pb[species][0].base;
  const int64_t cap0 = species == 0 && fresh ? cap : sl.cap[0];
  if (sl.ionizing && sl.birth_cap < (uint64_t)cap0) alloc_births(*c, sl, cap0);
  if (fresh) alloc_particles(sl, species, cap);
  try {
    sl.cur[species] = 0;
    const PBuf& b = sl.pb[species][0];
    const size_t e = sl.esz;
    std::vector<char> tmp(e * (size_t)std::max<int64_t>(n, 1));
    auto put = [&](void* dst, const double* src, int stride, int comp) {
      if (e == 4) {
        float* f = (float*)tmp.data();
        for (int64_t i = 0; i < n; ++i) f[i] = (float)src[i * stride + comp];
      } else {
        double* f = (double*)tmp.data();
        for (int64_t i = 0; i < n; ++i) f[i] = src[i * stride + comp];
      }
      hip_check(hipMemcpy(dst, tmp.data(), e * n, hipMemcpyHostToDevice), "load");
    };
    if (n) {
      for (int k = 0; k < dim; ++k) put(b.s[k], s, dim, k);
      for (int k = 0; k < 3; ++k) put(b.v[k], v, 3, k);
      hip_check(hipMemcpy(b.w, ww.data(), 4 * n, hipMemcpyHostToDevice), "load");
      hip_check(hipMemcpy(b.id, ii.data(), 4 * n, hipMemcpyHostToDevice), "load");
      if (b.acc) hip_check(hipMemset(b.acc, 0, e * n), "load");   // no filtered acceleration before the start
      sl.max_id_loaded[species] = mx + 1u;
    } else {
      sl.max_id_loaded[species] = 0;
    }
    cn.count[species] = (uint32_t)n;
    cn.next_id = std::max(cn.next_id, std::max(sl.max_id_loaded[0], sl.max_id_loaded[1]));
    write_counters(*c, sl, cn);
    if (dim >= 2 && n) {
      if (sl.prec == 32) hip_check(launch_relocate<float>(make_dev<float>(sl), species, c->stream, grid_for(n)), "relocate");
      else hip_check(launch_relocate<double>(make_dev<double>(sl), species, c->stream, grid_for(n)), "relocate");
    }
    // start cell-ordered, so deposits and gathers of a workgroup cluster
    if (n) sort_slot(*c, sl);
    upload_dev(*c, sl);
    c->sync();
  } catch (...) {
    sl.error_state = true;
    throw;
  }
  return PIC_OK;
  PIC_GUARD_END(c)
}

int64_t pic_count(pic_ctx c, int slot, int species) {
  PIC_GUARD_BEGIN
  Slot& sl = get_slot(c, slot);
  if (species < 0 || species >= sl.d.nspecies) throw Err(PIC_E_ARG, "bad species");
  Counters cn = read_counters(*c, sl);
  const uint32_t n = cn.count[species];
  if (!n) return 0;
  std::vector<uint32_t> w(n);
  hip_check(hipMemcpy(w.data(), sl.pb[species][sl.cur[species]].w, 4 * (size_t)n, hipMemcpyDeviceToHost), "read");
  return (int64_t)std::count_if(w.begin(), w.end(), [](uint32_t x) { return x != 0u; });
  PIC_GUARD_END(c)
}

uint32_t pic_next_id(pic_ctx c, int slot) {
  try {
    Slot& sl = get_slot(c, slot);
    return read_counters(*c, sl).next_id;
  } catch (...) {
    return 0;
  }
}

int pic_particles_read(pic_ctx c, int slot, int species, double* s, double* v, uint32_t* w, uint32_t* id,
                       uint32_t* cell) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (species < 0 || species >= sl.d.nspecies) throw Err(PIC_E_ARG, "bad species");
  Counters cn = read_counters(*c, sl);
  const size_t n = cn.count[species];
  const PBuf& b = sl.pb[species][sl.cur[species]];
  const int dim = sl.d.dim;
  const size_t e = sl.esz;
  std::vector<uint32_t> hw(n), hid(n), hc(n, 0);
  std::vector<double> hs(n * dim), hv(n * 3);
  if (n) {
    hip_check(hipMemcpy(hw.data(), b.w, 4 * n, hipMemcpyDeviceToHost), "read");
    hip_check(hipMemcpy(hid.data(), b.id, 4 * n, hipMemcpyDeviceToHost), "read");
    if (dim >= 2) hip_check(hipMemcpy(hc.data(), b.cell, 4 * n, hipMemcpyDeviceToHost), "read");
    std::vector<char> tmp(e * n);
    auto get = [&](const void* src, double* dst, int stride, int comp) {
      hip_check(hipMemcpy(tmp.data(), src, e * n, hipMemcpyDeviceToHost), "read");
      for (size_t i = 0; i < n; ++i)
        dst[i * stride + comp] = e == 4 ? (double)((float*)tmp.data())[i] : ((double*)tmp.data())[i];
    };
    for (int k = 0; k < dim; ++k) get(b.s[k], hs.data(), dim, k);
    for (int k = 0; k < 3; ++k) get(b.v[k], hv.data(), 3, k);
  }
  std::vector<size_t> order;
  for (size_t i = 0; i < n; ++i)
    if (hw[i]) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](size_t a, size_t bb) { return hid[a] < hid[bb]; });
  for (size_t j = 0; j < order.size(); ++j) {
    const size_t i = order[j];
    if (s) for (int k = 0; k < dim; ++k) s[j * dim + k] = hs[i * dim + k];
    if (v) for (int k = 0; k < 3; ++k) v[j * 3 + k] = hv[i * 3 + k];
    if (w) w[j] = hw[i];
    if (id) id[j] = hid[i];
    if (cell) {
      if (dim >= 2) {
        cell[j] = hc[i];
      } else {
        const int N = sl.d.ncells;
        int64_t ic;
        if (e == 4) ic = (int64_t)std::floor((float)hs[i] * (float)N);
        else ic = (int64_t)std::floor(hs[i] * (double)N);
        if (ic > N - 1) ic = N - 1;
        cell[j] = (uint32_t)ic;
      }
    }
  }
  return PIC_OK;
  PIC_GUARD_END(c)
}

int64_t pic_nleaves(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  Slot& sl = get_slot(c, slot);
  return sl.d.dim >= 2 ? (int64_t)sl.nleaves : 0;
  PIC_GUARD_END(c)
}

int pic_leaves_read(pic_ctx c, int slot, uint32_t* keys, uint8_t* levels) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (sl.d.dim < 2) throw Err(PIC_E_ARG, "not a tree slot");
  c->sync();
  if (keys) hip_check(hipMemcpy(keys, sl.key, 4 * (size_t)sl.nleaves, hipMemcpyDeviceToHost), "read");
  if (levels) hip_check(hipMemcpy(levels, sl.lv, sl.nleaves, hipMemcpyDeviceToHost), "read");
  return PIC_OK;
  PIC_GUARD_END(c)
}

int64_t pic_nq(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  return (int64_t)get_slot(c, slot).nq;
  PIC_GUARD_END(c)
}

int pic_field_set(pic_ctx c, int slot, int kind, const double* data) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (!data) throw Err(PIC_E_ARG, "null data");
  if (sl.d.dim == 1) {
    const bool ec = sl.d.field_scheme == PIC_FIELD_CIC_EC;
    if (kind != PIC_NODE_E_1D && kind != PIC_NODE_PHI_1D && kind != PIC_CELL_E_1D)
      throw Err(PIC_E_ARG, "bad field kind for 1D");
    if (kind == PIC_NODE_E_1D && ec) throw Err(PIC_E_ARG, "node E is for the momentum-conserving coupling (use PIC_CELL_E_1D)");
    if (kind == PIC_CELL_E_1D && !ec) throw Err(PIC_E_ARG, "cell E is for the energy-conserving coupling (use PIC_NODE_E_1D)");
    if (kind == PIC_CELL_E_1D) {   // N cell values, the unused last entry 0
      std::vector<double> e(data, data + sl.d.ncells);
      e.push_back(0.0);
      hip_check(hipMemcpy(sl.phi64, e.data(), 8 * e.size(), hipMemcpyHostToDevice), "upload");
    } else {
      hip_check(hipMemcpy(sl.phi64, data, 8 * (size_t)(sl.d.ncells + 1), hipMemcpyHostToDevice), "upload");
    }
    // data staged in phi64 (node potential or node E) -> E table
    if (sl.prec == 32) hip_check(launch_node_e_1d<float>(make_dev<float>(sl), sl.phi64, kind == PIC_NODE_PHI_1D, c->stream), "node_e");
    else hip_check(launch_node_e_1d<double>(make_dev<double>(sl), sl.phi64, kind == PIC_NODE_PHI_1D, c->stream), "node_e");
    c->sync();
    return PIC_OK;
  }
  if (sl.d.dim == 3) {   // octree: corner potentials -> nodal E, or corner E given
    const Mesh2D m3 = mesh_of(sl);
    const size_t n3 = sl.nleaves;
    if (kind == PIC_CORNER_PHI_3D) {
      hip_check(hipMemcpy(sl.cphi, data, 8 * 8 * n3, hipMemcpyHostToDevice), "upload");
      if (sl.prec == 32) hip_check(launch_corner_field3<float>(m3, sl.cphi, sl.grad, sl.e64, (float*)sl.E, c->stream), "corner3");
      else hip_check(launch_corner_field3<double>(m3, sl.cphi, sl.grad, sl.e64, (double*)sl.E, c->stream), "corner3");
    } else if (kind == PIC_CORNER_E_3D) {
      hip_check(hipMemcpy(sl.e64, data, 8 * 24 * n3, hipMemcpyHostToDevice), "upload");
      if (sl.prec == 32) hip_check(launch_round_table<float>(sl.e64, (float*)sl.E, (int64_t)(24 * n3), c->stream), "round");
      else hip_check(launch_round_table<double>(sl.e64, (double*)sl.E, (int64_t)(24 * n3), c->stream), "round");
    } else {
      throw Err(PIC_E_ARG, "bad field kind for 3D");
    }
    c->sync();
    return PIC_OK;
  }
  const Mesh2D m = mesh_of(sl);
  const size_t n = sl.nleaves;
  if (kind == PIC_CORNER_PHI_2D) {
    hip_check(hipMemcpy(sl.cphi, data, 8 * 4 * n, hipMemcpyHostToDevice), "upload");
  } else if (kind == PIC_CELL_PHI_2D) {
    hip_check(hipMemcpy(sl.phi64, data, 8 * n, hipMemcpyHostToDevice), "upload");
    hip_check(launch_cell_to_corner_phi(m, sl.phi64, sl.cphi, c->stream), "cell_to_corner");
  } else if (kind == PIC_CORNER_E_2D) {
    hip_check(hipMemcpy(sl.e64, data, 8 * 8 * n, hipMemcpyHostToDevice), "upload");
    if (sl.prec == 32) hip_check(launch_round_table<float>(sl.e64, (float*)sl.E, (int64_t)(8 * n), c->stream), "round");
    else hip_check(launch_round_table<double>(sl.e64, (double*)sl.E, (int64_t)(8 * n), c->stream), "round");
    refresh_cell_e(*c, sl);
    c->sync();
    return PIC_OK;
  } else if (kind == PIC_CELL_E_2D) {   // the cloud's gather table, given directly
    if (sl.d.field_scheme != PIC_FIELD_CIC_AMR) throw Err(PIC_E_ARG, "cell E is for cloud-in-cell slots");
    double* tmp = (double*)sl.alloc(8 * 2 * n);
    hip_check(hipMemcpy(tmp, data, 8 * 2 * n, hipMemcpyHostToDevice), "upload");
    if (sl.prec == 32) hip_check(launch_round_table<float>(tmp, (float*)sl.cellE, (int64_t)(2 * n), c->stream), "round");
    else hip_check(launch_round_table<double>(tmp, (double*)sl.cellE, (int64_t)(2 * n), c->stream), "round");
    c->sync();
    sl.release(tmp);
    return PIC_OK;
  } else {
    throw Err(PIC_E_ARG, "bad field kind for 2D");
  }
  if (sl.prec == 32) hip_check(launch_corner_field<float>(m, sl.cphi, sl.grad, sl.e64, (float*)sl.E, c->stream), "corner");
  else hip_check(launch_corner_field<double>(m, sl.cphi, sl.grad, sl.e64, (double*)sl.E, c->stream), "corner");
  refresh_cell_e(*c, sl);
  c->sync();
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_field_read(pic_ctx c, int slot, double* out) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  const bool cic = sl.d.dim == 2 && sl.d.field_scheme == PIC_FIELD_CIC_AMR;
  const size_t n = sl.d.dim == 1 ? (size_t)sl.d.ncells + 1
                   : sl.d.dim == 3 ? (size_t)sl.nleaves * 24 : (size_t)sl.nleaves * (cic ? 2 : 8);
  std::vector<char> tmp(sl.esz * n);
  c->sync();
  hip_check(hipMemcpy(tmp.data(), cic ? sl.cellE : sl.E, sl.esz * n, hipMemcpyDeviceToHost), "read");
  for (size_t i = 0; i < n; ++i) out[i] = sl.esz == 4 ? (double)((float*)tmp.data())[i] : ((double*)tmp.data())[i];
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_leapfrog_start(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  const int g = grid_for(std::max(sl.cap[0], sl.cap[1]));
  if (sl.prec == 32) hip_check(launch_leapfrog_start<float>(make_dev<float>(sl), c->stream, g), "leapfrog");
  else hip_check(launch_leapfrog_start<double>(make_dev<double>(sl), c->stream, g), "leapfrog");
  c->sync();
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_deposit(pic_ctx c, int slot, uint64_t* q_out, double* rho_out) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  hip_check(hipMemsetAsync(sl.Q, 0, 32 * (size_t)sl.nq, c->stream), "memset");
  const int g = grid_for(std::max(sl.cap[0], sl.cap[1]));
  if (sl.prec == 32) hip_check(launch_deposit<float>(make_dev<float>(sl), c->stream, g), "deposit");
  else hip_check(launch_deposit<double>(make_dev<double>(sl), c->stream, g), "deposit");
  Counters cn = read_counters(*c, sl);
  const unsigned long long* latest = sl.Q + (size_t)((cn.step + 1u) & 1u) * 2u * sl.nq;
  if (q_out) hip_check(hipMemcpy(q_out, latest, 8 * 2 * (size_t)sl.nq, hipMemcpyDeviceToHost), "read");
  if (rho_out) {
    const int F = sl.prec == 32 ? 24 : 32;
    double qw0[2] = {0.0, 0.0};
    for (int sp = 0; sp < sl.d.nspecies; ++sp) qw0[sp] = sl.d.species[sp].charge * sl.d.species[sp].w0;
    double* r = (double*)sl.alloc(8 * (size_t)sl.nq);
    const bool tree = sl.d.dim >= 2;
    const bool cloud = !tree || sl.d.field_scheme == PIC_FIELD_CIC_AMR;   // shares carry F more bits
    hip_check(launch_rho(latest, sl.nq, sl.d.nspecies, qw0[0], qw0[1], cloud ? 16 + F : 16,
                         tree ? 0.0 : sl.d.length / sl.d.ncells, tree ? sl.lv : nullptr, sl.d.length, sl.d.depth_z,
                         sl.d.dim == 3 ? 1 : 0, r, c->stream),
              "rho");
    hip_check(hipMemcpyAsync(rho_out, r, 8 * (size_t)sl.nq, hipMemcpyDeviceToHost, c->stream), "read");
    c->sync();
    sl.release(r);
  }
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_set_births_ranking(pic_ctx c, int slot, int method) {
  PIC_GUARD_BEGIN
  if (method < 0 || method > 2) throw Err(PIC_E_ARG, "births ranking method must be 0, 1 or 2");
  usable_slot(c, slot).births_method = method;
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_deposit_read(pic_ctx c, int slot, uint64_t* q_out) {
  PIC_GUARD_BEGIN
  if (!q_out) throw Err(PIC_E_ARG, "null output");
  Slot& sl = usable_slot(c, slot);
  Counters cn = read_counters(*c, sl);
  const unsigned long long* latest = sl.Q + (size_t)((cn.step + 1u) & 1u) * 2u * sl.nq;
  hip_check(hipMemcpy(q_out, latest, 8 * 2 * (size_t)sl.nq, hipMemcpyDeviceToHost), "read");
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_field_solve(pic_ctx c, int slot, double phi_left, const double* phi_init, double rtol, int maxit,
                    double* phi_out, double* e_out, int* iters, double* relres) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (sl.d.dim == 1) {
    double* pl = (double*)c->stage(&phi_left, sizeof(double));
    upload_dev(*c, sl);
    if (sl.prec == 32)
      hip_check(launch_field1d<float>((const InstDev<float>*)sl.devI, 1, sl.d.ncells, 0, pl, c->stream), "field1d");
    else
      hip_check(launch_field1d<double>((const InstDev<double>*)sl.devI, 1, sl.d.ncells, 0, pl, c->stream), "field1d");
    c->sync();
    const size_t n = (size_t)sl.d.ncells + 1;
    if (phi_out) hip_check(hipMemcpy(phi_out, sl.phi64, 8 * n, hipMemcpyDeviceToHost), "read");
    if (e_out) hip_check(hipMemcpy(e_out, sl.e64, 8 * n, hipMemcpyDeviceToHost), "read");
    if (iters) *iters = 1;
    if (relres) *relres = 0.0;
    return PIC_OK;
  }
  if (sl.d.dim == 3) throw Err(PIC_E_ARG, "octree slots take their field at the nodes (no solve)");
  const Mesh2D m = mesh_of(sl);
  const uint32_t n = sl.nleaves;
  if (!sl.stencil_ok) {
    for (void* p : {(void*)sl.st.nbr, (void*)sl.st.code, (void*)sl.st.diag, (void*)sl.st.bnd, (void*)sl.cg_ws})
      sl.release(p);
    sl.st = Stencil2D{nullptr, nullptr, nullptr, nullptr};   // (a failed allocation below leaves them null;
    sl.cg_ws = nullptr;                                        // stencil_ok stays false until all are built)
    sl.st.nbr = (uint32_t*)sl.alloc(4 * 8 * (size_t)n);
    sl.st.code = (uint32_t*)sl.alloc(4 * ((size_t)n + 1));
    sl.st.diag = (double*)sl.alloc(8 * (size_t)n);
    sl.st.bnd = (double*)sl.alloc(8 * (size_t)n);
    sl.cg_ws = (double*)sl.alloc(8 * (size_t)cg_ws_doubles(n));
    hip_check(hipMemsetAsync(sl.st.code + n, 0, 4, c->stream), "memset");
    hip_check(launch_build_stencil(m, sl.st, c->stream), "stencil");
    uint32_t bad = 0;
    hip_check(hipMemcpyAsync(&bad, sl.st.code + n, 4, hipMemcpyDeviceToHost, c->stream), "read");
    c->sync();
    if (bad) throw Err(PIC_E_STATE, "the tree is not 2:1 balanced across faces");
    sl.stencil_ok = true;
  }
  if (phi_init) hip_check(hipMemcpy(sl.phi64, phi_init, 8 * (size_t)n, hipMemcpyHostToDevice), "upload");
  Counters cn = read_counters(*c, sl);
  const unsigned long long* latest = sl.Q + (size_t)((cn.step + 1u) & 1u) * 2u * sl.nq;
  const double rtol2 = rtol * rtol;
  const uint32_t maxit_u = maxit > 0 ? (uint32_t)maxit : 0u;
  hip_check(launch_cg_setup(m, sl.st, latest, sl.d.nspecies, sl.kappa, sl.phi64, sl.cg_ws, c->stream), "cg_setup");
  // Iterations are queued in growing batches; the device stops them itself
  // once the residual test holds (a batch may end in no-op launches).  The
  // launch of iteration maxit only checks, so the loop always ends.
  const CgScal* scd = (const CgScal*)(sl.cg_ws + cg_scalars_offset(n));
  CgScal sc{};
  uint32_t k = 0;
  // a warm-started solve takes about as many iterations as the last one:
  // queue three quarters of that before the first read of the scalars
  int batch = std::max(4, std::min(1024, (int)(sl.cg_iters_prev / 4u * 3u)));
  for (;;) {
    const uint32_t kend = (uint32_t)std::min<uint64_t>((uint64_t)k + (uint64_t)batch, (uint64_t)maxit_u + 1u);
    for (; k < kend; ++k)
      hip_check(launch_cg_iter(m, sl.st, sl.phi64, sl.cg_ws, k, rtol2, maxit_u, c->stream), "cg_iter");
    hip_check(hipMemcpyAsync(&sc, scd, sizeof(sc), hipMemcpyDeviceToHost, c->stream), "read");
    c->sync();
    if (sc.done) break;
    if (k > maxit_u) throw Err(PIC_E_STATE, "CG did not stop");
    batch = std::min(batch * 2, 64);
  }
  const int it = (int)sc.it;
  sl.cg_iters_prev = sc.it;
  const double rr = sc.rr, bb = sc.bb;
  hip_check(launch_cell_to_corner_phi(m, sl.phi64, sl.cphi, c->stream), "cell_to_corner");
  if (sl.prec == 32) hip_check(launch_corner_field<float>(m, sl.cphi, sl.grad, sl.e64, (float*)sl.E, c->stream), "corner");
  else hip_check(launch_corner_field<double>(m, sl.cphi, sl.grad, sl.e64, (double*)sl.E, c->stream), "corner");
  refresh_cell_e(*c, sl);
  c->sync();
  if (phi_out) hip_check(hipMemcpy(phi_out, sl.phi64, 8 * (size_t)n, hipMemcpyDeviceToHost), "read");
  if (e_out) hip_check(hipMemcpy(e_out, sl.e64, 8 * 8 * (size_t)n, hipMemcpyDeviceToHost), "read");
  if (iters) *iters = it;
  const double res = bb > 0 ? std::sqrt(rr) / std::sqrt(bb) : 0.0;
  if (relres) *relres = res;
  // the device's stopping test, repeated: rr <= rtol^2 bb
  if (!(bb > 0 ? rr <= rtol2 * bb : true)) throw Err(PIC_E_NUMERIC, "CG did not reach the tolerance");
  return PIC_OK;
  PIC_GUARD_END(c)
}

static void step_impl(pic_ctx c, const pic_step_args* a, pic_step_stats* stats, bool noalloc) {
  if (!c || !a || a->nsteps < 0) throw Err(PIC_E_ARG, "bad step arguments");
  std::vector<Slot*> sel = selection(c, a);
  const int nsel = (int)sel.size();
  if (stats) {
    stats->loop_ms = 0;
    stats->step_ms = 0;
    stats->loop_launches = 0;
  }
  if (a->timing < 0) throw Err(PIC_E_ARG, "timing must be >= 0");
  if (noalloc && (a->batched <= 0 || a->graph_steps != 0 || a->timing != 0))
    throw Err(PIC_E_ARG, "the no-allocation step takes batched launches without graph replay or timing");
  if (a->batched)
    for (Slot* s : sel) {
      if (s->d.dim != sel[0]->d.dim || s->prec != sel[0]->prec)
        throw Err(PIC_E_ARG, "batched steps need slots of one dimension and one precision");
      if (s->d.dim == 2 && s->d.field_scheme == PIC_FIELD_CIC_AMR)
        throw Err(PIC_E_ARG, "batched steps take quadtree slots with the corner-field coupling");
      if (s->d.dim == 3) throw Err(PIC_E_ARG, "octree slots step one by one (no batched launch)");
      if (s->d.field_scheme == PIC_FIELD_DIPIC) throw Err(PIC_E_ARG, "direct implicit slots step one by one");
    }
  for (Slot* s : sel)
    if (s->d.field_scheme == PIC_FIELD_DIPIC && !a->solve_field)
      throw Err(PIC_E_ARG, "a direct implicit step solves the field (set solve_field and v_next)");
  for (Slot* s : sel)
    if (s->error_state) throw Err(PIC_E_STATE, "slot is in an error state (retire it)");
  bool any_ionizing = false;
  for (Slot* s : sel) any_ionizing = any_ionizing || s->ionizing;
  // without allocation the drive tables of a chunk sit in the workspace
  const int64_t chunk = (any_ionizing || noalloc) ? 64 : std::max(a->nsteps, 1);
  char* ws_base = noalloc ? (char*)scratch_device_ptr() : nullptr;
  // The call's steps are k = 0 .. nsteps-1 of every selected slot; slot j
  // runs its step k as global step start[j] + k.  Slots run in groups of
  // equal progress: a slot whose step found no room for its births stops at
  // its last committed step (the device leaves it untouched), is grown on
  // the host and continues later from there, with the same draws (they
  // depend on particle id and step only), so the result equals a run that
  // never stopped.
  std::vector<Counters> before = read_counters_many(*c, sel);
  std::vector<uint32_t> start(nsel);
  for (int j = 0; j < nsel; ++j) {
    start[j] = a->step0 >= 0 ? (uint32_t)a->step0 : before[j].step;
    if (before[j].step != start[j]) {
      Counters cn = before[j];
      cn.step = start[j];
      write_counters(*c, *sel[j], cn);
      before[j].step = start[j];
    }
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (a->timing) {
    t0 = get_event(*c, 0);
    t1 = get_event(*c, 1);
  }
  bool started = false;
  double loop_ms = 0;
  int64_t launches = 0;
  std::vector<int64_t> stalled(nsel, -1);   // progress at which a slot last stopped for room
  std::vector<int64_t> grown_at(nsel, -1);  // progress at which a stopped slot was last grown
  int64_t room_stops = 0;
  // the counters at the top of each round: those just read for the first,
  // then a fresh read after the round's launches (the last one also gives
  // the call's statistics)
  std::vector<Counters> cur = before;
  bool fresh = true;
  for (;;) {
    if (!fresh) cur = read_counters_many(*c, sel);
    fresh = false;
    int64_t dmin = a->nsteps;
    std::vector<int64_t> done(nsel);
    for (int j = 0; j < nsel; ++j) {
      done[j] = (int64_t)(uint32_t)(cur[j].step - start[j]);
      if (cur[j].flags & kFlagNeedRoom) {
        // stopped again at the step it was grown for: the growth did not help
        if (grown_at[j] == done[j]) throw Err(PIC_E_CAPACITY, "no room for the next step after growing the slot");
        if (stalled[j] != done[j]) ++room_stops;
        stalled[j] = done[j];
      }
      if (done[j] < a->nsteps) dmin = std::min(dmin, done[j]);
    }
    if (dmin >= a->nsteps) break;
    std::vector<Slot*> grp;
    std::vector<int> gj;
    for (int j = 0; j < nsel; ++j)
      if (done[j] == dmin) {
        grp.push_back(sel[j]);
        gj.push_back(j);
      }
    const int64_t n = std::min<int64_t>(chunk, a->nsteps - dmin);
    pic_step_args sub = *a;
    sub.step0 = -1;
    sub.nsteps = (int)n;
    const int ng = (int)grp.size();
    std::vector<double> vn;
    if (a->solve_field && a->v_next) {
      vn.resize((size_t)n * ng);
      for (int64_t k = 0; k < n; ++k)
        for (int q = 0; q < ng; ++q) vn[(size_t)k * ng + q] = a->v_next[(size_t)(dmin + k) * nsel + gj[q]];
      sub.v_next = vn.data();
    }
    Workspace ws{ws_base, kNoAllocScratchBytes, 0};
    if (noalloc && a->solve_field) {
      if (!a->v_next) throw Err(PIC_E_ARG, "solve_field needs v_next");
      // drive tables [slot][step], the layout batched_steps reads
      std::vector<double> vt((size_t)n * ng);
      for (int q = 0; q < ng; ++q)
        for (int64_t k = 0; k < n; ++k) vt[(size_t)q * n + k] = vn[(size_t)k * ng + q];
      void* dv = ws.take(8 * vt.size());
      hip_check(hipMemcpyAsync(dv, c->stage(vt.data(), 8 * vt.size()), 8 * vt.size(), hipMemcpyHostToDevice,
                               c->stream),
                "drive tables");
    }
    {
      // the counters and device views of the group go out in one gathered
      // upload (a no-allocation step uploads them one by one)
      struct Defer {
        Ctx& c;
        Defer(Ctx& c_, bool on) : c(c_) { c.defer_uploads = on; }
        ~Defer() {
          c.defer_uploads = false;
          try {
            c.flush_uploads();
          } catch (...) {
          }
        }
      } defer(*c, !noalloc);
      for (int q = 0; q < ng; ++q) {
        if (cur[gj[q]].flags & kFlagNeedRoom) grown_at[gj[q]] = dmin;
        prepare_slot(*c, *grp[q], &sub, sub.v_next, q, ng, n, cur[gj[q]], noalloc);
      }
      c->defer_uploads = false;
      c->flush_uploads();
    }
    if (a->timing && !started) {   // the call's wall time starts after the first preparation
      hip_check(hipEventRecord(t0, c->stream), "event");
      started = true;
    }
    if (a->batched) {
      double lm = 0;
      Workspace* w = noalloc ? &ws : nullptr;
      if (grp[0]->prec == 32) batched_steps<float>(*c, grp, &sub, 0, n, a->timing ? &lm : nullptr, w);
      else batched_steps<double>(*c, grp, &sub, 0, n, a->timing ? &lm : nullptr, w);
      loop_ms += lm;
      if (a->timing) launches += n;
    } else {
      std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
      for (int64_t k = 0; k < n; ++k) {
        for (int q = 0; q < ng; ++q) {
          Slot& sl = *grp[q];
          hipEvent_t e0 = nullptr, e1 = nullptr;
          if (a->timing > 0 && (dmin + k) % a->timing == 0) {
            e0 = get_event(*c, 2 + 2 * evs.size());
            e1 = get_event(*c, 3 + 2 * evs.size());
            evs.push_back({e0, e1});
          }
          const int g = step_grid(sl, a->grid);
          if (sl.prec == 32) plain_step<float>(*c, sl, a->solve_field != 0, g, e0, e1);
          else plain_step<double>(*c, sl, a->solve_field != 0, g, e0, e1);
          if (a->sort_every > 0 && (dmin + k + 1) % a->sort_every == 0) sort_slot(*c, sl);
        }
      }
      for (int q = 0; q < ng; ++q) {
        const int g = step_grid(*grp[q], a->grid);
        if (grp[q]->prec == 32) reduce_plain_stats<float>(*c, *grp[q], g);
        else reduce_plain_stats<double>(*c, *grp[q], g);
      }
      if (a->timing) {
        c->sync();
        for (auto& p : evs) {
          float ms = 0;
          hip_check(hipEventElapsedTime(&ms, p.first, p.second), "elapsed");
          loop_ms += ms;
        }
        launches += (int64_t)evs.size();
      }
    }
  }
  if (a->timing && started) {
    hip_check(hipEventRecord(t1, c->stream), "event");
    c->sync();
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, t0, t1), "elapsed");
    if (stats) stats->step_ms = ms;
  }
  if (stats) {
    stats->loop_ms = loop_ms;
    stats->loop_launches = launches;
  }
  finish_stats(*c, sel, before, cur, stats);
  if (stats) stats->room_stops = room_stops;
}

int pic_step(pic_ctx c, const pic_step_args* a, pic_step_stats* stats) {
  PIC_GUARD_BEGIN
  step_impl(c, a, stats, false);
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_step_noalloc(pic_ctx c, const pic_step_args* a, pic_step_stats* stats) {
  PIC_GUARD_BEGIN
  if (!c) throw Err(PIC_E_ARG, "null context");
  struct Hold {   // no block goes back to the device or the caller's allocator during the call
    Ctx& C;
    explicit Hold(Ctx& x) : C(x) { C.hold_pool = true; }
    ~Hold() { C.hold_pool = false; }
  } hold(*c);
  step_impl(c, a, stats, true);
  return PIC_OK;
  PIC_GUARD_END(c)
}

int64_t pic_step_index(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  Slot& sl = get_slot(c, slot);
  return (int64_t)read_counters(*c, sl).step;
  PIC_GUARD_END(c)
}

int pic_set_slot_limit(pic_ctx c, int slot, int64_t max_bytes) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (max_bytes < 0) throw Err(PIC_E_ARG, "the limit must be >= 0");
  sl.byte_limit = (size_t)max_bytes;
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_sort(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  sort_slot(*c, sl);
  c->sync();
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_locate(pic_ctx c, int slot, int64_t n, const double* s, uint32_t* leaf) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  const int dim = sl.d.dim;
  if (dim < 2) throw Err(PIC_E_ARG, "not a tree slot");
  for (int64_t i = 0; i < dim * n; ++i)
    if (!(s[i] >= 0.0 && s[i] < 1.0)) throw Err(PIC_E_ARG, "point outside [0,1)");
  double* ds = nullptr;
  uint32_t* dl = nullptr;
  hip_check(hipMalloc(&ds, 8 * dim * (size_t)std::max<int64_t>(n, 1)), "hipMalloc");
  hip_check(hipMalloc(&dl, 4 * (size_t)std::max<int64_t>(n, 1)), "hipMalloc");
  hip_check(hipMemcpy(ds, s, 8 * dim * (size_t)n, hipMemcpyHostToDevice), "upload");
  if (dim == 3)
    hipLaunchKernelGGL(k_locate_points3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, sl.key, sl.lv,
                       sl.lut, sl.lut_level, ds, n, dl);
  else
    hipLaunchKernelGGL(k_locate_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, sl.key, sl.lv,
                       sl.lut, sl.lut_level, ds, n, dl);
  hip_check(hipGetLastError(), "locate");
  c->sync();
  hip_check(hipMemcpy(leaf, dl, 4 * (size_t)n, hipMemcpyDeviceToHost), "read");
  (void)hipFree(ds);
  (void)hipFree(dl);
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_gather(pic_ctx c, int slot, int64_t n, const double* s, double* out) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  const int dim = sl.d.dim;
  if (n < 0 || (n > 0 && (!s || !out))) throw Err(PIC_E_ARG, "bad arguments");
  for (int64_t i = 0; i < n * dim; ++i)
    if (!in_unit(s[i], sl.prec)) throw Err(PIC_E_ARG, "point outside [0,1) in the particle precision");
  if (n == 0) return PIC_OK;
  double* ds = (double*)sl.alloc(8 * (size_t)(n * dim));
  double* dout = (double*)sl.alloc(8 * (size_t)(n * dim));
  hip_check(hipMemcpy(ds, s, 8 * (size_t)(n * dim), hipMemcpyHostToDevice), "upload");
  if (sl.prec == 32) hip_check(launch_gather_points<float>(make_dev<float>(sl), ds, n, dout, c->stream), "gather");
  else hip_check(launch_gather_points<double>(make_dev<double>(sl), ds, n, dout, c->stream), "gather");
  c->sync();
  hip_check(hipMemcpy(out, dout, 8 * (size_t)(n * dim), hipMemcpyDeviceToHost), "read");
  sl.release(ds);
  sl.release(dout);
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_derived(pic_ctx c, int slot, int species, double* out) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (species < 0 || species > 1) throw Err(PIC_E_ARG, "bad species");
  if (sl.prec == 32) {
    SpeciesK<float> k = to_dev<float>(sl.hk[species]);
    double v[] = {k.qm_dt, k.dt_L, (double)k.tcand, k.a_el, k.a_iz, k.v_iz2, k.mu2, k.vmax2, k.v_thg, k.a_cx, k.gmax, k.hqm_dt};
    std::memcpy(out, v, sizeof(v));
  } else {
    SpeciesK<double> k = to_dev<double>(sl.hk[species]);
    double v[] = {k.qm_dt, k.dt_L, (double)k.tcand, k.a_el, k.a_iz, k.v_iz2, k.mu2, k.vmax2, k.v_thg, k.a_cx, k.gmax, k.hqm_dt};
    std::memcpy(out, v, sizeof(v));
  }
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_philox(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out) {
  pic_ctx c = nullptr;
  PIC_GUARD_BEGIN
  if (n < 0 || !ctr || !key || !out) throw Err(PIC_E_ARG, "bad arguments");
  uint32_t *dc = nullptr, *dout = nullptr;
  hip_check(hipMalloc(&dc, 16 * (size_t)std::max<int64_t>(n, 1)), "hipMalloc");
  hip_check(hipMalloc(&dout, 16 * (size_t)std::max<int64_t>(n, 1)), "hipMalloc");
  hip_check(hipMemcpy(dc, ctr, 16 * (size_t)n, hipMemcpyHostToDevice), "upload");
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, dc, key[0], key[1], dout, n);
  hip_check(hipGetLastError(), "philox");
  hip_check(hipDeviceSynchronize(), "sync");
  hip_check(hipMemcpy(out, dout, 16 * (size_t)n, hipMemcpyDeviceToHost), "read");
  (void)hipFree(dc);
  (void)hipFree(dout);
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_admit(pic_ctx c, const pic_instance_desc* d, int* slot) {
  PIC_GUARD_BEGIN
  if (!c || !d || !slot) throw Err(PIC_E_ARG, "bad arguments");
  int s = -1;
  for (size_t i = 0; i < c->slots.size(); ++i)
    if (!c->slots[i].live) {
      s = (int)i;
      break;
    }
  if (s < 0) {
    c->slots.emplace_back();
    s = (int)c->slots.size() - 1;
  }
  try {
    build_slot(*c, c->slots[s], *d);
    upload_dev(*c, c->slots[s]);
    c->sync();
  } catch (...) {
    c->slots[s].release_all();
    c->slots[s].live = false;
    throw;
  }
  *slot = s;
  return PIC_OK;
  PIC_GUARD_END(c)
}

int pic_retire(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  Slot& sl = get_slot(c, slot);
  c->sync();
  sl.release_all();
  sl = Slot();
  return PIC_OK;
  PIC_GUARD_END(c)
}

int64_t pic_slot_bytes(pic_ctx c, int slot) {
  PIC_GUARD_BEGIN
  return (int64_t)get_slot(c, slot).bytes_held;
  PIC_GUARD_END(c)
}

int pic_adapt(pic_ctx c, int slot, const pic_adapt_args* a, pic_adapt_stats* s) {
  PIC_GUARD_BEGIN
  Slot& sl = usable_slot(c, slot);
  if (!a) throw Err(PIC_E_ARG, "null adapt arguments");
  adapt_slot(*c, sl, a->n_lo, a->n_hi, s);
  return PIC_OK;
  PIC_GUARD_END(c)
}

}  // extern "C"
