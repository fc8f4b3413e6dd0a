// Host side of the C ABI declared in include/pic.h: instance state on the
// device, derived constants, quadtree construction, and the launch sequences
// of the ES-PIC step (arXiv:1604.07713, Sec. 3, 3.1, 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "k_mesh.hpp"
#include "k_adapt.hpp"
#include "pic_internal.hpp"
#include "api_internal.hpp"

using namespace pic;

namespace pic {

const double kQE = 1.602176634e-19;
const double kEPS0 = 8.8541878128e-12;
const double kKB = 1.380649e-23;

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Err(PIC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t DevPool::class_of(size_t bytes) {
  if (bytes <= 4096) return 4096;
  int top = 63 - __builtin_clzll((unsigned long long)bytes);
  const size_t q = size_t(1) << (top - 2);   // four classes per power of two
  return (bytes + q - 1) / q * q;
}

void* DevPool::get(size_t cls) {
  if (has_ext) {
    void* p = ext.alloc(cls, (void*)stream, ext.user);
    if (!p) throw Err(PIC_E_NOMEM, "the caller's allocator refused " + std::to_string(cls) + " bytes");
    return p;
  }
  auto it = free_.find(cls);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    free_bytes -= cls;
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess || !p) {
    (void)hipGetLastError();
    // give the cached blocks back and try once more
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    free_bytes = 0;
    if (hipMalloc(&p, cls) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Err(PIC_E_NOMEM, "device allocation of " + std::to_string(cls) + " bytes failed");
    }
  }
  return p;
}

void DevPool::put(void* p, size_t cls) { pending_.emplace_back(cls, p); }

void DevPool::synced(size_t held) {
  if (has_ext) {
    for (auto& e : pending_) ext.free(e.second, ext.user);
    pending_.clear();
    return;
  }
  const size_t limit = std::min(kMaxFree, std::max(kMinFree, held / 4));
  for (auto& e : pending_) {
    if (free_bytes + e.first > limit) {
      (void)hipFree(e.second);
    } else {
      free_.emplace(e.first, e.second);
      free_bytes += e.first;
    }
  }
  pending_.clear();
  // the limit may have dropped (slots retired): free the largest blocks first
  while (free_bytes > limit && !free_.empty()) {
    auto it = std::prev(free_.end());
    (void)hipFree(it->second);
    free_bytes -= it->first;
    free_.erase(it);
  }
}

void DevPool::clear() {
  if (has_ext) {
    for (auto& e : pending_) ext.free(e.second, ext.user);
    pending_.clear();
    return;
  }
  for (auto& e : pending_) (void)hipFree(e.second);
  pending_.clear();
  for (auto& kv : free_) (void)hipFree(kv.second);
  free_.clear();
  free_bytes = 0;
}

void Ctx::release_tables() {
  void** tab[] = {&b_insts, &b_items, (void**)&b_part, (void**)&b_rowbeg, &b_jobs, &b_blob};
  size_t* have[] = {&b_insts_bytes, &b_items_bytes, &b_part_bytes, &b_rowbeg_bytes, &b_jobs_bytes, &b_blob_bytes};
  for (int i = 0; i < 6; ++i) {
    if (*tab[i]) pool.put(*tab[i], *have[i]);
    *tab[i] = nullptr;
    *have[i] = 0;
  }
}

void* Slot::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  const size_t cls = DevPool::class_of(bytes);
  void* p = nullptr;
  size_t held = bytes;
  const bool from_pool = pool && pool->pooled(cls);
  if (from_pool) {
    p = pool->get(cls);
    held = cls;
  } else if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Err(PIC_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  allocs.push_back(p);
  alloc_bytes.push_back(held);
  alloc_pooled.push_back(from_pool ? 1 : 0);
  bytes_held += held;
  return p;
}

static void give_back(DevPool* pool, void* p, size_t held, bool from_pool) {
  if (from_pool && pool) pool->put(p, held);
  else (void)hipFree(p);
}

void Slot::release(void* p) {
  if (!p) return;
  for (size_t i = 0; i < allocs.size(); ++i)
    if (allocs[i] == p) {
      give_back(pool, p, alloc_bytes[i], alloc_pooled[i] != 0);
      bytes_held -= alloc_bytes[i];
      allocs.erase(allocs.begin() + i);
      alloc_bytes.erase(alloc_bytes.begin() + i);
      alloc_pooled.erase(alloc_pooled.begin() + i);
      return;
    }
}

void Slot::release_all() {
  for (size_t i = 0; i < allocs.size(); ++i) give_back(pool, allocs[i], alloc_bytes[i], alloc_pooled[i] != 0);
  allocs.clear();
  alloc_bytes.clear();
  alloc_pooled.clear();
  bytes_held = 0;
}

// ---------------------------------------------------------------------------
// derived per-species constants (FP64 on the host, rounded to the precision)
// ---------------------------------------------------------------------------
void derive(Slot& sl) {
  const pic_instance_desc& d = sl.d;
  for (int s = 0; s < 2; ++s) {
    HostK& k = sl.hk[s];
    k = HostK();
    if (s >= d.nspecies) continue;
    const pic_species_desc& sp = d.species[s];
    k.qm_dt = (sp.charge * d.dt) / sp.mass;
    k.dt_L = d.dt / d.length;
    k.v_thg = std::sqrt((kKB * d.gas_temperature) / d.gas_mass);
    k.mcc = sp.mcc;
    if (sp.mcc == PIC_MCC_ELECTRON) {
      const double vmax = std::sqrt(((2.0 * kQE) * sp.eps_max) / sp.mass);
      const double sig_t = sp.sigma_el + sp.sigma_iz;
      const double nu_max = (d.gas_density * sig_t) * vmax;
      const double pnull = -std::expm1(-(nu_max * d.dt));
      k.tcand = (uint32_t)std::floor(std::ldexp(pnull, 24));
      k.a_el = sp.sigma_el / (sig_t * vmax);
      k.a_iz = sp.sigma_iz / (sig_t * vmax);
      k.v_iz2 = ((2.0 * kQE) * sp.eps_iz) / sp.mass;
      k.vmax2 = vmax * vmax;
      k.mu2 = (2.0 * sp.mass) / d.gas_mass;
    } else if (sp.mcc == PIC_MCC_ION_CX) {
      const double g = std::sqrt(((2.0 * kQE) * sp.eps_max) / sp.mass) + 11.0 * k.v_thg;
      const double nu_max = (d.gas_density * sp.sigma_cx) * g;
      const double pnull = -std::expm1(-(nu_max * d.dt));
      k.tcand = (uint32_t)std::floor(std::ldexp(pnull, 24));
      k.gmax = g;
      k.a_cx = 1.0 / g;
    }
    const int F = sl.prec == 32 ? 24 : 32;
    if (d.dim == 1) {
      const double dx = d.length / d.ncells;
      sl.kappa[s] = (((sp.charge * sp.w0) * std::ldexp(1.0, -(16 + F))) * dx) / kEPS0;
      // direct implicit: (q/m)(dt^2/2) rho_s / eps0 per unit charge sum (rho over a cell)
      sl.chi[s] = (((sp.charge / sp.mass) * ((d.dt * d.dt) * 0.5)) * (((sp.charge * sp.w0) * std::ldexp(1.0, -(16 + F))) / dx)) /
                  kEPS0;
    } else {
      const int f2 = d.field_scheme == PIC_FIELD_CIC_AMR ? F : 0;   // cloud shares carry F more bits
      sl.kappa[s] = (((sp.charge * sp.w0) * std::ldexp(1.0, -(16 + f2))) / d.depth_z) / kEPS0;
    }
  }
  if (d.dim == 1) sl.inv2dx = 1.0 / (2.0 * (d.length / d.ncells));
}

template <class T>
SpeciesK<T> to_dev(const HostK& h) {
  SpeciesK<T> k;
  k.qm_dt = (T)h.qm_dt;
  k.hqm_dt = (T)0.5 * k.qm_dt;
  k.dt_L = (T)h.dt_L;
  k.a_el = (T)h.a_el;
  k.a_iz = (T)h.a_iz;
  k.v_iz2 = (T)h.v_iz2;
  k.mu2 = (T)h.mu2;
  k.vmax2 = (T)h.vmax2;
  k.v_thg = (T)h.v_thg;
  k.a_cx = (T)h.a_cx;
  k.gmax = (T)h.gmax;
  k.tcand = h.tcand;
  k.mcc = h.mcc;
  return k;
}

// ---------------------------------------------------------------------------
// host linear quadtree for mesh construction
// ---------------------------------------------------------------------------
uint32_t morton_host(uint32_t x, uint32_t y) {
  uint32_t k = 0;
  for (int b = 0; b < 16; ++b) {
    k |= ((x >> b) & 1u) << (2 * b);
    k |= ((y >> b) & 1u) << (2 * b + 1);
  }
  return k;
}
void unmorton_host(uint32_t k, uint32_t& x, uint32_t& y) {
  x = y = 0;
  for (int b = 0; b < 16; ++b) {
    x |= ((k >> (2 * b)) & 1u) << b;
    y |= ((k >> (2 * b + 1)) & 1u) << b;
  }
}

size_t host_locate(const std::vector<HostLeaf>& L, uint32_t X, uint32_t Y) {
  const uint32_t m = morton_host(X, Y);
  size_t lo = 0, hi = L.size() - 1;
  while (lo < hi) {
    const size_t mid = (lo + hi + 1) / 2;
    if (L[mid].key <= m) lo = mid; else hi = mid - 1;
  }
  return lo;
}

std::vector<HostLeaf> host_refine(const std::vector<HostLeaf>& L, const std::vector<char>& mark) {
  std::vector<HostLeaf> out;
  out.reserve(L.size() + 3 * std::count(mark.begin(), mark.end(), 1));
  for (size_t i = 0; i < L.size(); ++i) {
    if (!mark[i]) {
      out.push_back(L[i]);
      continue;
    }
    uint32_t X, Y;
    unmorton_host(L[i].key, X, Y);
    const uint32_t half = 1u << (16 - L[i].lv - 1);
    for (int c = 0; c < 4; ++c)
      out.push_back(HostLeaf{morton_host(X + (c & 1) * half, Y + (c >> 1) * half), (uint8_t)(L[i].lv + 1)});
  }
  return out;
}

// Leaves that a finer leaf two or more levels deeper touches (face or
// corner).  Probes one unit outside each leaf's side midpoints and corners
// find every coarser leaf that touches it.
bool host_unbalanced(const std::vector<HostLeaf>& L, std::vector<char>& mark, int64_t* nmark) {
  bool any = false;
  for (size_t i = 0; i < L.size(); ++i) {
    uint32_t X, Y;
    unmorton_host(L[i].key, X, Y);
    const uint32_t S = 1u << (16 - L[i].lv);
    const int64_t px[8] = {(int64_t)X - 1, (int64_t)X + S, (int64_t)X + S / 2, (int64_t)X + S / 2,
                           (int64_t)X - 1, (int64_t)X + S, (int64_t)X - 1, (int64_t)X + S};
    const int64_t py[8] = {(int64_t)Y + S / 2, (int64_t)Y + S / 2, (int64_t)Y - 1, (int64_t)Y + S,
                           (int64_t)Y - 1, (int64_t)Y - 1, (int64_t)Y + S, (int64_t)Y + S};
    for (int k = 0; k < 8; ++k) {
      if (px[k] < 0 || py[k] < 0 || px[k] >= 65536 || py[k] >= 65536) continue;
      const size_t j = host_locate(L, (uint32_t)px[k], (uint32_t)py[k]);
      if ((int)L[j].lv < (int)L[i].lv - 1) {
        if (!mark[j] && nmark) ++*nmark;
        mark[j] = 1;
        any = true;
      }
    }
  }
  return any;
}

// 2:1 balance over faces and corners: refine a leaf while a leaf touching it
// is two or more levels finer.
int64_t host_balance(std::vector<HostLeaf>& L) {
  int64_t nref = 0;
  for (;;) {
    std::vector<char> mark(L.size(), 0);
    if (!host_unbalanced(L, mark, &nref)) return nref;
    L = host_refine(L, mark);
  }
}

// A tree given leaf by leaf (Morton order): every leaf an aligned Morton
// range of 4^(16 - level) keys, the ranges following each other from 0 to
// 2^32 without gap or overlap, levels within bounds, 2:1 balanced across
// faces and corners.  Anything else is refused (PIC_E_ARG), not repaired.
std::vector<HostLeaf> host_explicit_tree(const pic_instance_desc& d) {
  if (!d.leaf_keys || !d.leaf_levels || d.nleaves > (int64_t)1 << 28)
    throw Err(PIC_E_ARG, "explicit tree needs leaf_keys and leaf_levels (at most 2^28 leaves)");
  std::vector<HostLeaf> L((size_t)d.nleaves);
  uint64_t pos = 0;
  for (int64_t i = 0; i < d.nleaves; ++i) {
    const int lv = d.leaf_levels[i];
    if (lv < d.min_level || lv > d.max_level) throw Err(PIC_E_ARG, "explicit tree: leaf level outside [min, max]");
    if ((uint64_t)d.leaf_keys[i] != pos)
      throw Err(PIC_E_ARG, "explicit tree: leaves must tile the square in Morton order (gap, overlap or misaligned key)");
    pos += (uint64_t)1 << (2 * (16 - lv));
    L[i] = HostLeaf{d.leaf_keys[i], (uint8_t)lv};
  }
  if (pos != ((uint64_t)1 << 32)) throw Err(PIC_E_ARG, "explicit tree: leaves do not cover the square");
  std::vector<char> mark(L.size(), 0);
  if (host_unbalanced(L, mark, nullptr)) throw Err(PIC_E_ARG, "explicit tree: not 2:1 balanced across faces and corners");
  return L;
}

std::vector<HostLeaf> host_build_tree(const pic_instance_desc& d) {
  if (d.nleaves > 0) return host_explicit_tree(d);
  std::vector<HostLeaf> L;
  const int B = d.base_level;
  const uint32_t n = 1u << B;
  for (uint32_t iy = 0; iy < n; ++iy)
    for (uint32_t ix = 0; ix < n; ++ix)
      L.push_back(HostLeaf{morton_host(ix << (16 - B), iy << (16 - B)), (uint8_t)B});
  std::sort(L.begin(), L.end(), [](const HostLeaf& a, const HostLeaf& b) { return a.key < b.key; });
  if (d.refine_disk) {
    for (;;) {
      std::vector<char> mark(L.size(), 0);
      bool any = false;
      for (size_t i = 0; i < L.size(); ++i) {
        if (L[i].lv >= d.disk_level || L[i].lv >= d.max_level) continue;
        uint32_t X, Y;
        unmorton_host(L[i].key, X, Y);
        const double h = std::ldexp(1.0, -(int)L[i].lv);
        const double x0 = X / 65536.0, y0 = Y / 65536.0, x1 = x0 + h, y1 = y0 + h;
        const double dx = std::max(std::max(x0 - d.disk_cx, 0.0), d.disk_cx - x1);
        const double dy = std::max(std::max(y0 - d.disk_cy, 0.0), d.disk_cy - y1);
        if (dx * dx + dy * dy <= d.disk_r * d.disk_r) {
          mark[i] = 1;
          any = true;
        }
      }
      if (!any) break;
      L = host_refine(L, mark);
    }
  }
  host_balance(L);
  return L;
}

// ---------------------------------------------------------------------------
// pinned staging arena for small host->device uploads
// ---------------------------------------------------------------------------
void* Ctx::stage(const void* src, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes > arena_size) throw Err(PIC_E_ARG, "staging upload too large");
  if (arena_off + bytes > arena_size) {
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    arena_off = 0;
  }
  char* p = (char*)arena + arena_off;
  arena_off += bytes;
  std::memcpy(p, src, bytes);
  return p;
}

void* Ctx::pinned(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes > arena_size) throw Err(PIC_E_ARG, "pinned scratch too large");
  if (arena_off + bytes > arena_size) {
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    arena_off = 0;
  }
  char* p = (char*)arena + arena_off;
  arena_off += bytes;
  return p;
}

__global__ void k_copy_blobs(const Blob* b) {
  const Blob x = b[blockIdx.x];
  const uint32_t* s = (const uint32_t*)x.src;
  uint32_t* d = (uint32_t*)x.dst;
  for (uint32_t i = threadIdx.x; i < x.bytes / 4u; i += blockDim.x) d[i] = s[i];
}

// Device buffer of a gathered batch.  A replaced buffer goes back to the
// pool, which reuses it only after the next synchronization.
void* Ctx::blob_buffer(size_t bytes) {
  if (b_blob_bytes < bytes) {
    if (b_blob) pool.put(b_blob, b_blob_bytes);
    b_blob = nullptr;
    b_blob_bytes = 0;
    const size_t cls = DevPool::class_of(bytes);
    b_blob = pool.get(cls);
    b_blob_bytes = cls;
  }
  return b_blob;
}

void Ctx::upload(void* dst, const void* src, size_t bytes) {
  if (!defer_uploads) {
    hip_check(hipMemcpyAsync(dst, stage(src, bytes), bytes, hipMemcpyHostToDevice, stream), "upload");
    return;
  }
  if (bytes % 4) throw Err(PIC_E_ARG, "gathered uploads take whole 32-bit words");
  pend.push_back(Blob{dst, (const void*)(uintptr_t)pend_data.size(), (uint32_t)bytes, 0u});
  pend_data.insert(pend_data.end(), (const char*)src, (const char*)src + bytes);
  pend_data.resize((pend_data.size() + 15) & ~(size_t)15);
}

void Ctx::flush_uploads() {
  if (pend.empty()) return;
  const size_t n = pend.size();
  const size_t tab = (n * sizeof(Blob) + 255) & ~(size_t)255;
  const size_t total = tab + pend_data.size();
  char* D = (char*)blob_buffer(total);
  std::vector<char> host(total);
  for (size_t j = 0; j < n; ++j) {
    Blob b = pend[j];
    b.src = D + tab + (size_t)(uintptr_t)b.src;
    std::memcpy(host.data() + j * sizeof(Blob), &b, sizeof(Blob));
  }
  std::memcpy(host.data() + tab, pend_data.data(), pend_data.size());
  pend.clear();
  pend_data.clear();
  hip_check(hipMemcpyAsync(D, stage(host.data(), total), total, hipMemcpyHostToDevice, stream), "gathered upload");
  hipLaunchKernelGGL(k_copy_blobs, dim3((unsigned)n), dim3(64), 0, stream, (const Blob*)D);
  hip_check(hipGetLastError(), "copy blobs");
}

// Counters of many slots: one table upload, one gather kernel and one
// download (or per-slot downloads for a few slots and in no-allocation
// steps, which take no device buffer).
std::vector<Counters> read_counters_many(Ctx& C, const std::vector<Slot*>& sel) {
  C.flush_uploads();
  const size_t n = sel.size();
  std::vector<Counters> out(n);
  Counters* h = (Counters*)C.pinned(sizeof(Counters) * n);
  if (n >= 4 && !C.hold_pool) {
    const size_t tab = (n * sizeof(Blob) + 255) & ~(size_t)255;
    char* D = (char*)C.blob_buffer(tab + sizeof(Counters) * n);
    std::vector<Blob> t(n);
    for (size_t j = 0; j < n; ++j)
      t[j] = Blob{D + tab + j * sizeof(Counters), sel[j]->ctr, (uint32_t)sizeof(Counters), 0u};
    hip_check(hipMemcpyAsync(D, C.stage(t.data(), n * sizeof(Blob)), n * sizeof(Blob), hipMemcpyHostToDevice,
                             C.stream),
              "counters table");
    hipLaunchKernelGGL(k_copy_blobs, dim3((unsigned)n), dim3(64), 0, C.stream, (const Blob*)D);
    hip_check(hipGetLastError(), "gather counters");
    hip_check(hipMemcpyAsync(h, D + tab, sizeof(Counters) * n, hipMemcpyDeviceToHost, C.stream), "read counters");
  } else {
    for (size_t j = 0; j < n; ++j)
      hip_check(hipMemcpyAsync(h + j, sel[j]->ctr, sizeof(Counters), hipMemcpyDeviceToHost, C.stream),
                "read counters");
  }
  hip_check(hipStreamSynchronize(C.stream), "hipStreamSynchronize");
  std::memcpy(out.data(), h, sizeof(Counters) * n);
  C.sync();
  return out;
}

void Ctx::sync() {
  flush_uploads();
  hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  arena_off = 0;
  if (hold_pool) return;
  size_t held = 0;
  for (const Slot& s : slots) held += s.bytes_held;
  pool.synced(held);
}

// ---------------------------------------------------------------------------
// slot construction
// ---------------------------------------------------------------------------
void validate(const pic_instance_desc& d) {
  if (d.dim < 1 || d.dim > 3) throw Err(PIC_E_ARG, "dim must be 1, 2 or 3");
  if (d.precision != PIC_FP32 && d.precision != PIC_FP64) throw Err(PIC_E_ARG, "precision must be 32 or 64");
  if (!(d.length > 0) || !(d.dt > 0)) throw Err(PIC_E_ARG, "length and dt must be positive");
  if (d.nspecies < 1 || d.nspecies > 2) throw Err(PIC_E_ARG, "nspecies must be 1 or 2");
  if (d.dim == 1 && (d.ncells < 2 || d.ncells > 8192)) throw Err(PIC_E_ARG, "1D ncells must be in [2, 8192]");
  if (d.dim == 2 && (d.min_level < 0 || d.max_level > 14 || d.min_level > d.max_level || d.base_level < d.min_level ||
                     d.base_level > d.max_level))
    throw Err(PIC_E_ARG, "2D levels must satisfy 0 <= min <= base <= max <= 14");
  if (d.field_scheme != PIC_FIELD_CIC_EM && d.field_scheme != PIC_FIELD_CIC_EC &&
      d.field_scheme != PIC_FIELD_CIC_AMR && d.field_scheme != PIC_FIELD_DIPIC)
    throw Err(PIC_E_ARG, "unknown field_scheme");
  if (d.dim >= 2 && d.field_scheme == PIC_FIELD_CIC_EC)
    throw Err(PIC_E_ARG, "the energy-conserving coupling is for the uniform 1D mesh");
  if (d.dim == 3 && (d.min_level < 0 || d.max_level > 10 || d.min_level > d.max_level ||
                     d.base_level < d.min_level || d.base_level > d.max_level))
    throw Err(PIC_E_ARG, "3D levels must satisfy 0 <= min <= base <= max <= 10");
  if (d.dim == 3 && d.field_scheme != PIC_FIELD_CIC_EM)
    throw Err(PIC_E_ARG, "the octree takes the nodal-E gather with NGP deposit");
  if (d.dim == 1 && d.field_scheme == PIC_FIELD_CIC_AMR)
    throw Err(PIC_E_ARG, "the cloud-in-cell on the tree is for 2D slots");
  if (d.dim != 1 && d.field_scheme == PIC_FIELD_DIPIC)
    throw Err(PIC_E_ARG, "the direct implicit step is for the uniform 1D mesh");
  if (d.nleaves < 0 || (d.nleaves > 0 && d.dim != 2)) throw Err(PIC_E_ARG, "an explicit tree is for quadtree slots");
  for (int s = 0; s < d.nspecies; ++s) {
    const pic_species_desc& sp = d.species[s];
    if (!(sp.mass > 0)) throw Err(PIC_E_ARG, "species mass must be positive");
    if (sp.mcc == PIC_MCC_ELECTRON && d.nspecies < 2) throw Err(PIC_E_ARG, "ionization needs an ion species");
    if (sp.mcc != PIC_MCC_NONE && !(d.gas_mass > 0 && d.gas_temperature > 0))
      throw Err(PIC_E_ARG, "collisions need gas mass and temperature");
    if (sp.mcc == PIC_MCC_ELECTRON && s != 0) throw Err(PIC_E_ARG, "electron collisions apply to species 0");
  }
}

// Adopt device leaf arrays (allocated through sl.alloc) as the slot's tree and
// size every per-leaf array for it.
void set_mesh2d_device(Ctx& C, Slot& sl, uint32_t* key, uint8_t* lv, uint32_t n, int maxlv) {
  // the old tree and cell potential stay until the potential is carried over
  uint32_t* okey = sl.key;
  uint8_t* olv = sl.lv;
  uint32_t* olut = sl.lut;
  double* ophi = sl.phi64;
  const int olut_level = sl.lut_level;
  const bool carry = okey && olv && olut && ophi && sl.nleaves > 0;
  // (a failed allocation below leaves released tables null; its caller marks
  // the slot failed)
  sl.release(sl.xy);
  sl.xy = nullptr;
  sl.key = key;
  sl.lv = lv;
  sl.nleaves = n;
  sl.xy = (uint32_t*)sl.alloc(4 * (size_t)n);
  // point-location table at the finest level up to 11 (4^11 + 1 entries,
  // 16 MiB): below it every lookup is one load; deeper trees finish with a
  // binary search inside the table cell
  sl.lut_level = std::min(sl.d.max_level, kLutMaxLevel);
  sl.lut_direct = maxlv <= sl.lut_level;
  sl.lut = nullptr;
  sl.lut = (uint32_t*)sl.alloc(4 * ((size_t(1) << (2 * sl.lut_level)) + 1));
  hip_check(launch_leaf_xy(sl.key, sl.lv, sl.nleaves, sl.xy, C.stream), "leaf_xy");
  hip_check(launch_build_lut(sl.key, sl.lv, sl.nleaves, sl.lut, sl.lut_level, C.stream), "build_lut");
  // per-leaf field and deposit arrays
  for (void* p : {(void*)sl.E, (void*)sl.e64, (void*)sl.cphi, (void*)sl.grad, (void*)sl.Q, (void*)sl.off,
                  (void*)sl.st.nbr, (void*)sl.st.code, (void*)sl.st.diag, (void*)sl.st.bnd, (void*)sl.cg_ws,
                  sl.cellE})
    sl.release(p);
  sl.E = nullptr;
  sl.e64 = sl.cphi = sl.grad = nullptr;
  sl.Q = nullptr;
  sl.off = sl.scan_tmp = nullptr;
  sl.cellE = nullptr;
  sl.st = Stencil2D{nullptr, nullptr, nullptr, nullptr};
  sl.cg_ws = nullptr;
  sl.stencil_ok = false;
  sl.nq = sl.nleaves;
  sl.E = sl.alloc(sl.esz * 8 * sl.nleaves);
  sl.e64 = (double*)sl.alloc(8 * 8 * (size_t)sl.nleaves);
  sl.cphi = (double*)sl.alloc(8 * 4 * (size_t)sl.nleaves);
  sl.grad = (double*)sl.alloc(8 * 8 * (size_t)sl.nleaves);
  sl.phi64 = nullptr;   // the old cell potential is held in ophi until it is carried over
  sl.phi64 = (double*)sl.alloc(8 * (size_t)sl.nleaves);
  sl.Q = (unsigned long long*)sl.alloc(8 * 4 * (size_t)sl.nq);
  // one offset array per species (the batched sort takes both at once),
  // then the scratch of the multi-block scan of the per-species sort
  sl.off = (uint32_t*)sl.alloc(4 * (2 * ((size_t)sl.nq + 1) + scan_tmp_words((uint32_t)sl.nq)));
  sl.scan_tmp = sl.off + 2 * ((size_t)sl.nq + 1);
  hip_check(hipMemsetAsync(sl.E, 0, sl.esz * 8 * sl.nleaves, C.stream), "memset");
  if (sl.d.field_scheme == PIC_FIELD_CIC_AMR) {   // the cloud's cell-centred E table
    sl.cellE = sl.alloc(sl.esz * 2 * sl.nleaves);
    hip_check(hipMemsetAsync(sl.cellE, 0, sl.esz * 2 * sl.nleaves, C.stream), "memset");
  }
  hip_check(hipMemsetAsync(sl.e64, 0, 64 * (size_t)sl.nleaves, C.stream), "memset");
  hip_check(hipMemsetAsync(sl.Q, 0, 32 * (size_t)sl.nq, C.stream), "memset");
  // the next 2D solve starts from the potential of the old tree
  if (carry)
    hip_check(launch_remap_cells(sl.xy, sl.lv, sl.nleaves, okey, olv, olut, olut_level, ophi, sl.phi64, C.stream),
              "remap");
  else
    hip_check(hipMemsetAsync(sl.phi64, 0, 8 * (size_t)sl.nleaves, C.stream), "memset");
  if (okey != key) sl.release(okey);
  if (olv != lv) sl.release(olv);
  sl.release(olut);
  sl.release(ophi);
}

// ---------------------------------------------------------------------------
// octree (3D): host construction in Morton order of 10-bit coordinates
// ---------------------------------------------------------------------------
uint32_t morton3_host(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t k = 0;
  for (int b = 0; b < 10; ++b) {
    k |= ((x >> b) & 1u) << (3 * b);
    k |= ((y >> b) & 1u) << (3 * b + 1);
    k |= ((z >> b) & 1u) << (3 * b + 2);
  }
  return k;
}
void unmorton3_host(uint32_t k, uint32_t X[3]) {
  X[0] = X[1] = X[2] = 0;
  for (int b = 0; b < 10; ++b)
    for (int a = 0; a < 3; ++a) X[a] |= ((k >> (3 * b + a)) & 1u) << b;
}
static size_t host_locate3(const std::vector<HostLeaf>& L, uint32_t X, uint32_t Y, uint32_t Z) {
  const uint32_t m = morton3_host(X, Y, Z);
  size_t lo = 0, hi = L.size() - 1;
  while (lo < hi) {
    const size_t mid = (lo + hi + 1) / 2;
    if (L[mid].key <= m) lo = mid; else hi = mid - 1;
  }
  return lo;
}
static std::vector<HostLeaf> host_refine3(const std::vector<HostLeaf>& L, const std::vector<char>& mark) {
  std::vector<HostLeaf> out;
  out.reserve(L.size() + 7 * std::count(mark.begin(), mark.end(), 1));
  for (size_t i = 0; i < L.size(); ++i) {
    if (!mark[i]) {
      out.push_back(L[i]);
      continue;
    }
    uint32_t X[3];
    unmorton3_host(L[i].key, X);
    const uint32_t half = 1u << (10 - L[i].lv - 1);
    for (int c = 0; c < 8; ++c)
      out.push_back(HostLeaf{morton3_host(X[0] + (c & 1) * half, X[1] + ((c >> 1) & 1) * half,
                                          X[2] + (c >> 2) * half),
                             (uint8_t)(L[i].lv + 1)});
  }
  return out;
}
// 2:1 over faces, edges and corners: probes one unit outside the 6 face
// centres, 12 edge midpoints and 8 corners of every leaf find each coarser
// leaf touching it; one two or more levels coarser is refined.
static int64_t host_balance3(std::vector<HostLeaf>& L) {
  int64_t nref = 0;
  for (;;) {
    std::vector<char> mark(L.size(), 0);
    bool any = false;
    for (size_t i = 0; i < L.size(); ++i) {
      uint32_t X[3];
      unmorton3_host(L[i].key, X);
      const int64_t S = (int64_t)1 << (10 - L[i].lv);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            const int dd[3] = {dx, dy, dz};
            int64_t P[3];
            bool in = true;
            for (int a = 0; a < 3; ++a) {
              P[a] = dd[a] < 0 ? (int64_t)X[a] - 1 : dd[a] > 0 ? (int64_t)X[a] + S : (int64_t)X[a] + S / 2;
              if (P[a] < 0 || P[a] >= 1024) in = false;
            }
            if (!in) continue;
            const size_t j = host_locate3(L, (uint32_t)P[0], (uint32_t)P[1], (uint32_t)P[2]);
            if ((int)L[j].lv < (int)L[i].lv - 1) {
              if (!mark[j]) ++nref;
              mark[j] = 1;
              any = true;
            }
          }
    }
    if (!any) return nref;
    L = host_refine3(L, mark);
  }
}
// base level everywhere, every leaf whose closed box meets the closed ball
// refined until disk_level, then 2:1 balance (Sec. 3.1 octree)
std::vector<HostLeaf> host_build_tree3(const pic_instance_desc& d) {
  std::vector<HostLeaf> L;
  const int B = d.base_level;
  const uint32_t n = 1u << B;
  for (uint32_t iz = 0; iz < n; ++iz)
    for (uint32_t iy = 0; iy < n; ++iy)
      for (uint32_t ix = 0; ix < n; ++ix)
        L.push_back(HostLeaf{morton3_host(ix << (10 - B), iy << (10 - B), iz << (10 - B)), (uint8_t)B});
  std::sort(L.begin(), L.end(), [](const HostLeaf& a, const HostLeaf& b) { return a.key < b.key; });
  if (d.refine_disk) {
    const double c[3] = {d.disk_cx, d.disk_cy, d.disk_cz};
    for (;;) {
      std::vector<char> mark(L.size(), 0);
      bool any = false;
      for (size_t i = 0; i < L.size(); ++i) {
        if (L[i].lv >= d.disk_level || L[i].lv >= d.max_level) continue;
        uint32_t X[3];
        unmorton3_host(L[i].key, X);
        const double h = std::ldexp(1.0, -(int)L[i].lv);
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          const double lo = X[a] / 1024.0, hi = lo + h;
          const double g = std::max(std::max(lo - c[a], 0.0), c[a] - hi);
          r2 = r2 + g * g;
        }
        if (r2 <= d.disk_r * d.disk_r) {
          mark[i] = 1;
          any = true;
        }
      }
      if (!any) break;
      L = host_refine3(L, mark);
    }
  }
  host_balance3(L);
  return L;
}

// Mesh tables of an octree slot: keys, levels, packed corners, lookup table
// at level min(max_level, 7) (8^7 + 1 entries, 8 MiB), corner field tables.
void set_mesh3(Ctx& C, Slot& sl, const std::vector<HostLeaf>& L) {
  const size_t n = L.size();
  std::vector<uint32_t> keys(n);
  std::vector<uint8_t> lv(n);
  int mx = 0;
  for (size_t i = 0; i < n; ++i) {
    keys[i] = L[i].key;
    lv[i] = L[i].lv;
    mx = std::max(mx, (int)L[i].lv);
  }
  sl.key = (uint32_t*)sl.alloc(4 * n);
  sl.lv = (uint8_t*)sl.alloc(n);
  hip_check(hipMemcpy(sl.key, keys.data(), 4 * n, hipMemcpyHostToDevice), "upload keys");
  hip_check(hipMemcpy(sl.lv, lv.data(), n, hipMemcpyHostToDevice), "upload levels");
  sl.nleaves = (uint32_t)n;
  sl.nq = sl.nleaves;
  sl.xy = (uint32_t*)sl.alloc(4 * n);
  sl.lut_level = std::min(sl.d.max_level, 7);
  sl.lut_direct = mx <= sl.lut_level;
  sl.lut = (uint32_t*)sl.alloc(4 * ((size_t(1) << (3 * sl.lut_level)) + 1));
  hip_check(launch_leaf_xyz(sl.key, sl.nleaves, sl.xy, C.stream), "leaf_xyz");
  hip_check(launch_build_lut3(sl.key, sl.nleaves, sl.lut, sl.lut_level, C.stream), "build_lut3");
  sl.E = sl.alloc(sl.esz * 24 * n);
  sl.e64 = (double*)sl.alloc(8 * 24 * n);
  sl.cphi = (double*)sl.alloc(8 * 8 * n);
  sl.grad = (double*)sl.alloc(8 * 24 * n);
  sl.phi64 = (double*)sl.alloc(8 * n);
  sl.Q = (unsigned long long*)sl.alloc(8 * 4 * (size_t)sl.nq);
  sl.off = (uint32_t*)sl.alloc(4 * (2 * ((size_t)sl.nq + 1) + scan_tmp_words((uint32_t)sl.nq)));
  sl.scan_tmp = sl.off + 2 * ((size_t)sl.nq + 1);
  hip_check(hipMemsetAsync(sl.E, 0, sl.esz * 24 * n, C.stream), "memset");
  hip_check(hipMemsetAsync(sl.e64, 0, 8 * 24 * n, C.stream), "memset");
  hip_check(hipMemsetAsync(sl.Q, 0, 32 * (size_t)sl.nq, C.stream), "memset");
}

void set_mesh2d(Ctx& C, Slot& sl, const std::vector<HostLeaf>& L) {
  std::vector<uint32_t> keys(L.size());
  std::vector<uint8_t> lv(L.size());
  int mx = 0;
  for (size_t i = 0; i < L.size(); ++i) {
    keys[i] = L[i].key;
    lv[i] = L[i].lv;
    mx = std::max(mx, (int)L[i].lv);
  }
  uint32_t* dk = (uint32_t*)sl.alloc(4 * L.size());
  uint8_t* dl = (uint8_t*)sl.alloc(L.size());
  hip_check(hipMemcpy(dk, keys.data(), 4 * L.size(), hipMemcpyHostToDevice), "upload keys");
  hip_check(hipMemcpy(dl, lv.data(), L.size(), hipMemcpyHostToDevice), "upload levels");
  set_mesh2d_device(C, sl, dk, dl, (uint32_t)L.size(), mx);
}

void build_slot(Ctx& C, Slot& sl, const pic_instance_desc& d) {
  validate(d);
  sl = Slot();
  sl.live = true;
  sl.pool = &C.pool;
  C.pool.stream = C.stream;
  sl.d = d;
  sl.prec = d.precision;
  sl.esz = d.precision == 32 ? 4 : 8;
  derive(sl);
  sl.ctr = (Counters*)sl.alloc(sizeof(Counters));
  hip_check(hipMemsetAsync(sl.ctr, 0, sizeof(Counters), C.stream), "memset");
  sl.part = (unsigned long long*)sl.alloc(sizeof(unsigned long long) * kNStat * kMaxStepGrid);
  hip_check(hipMemsetAsync(sl.part, 0, sizeof(unsigned long long) * kNStat * kMaxStepGrid, C.stream), "memset");
  sl.devI = sl.alloc(sizeof(InstDev<double>));
  if (d.dim == 1) {
    const int N = d.ncells;
    sl.nq = N + 1;
    sl.sort_shift = sort_shift_1d(N);
    sl.E = sl.alloc(sl.esz * (N + 1));
    sl.e64 = (double*)sl.alloc(8 * (N + 1));
    sl.phi64 = (double*)sl.alloc(8 * (N + 1));
    sl.Q = (unsigned long long*)sl.alloc(8 * 4 * (size_t)sl.nq);
    sl.off = (uint32_t*)sl.alloc(8 * ((size_t)N + 1));   // one offset array per species (batched sort)
    hip_check(hipMemsetAsync(sl.E, 0, sl.esz * (N + 1), C.stream), "memset");
    hip_check(hipMemsetAsync(sl.e64, 0, 8 * (N + 1), C.stream), "memset");
    hip_check(hipMemsetAsync(sl.phi64, 0, 8 * (N + 1), C.stream), "memset");
    hip_check(hipMemsetAsync(sl.Q, 0, 32 * (size_t)sl.nq, C.stream), "memset");
    if (d.field_scheme == PIC_FIELD_DIPIC) {
      sl.Qp = (unsigned long long*)sl.alloc(8 * 2 * (size_t)sl.nq);
      sl.dws = (double*)sl.alloc(8 * 3 * (size_t)sl.nq);
      hip_check(hipMemsetAsync(sl.Qp, 0, 16 * (size_t)sl.nq, C.stream), "memset");
    }
  } else if (d.dim == 3) {
    set_mesh3(C, sl, host_build_tree3(d));
  } else {
    set_mesh2d(C, sl, host_build_tree(d));
  }
  // the caller's leaf arrays are read only while building
  sl.d.leaf_keys = nullptr;
  sl.d.leaf_levels = nullptr;
  sl.ionizing = d.nspecies == 2 && d.species[0].mcc == PIC_MCC_ELECTRON;
}

// ---------------------------------------------------------------------------
// particle buffers
// ---------------------------------------------------------------------------
size_t pbuf_bytes(const Slot& sl, int64_t cap) {
  const size_t acc = sl.d.field_scheme == PIC_FIELD_DIPIC ? sl.esz : 0;
  return ((size_t)std::max(sl.d.dim, 2) * sl.esz + 3 * sl.esz + acc + 12) * (size_t)cap + 10 * 256;
}

// A fresh particle buffer of 'cap' slots (nothing of the slot changes if the
// allocation fails).
PBuf new_pbuf(Slot& sl, int64_t cap) {
  // kernels address each particle array with 32-bit byte offsets
  if ((uint64_t)cap * sl.esz >= (1ull << 32) || cap > 0x7FFFFFFF)
    throw Err(PIC_E_CAPACITY, "particle capacity exceeds the per-array limit of 4 GiB");
  PBuf b;
  const size_t e = sl.esz;
  const size_t c = (size_t)cap;
  char* p = (char*)sl.alloc(pbuf_bytes(sl, cap));
  b.base = p;
  size_t o = 0;
  auto carve = [&](size_t n) {
    void* q = p + o;
    o += (n + 255) & ~(size_t)255;
    return q;
  };
  b.s[0] = carve(e * c);
  b.s[1] = sl.d.dim >= 2 ? carve(e * c) : nullptr;
  b.s[2] = sl.d.dim == 3 ? carve(e * c) : nullptr;
  for (int k = 0; k < 3; ++k) b.v[k] = carve(e * c);
  b.w = (uint32_t*)carve(4 * c);
  b.id = (uint32_t*)carve(4 * c);
  b.cell = sl.d.dim >= 2 ? (uint32_t*)carve(4 * c) : nullptr;
  b.acc = sl.d.field_scheme == PIC_FIELD_DIPIC ? carve(e * c) : nullptr;
  return b;
}

// Both particle buffers (live and sort target) of a species for 'cap'
// particles.  The new blocks are allocated before the old ones are given
// back, so a failed allocation leaves the slot as it was.
void alloc_particles(Slot& sl, int sp, int64_t cap) {
  PBuf b0 = new_pbuf(sl, cap);
  PBuf b1;
  try {
    b1 = new_pbuf(sl, cap);
  } catch (...) {
    sl.release(b0.base);
    throw;
  }
  for (int k = 0; k < 2; ++k) sl.release(sl.pb[sp][k].base);
  sl.pb[sp][0] = b0;
  sl.pb[sp][1] = b1;
  sl.cap[sp] = cap;
}

size_t births_bytes(const Slot& sl, int64_t cap) {
  return (20 + (6 + (size_t)std::max(sl.d.dim, 2)) * sl.esz) * (size_t)cap + 4 * (3 * kBirthBins + 1) + 21 * 256;
}

// Births staging of 'cap' entries.  The new block is allocated before the
// old one is given back, so a failed allocation leaves the slot as it was.
void alloc_births(Ctx& C, Slot& sl, int64_t cap) {
  if (!sl.ionizing) return;
  const size_t e = sl.esz, c = (size_t)cap;
  char* p = (char*)sl.alloc(births_bytes(sl, cap));
  if (sl.birth_base) sl.release(sl.birth_base);
  sl.birth_base = p;
  size_t o = 0;
  auto carve = [&](size_t n) {
    void* q = p + o;
    o += (n + 255) & ~(size_t)255;
    return q;
  };
  sl.br_parent = (uint32_t*)carve(4 * c);
  sl.br_rank = (uint32_t*)carve(4 * c);
  hip_check(hipMemsetAsync(sl.br_rank, 0, 4 * c, C.stream), "memset");   // the births kernels keep it zero
  sl.br_cell = (uint32_t*)carve(4 * c);
  sl.br_w = (uint32_t*)carve(4 * c);
  for (int k = 0; k < 3; ++k) sl.br_s[k] = k < std::max(sl.d.dim, 2) ? carve(e * c) : nullptr;
  for (int k = 0; k < 3; ++k) sl.br_ve[k] = carve(e * c);
  for (int k = 0; k < 3; ++k) sl.br_vi[k] = carve(e * c);
  sl.br_sorted = (uint32_t*)carve(4 * c);
  sl.br_bin = (uint32_t*)carve(4 * kBirthBins);
  hip_check(hipMemsetAsync(sl.br_bin, 0, 4 * kBirthBins, C.stream), "memset");   // kept zero as br_rank
  sl.br_bin_off = (uint32_t*)carve(4 * (kBirthBins + 1));
  sl.br_cursor = (uint32_t*)carve(4 * kBirthBins);
  sl.birth_cap = (uint32_t)cap;
}

// ---------------------------------------------------------------------------
// launch checks (PIC_CHECK_LAUNCHES=1 in the environment): every kernel-side
// view of a slot is checked on the host, before it is used, against the
// slot's live blocks: each array a kernel addresses lies inside one live
// block with the extent its count implies, and particle arrays stay below
// 4 GiB (the kernels' 32-bit byte offsets).  A failed check is PIC_E_STATE,
// raised instead of the launch.
// ---------------------------------------------------------------------------
bool launch_checks() {
  static const bool on = [] {
    const char* e = std::getenv("PIC_CHECK_LAUNCHES");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

void check_block(const Slot& sl, const void* p, size_t bytes, const char* what) {
  if (!bytes) return;
  if (!p) throw Err(PIC_E_STATE, std::string("launch check: ") + what + " is null");
  const char* q = (const char*)p;
  for (size_t i = 0; i < sl.allocs.size(); ++i) {
    const char* a = (const char*)sl.allocs[i];
    if (q >= a && q + bytes <= a + sl.alloc_bytes[i]) return;
  }
  throw Err(PIC_E_STATE, std::string("launch check: ") + what + " (" + std::to_string(bytes) +
                             " bytes) is not inside a live block of the slot");
}

// The particle arrays of one buffer for 'cap' particles.
void check_pbuf(const Slot& sl, const PBuf& b, int64_t cap) {
  const size_t c = (size_t)cap, e = sl.esz;
  if ((uint64_t)c * e >= (1ull << 32)) throw Err(PIC_E_STATE, "launch check: a particle array reaches 4 GiB");
  for (int k = 0; k < sl.d.dim; ++k) check_block(sl, b.s[k], c * e, "positions");
  for (int k = 0; k < 3; ++k) check_block(sl, b.v[k], c * e, "velocities");
  check_block(sl, b.w, 4 * c, "weights");
  check_block(sl, b.id, 4 * c, "ids");
  if (sl.d.dim >= 2) check_block(sl, b.cell, 4 * c, "leaf indices");
  if (sl.d.field_scheme == PIC_FIELD_DIPIC) check_block(sl, b.acc, c * e, "filtered accelerations");
}

// Mesh, field and deposit tables.
void check_tables(const Slot& sl) {
  const size_t e = sl.esz, L = sl.nleaves, dim = (size_t)sl.d.dim;
  const size_t n1 = (size_t)sl.d.ncells + 1;
  check_block(sl, sl.ctr, sizeof(Counters), "counters");
  check_block(sl, sl.part, 8 * (size_t)kNStat * kMaxStepGrid, "stats rows");
  if (sl.nq != (dim == 1 ? n1 : L)) throw Err(PIC_E_STATE, "launch check: deposit length does not match the mesh");
  check_block(sl, sl.Q, 32 * (size_t)sl.nq, "deposit");
  if (dim == 1) {
    check_block(sl, sl.E, n1 * e, "field table");
    check_block(sl, sl.phi64, 8 * n1, "potential");
    check_block(sl, sl.e64, 8 * n1, "FP64 field");
    if (sl.d.field_scheme == PIC_FIELD_DIPIC) {
      check_block(sl, sl.Qp, 16 * (size_t)sl.nq, "predicted deposit");
      check_block(sl, sl.dws, 24 * (size_t)sl.nq, "implicit solve scratch");
    }
  } else {
    const size_t corners = dim == 2 ? 4 : 8, lut = (size_t(1) << (dim * (size_t)sl.lut_level)) + 1;
    if (L == 0) throw Err(PIC_E_STATE, "launch check: empty tree");
    check_block(sl, sl.key, 4 * L, "leaf keys");
    check_block(sl, sl.lv, L, "leaf levels");
    check_block(sl, sl.xy, 4 * L, "leaf corners");
    check_block(sl, sl.lut, 4 * lut, "point-location table");
    check_block(sl, sl.E, corners * dim * L * e, "field table");
    check_block(sl, sl.e64, 8 * corners * dim * L, "FP64 field");
    check_block(sl, sl.cphi, 8 * corners * L, "corner potential");
    check_block(sl, sl.grad, 8 * corners * dim * L, "corner gradients");
    check_block(sl, sl.phi64, 8 * L, "cell potential");
    check_block(sl, sl.off, 4 * 2 * (L + 1), "leaf offsets");
    if (sl.d.field_scheme == PIC_FIELD_CIC_AMR) check_block(sl, sl.cellE, 2 * L * e, "cell-centred field");
  }
}

template <class T>
void check_view(const Slot& sl, const InstDev<T>& I) {
  check_tables(sl);
  for (int sp = 0; sp < sl.d.nspecies; ++sp) {
    const PBuf& b = sl.pb[sp][sl.cur[sp]];
    if (!b.base) continue;   // nothing loaded: the kernels see no particles of this species
    if ((void*)I.s[sp][0] != b.s[0] || I.cap[sp] != (uint32_t)sl.cap[sp])
      throw Err(PIC_E_STATE, "launch check: particle view does not match the live buffer");
    check_pbuf(sl, b, sl.cap[sp]);
  }
  if (I.v_len) check_block(sl, I.v_table, 8 * (size_t)I.v_len, "drive table");
  if (sl.ionizing && I.birth_cap) {
    const size_t c = I.birth_cap, e = sizeof(T);
    if ((uint64_t)c * e >= (1ull << 32)) throw Err(PIC_E_STATE, "launch check: births staging reaches 4 GiB");
    for (const void* p : {(const void*)I.br.parent, (const void*)I.br.rank, (const void*)I.br.cell,
                          (const void*)I.br.w, (const void*)I.br.sorted})
      check_block(sl, p, 4 * c, "births staging");
    for (int k = 0; k < std::max(sl.d.dim, 2); ++k) check_block(sl, I.br.s[k], c * e, "births staging");
    for (int k = 0; k < 3; ++k) {
      check_block(sl, I.br.ve[k], c * e, "births staging");
      check_block(sl, I.br.vi[k], c * e, "births staging");
    }
    check_block(sl, I.br.bin, 4 * (size_t)kBirthBins, "births bins");
    check_block(sl, I.br.cursor, 4 * (size_t)kBirthBins, "births bins");
    check_block(sl, I.br.bin_off, 4 * ((size_t)kBirthBins + 1), "births bins");
  }
}

// The sort target of a species and the per-cell offsets of the sort.
void check_sort_target(const Slot& sl, int sp) {
  if (!launch_checks()) return;
  check_pbuf(sl, sl.pb[sp][1 - sl.cur[sp]], sl.cap[sp]);
  const size_t n = sl.d.dim == 1 ? (size_t)sl.d.ncells + 1 : (size_t)sl.nleaves + 1;
  check_block(sl, sl.off, 4 * 2 * n, "cell offsets");
}

template <class T>
InstDev<T> make_dev(const Slot& sl) {
  InstDev<T> I;
  std::memset(&I, 0, sizeof(I));
  const pic_instance_desc& d = sl.d;
  I.dim = d.dim;
  I.N = d.dim == 1 ? d.ncells : 0;
  I.particle_bc = d.particle_bc;
  I.nspecies = d.nspecies;
  I.key0 = (uint32_t)d.seed;
  I.key1 = (uint32_t)(d.seed >> 32) ^ d.instance_key;
  for (int s = 0; s < 2; ++s) {
    I.sk[s] = to_dev<T>(sl.hk[s]);
    const PBuf& b = sl.pb[s][sl.cur[s]];
    I.s[s][0] = (T*)b.s[0];
    I.s[s][1] = (T*)b.s[1];
    I.s[s][2] = (T*)b.s[2];
    I.acc[s] = (T*)b.acc;
    for (int k = 0; k < 3; ++k) I.v[s][k] = (T*)b.v[k];
    I.w[s] = b.w;
    I.id[s] = b.id;
    I.cell[s] = b.cell;
    I.cap[s] = (uint32_t)sl.cap[s];
  }
  I.E = (const T*)sl.E;
  I.leaf_key = sl.key;
  I.leaf_xy = sl.xy;
  I.leaf_lv = sl.lv;
  I.lut = sl.lut;
  I.lut_level = sl.lut_level;
  I.lut_direct = sl.lut_direct ? 1 : 0;
  I.nleaves = sl.nleaves;
  I.Q = sl.Q;
  I.nq = sl.nq;
  I.br.parent = sl.br_parent;
  I.br.rank = sl.br_rank;
  I.br.bin = sl.br_bin;
  I.br.bin_off = sl.br_bin_off;
  I.br.cursor = sl.br_cursor;
  I.br.sorted = sl.br_sorted;
  I.br.cell = sl.br_cell;
  I.br.w = sl.br_w;
  for (int k = 0; k < 3; ++k) I.br.s[k] = (T*)sl.br_s[k];
  for (int k = 0; k < 3; ++k) {
    I.br.ve[k] = (T*)sl.br_ve[k];
    I.br.vi[k] = (T*)sl.br_vi[k];
  }
  I.birth_cap = sl.birth_cap;
  I.ctr = sl.ctr;
  I.v_table = sl.v_table;
  I.v_len = sl.v_len;
  I.part = sl.part;
  I.nparts = (uint32_t)grid_for(sl.cap[0] + sl.cap[1]);
  I.kappa[0] = sl.kappa[0];
  I.kappa[1] = sl.kappa[1];
  I.inv2dx = sl.inv2dx;
  I.cell_e = sl.d.dim == 1 && sl.d.field_scheme == PIC_FIELD_CIC_EC ? 1 : 0;
  I.cic_amr = sl.d.dim == 2 && sl.d.field_scheme == PIC_FIELD_CIC_AMR ? 1 : 0;
  I.dipic = sl.d.dim == 1 && sl.d.field_scheme == PIC_FIELD_DIPIC ? 1 : 0;
  I.sort_shift = sl.sort_shift;
  I.chi[0] = sl.chi[0];
  I.chi[1] = sl.chi[1];
  I.Qp = sl.Qp;
  I.dws = sl.dws;
  I.cellE = (const T*)sl.cellE;
  I.births_binned = slot_births_binned(sl) ? 1 : 0;
  I.phi64 = sl.phi64;
  I.e64 = sl.e64;
  if (launch_checks()) check_view(sl, I);
  return I;
}

// upload the kernel-side view of a slot (device copy used by table-driven kernels)
void upload_dev(Ctx& C, Slot& sl) {
  if (sl.prec == 32) {
    InstDev<float> I = make_dev<float>(sl);
    C.upload(sl.devI, &I, sizeof(I));
  } else {
    InstDev<double> I = make_dev<double>(sl);
    C.upload(sl.devI, &I, sizeof(I));
  }
}

Counters read_counters(Ctx& C, Slot& sl) {
  C.flush_uploads();
  Counters c;
  hip_check(hipMemcpyAsync(&c, sl.ctr, sizeof(c), hipMemcpyDeviceToHost, C.stream), "read counters");
  C.sync();
  return c;
}

void write_counters(Ctx& C, Slot& sl, const Counters& c) { C.upload(sl.ctr, &c, sizeof(c)); }

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > kMaxGrid) g = kMaxGrid;
  return (int)g;
}

// Grow the particle capacity of a species, keeping the first 'count' slots.
// Both new buffers (live and sort target) are allocated before anything of
// the slot changes, so a failed allocation leaves the slot as it was.
void grow(Ctx& C, Slot& sl, int sp, int64_t newcap, uint32_t count) {
  const int cur = sl.cur[sp], other = 1 - cur;
  PBuf nb = new_pbuf(sl, newcap);
  PBuf no;
  try {
    no = new_pbuf(sl, newcap);
  } catch (...) {
    sl.release(nb.base);
    throw;
  }
  const PBuf old = sl.pb[sp][cur];
  const size_t e = sl.esz;
  if (count) {
    hip_check(hipMemcpyAsync(nb.s[0], old.s[0], e * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    if (sl.d.dim >= 2) {
      hip_check(hipMemcpyAsync(nb.s[1], old.s[1], e * count, hipMemcpyDeviceToDevice, C.stream), "grow");
      hip_check(hipMemcpyAsync(nb.cell, old.cell, 4 * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    }
    if (sl.d.dim == 3)
      hip_check(hipMemcpyAsync(nb.s[2], old.s[2], e * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    if (old.acc) hip_check(hipMemcpyAsync(nb.acc, old.acc, e * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    for (int k = 0; k < 3; ++k)
      hip_check(hipMemcpyAsync(nb.v[k], old.v[k], e * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    hip_check(hipMemcpyAsync(nb.w, old.w, 4 * count, hipMemcpyDeviceToDevice, C.stream), "grow");
    hip_check(hipMemcpyAsync(nb.id, old.id, 4 * count, hipMemcpyDeviceToDevice, C.stream), "grow");
  }
  C.sync();
  sl.release(old.base);
  if (sl.pb[sp][other].base) sl.release(sl.pb[sp][other].base);
  sl.pb[sp][cur] = nb;
  sl.pb[sp][other] = no;
  sl.cap[sp] = newcap;
}

// Capacity for the next steps.  A step of an ionizing slot is started only
// with room for its worst case of births (every electron alive ionizes
// once): 2 count[0] electron slots, count[1] + count[0] ion slots and
// count[0] staged births; the need adds the births expected over the coming
// steps.  Growth is to twice that need (less if the slot's memory limit or
// the 32-bit array addressing says so, but never below the need).  Throws PIC_E_CAPACITY (or PIC_E_NOMEM) with the slot unchanged
// when the need cannot be met; the ids still needed are checked too.
void ensure_capacity(Ctx& C, Slot& sl, const Counters& c, int64_t steps_ahead) {
  // births expected over the coming steps (the rate of the previous steps,
  // with a margin): room for them too, so that steps rarely stop for room
  // (a stop only costs time: the slot then waits for the others and is
  // grown before it goes on)
  const int64_t expect = sl.ionizing ? (int64_t)(sl.births_rate * 2.0 * (double)std::max<int64_t>(steps_ahead, 1)) : 0;
  int64_t need[2] = {0, 0};
  for (int sp = 0; sp < sl.d.nspecies; ++sp) {
    need[sp] = c.count[sp];
    if (sl.ionizing) need[sp] += (int64_t)c.count[0] + 2 * expect + 1024;
  }
  if (sl.ionizing && (uint64_t)c.next_id + 2ull * c.count[0] > 0xFFFFFFFFull)
    throw Err(PIC_E_CAPACITY, "particle ids exhausted: the next step could need ids beyond 2^32 - 1");
  bool changed = false;
  const int64_t arr_limit = std::min<int64_t>((int64_t)(((1ull << 32) - 1) / sl.esz), 0x7FFFFFFF);
  // each growth is whole or not done; if a later one fails, the device view
  // is brought up to the earlier ones before the error goes out
  try {
    for (int sp = 0; sp < sl.d.nspecies; ++sp) {
      if (need[sp] <= sl.cap[sp]) continue;
      if (need[sp] > arr_limit) throw Err(PIC_E_CAPACITY, "particle capacity exceeds the per-array limit of 4 GiB");
      int64_t want = std::max(need[sp], std::min(2 * need[sp] + 1024, arr_limit));
      if (sl.byte_limit) {
        // bytes after the growth: the two particle buffers of this species are
        // replaced (births staging follows species 0)
        auto after = [&](int64_t cap) {
          size_t b = sl.bytes_held - 2 * pbuf_bytes(sl, sl.cap[sp]) + 2 * pbuf_bytes(sl, cap);
          if (sp == 0 && sl.ionizing) b = b - (sl.birth_base ? births_bytes(sl, sl.birth_cap) : 0) + births_bytes(sl, cap);
          return b;
        };
        if (after(want) > sl.byte_limit) want = need[sp];
        if (after(want) > sl.byte_limit)
          throw Err(PIC_E_CAPACITY, "the slot's memory limit leaves no room for the next step");
      }
      grow(C, sl, sp, want, c.count[sp]);
      changed = true;
    }
    if (sl.ionizing && sl.birth_cap < (uint64_t)sl.cap[0]) {
      alloc_births(C, sl, sl.cap[0]);
      changed = true;
    }
  } catch (...) {
    if (changed) {
      try {
        upload_dev(C, sl);
      } catch (...) {
        sl.error_state = true;
      }
    }
    throw;
  }
  if (changed) upload_dev(C, sl);
}

// The room check of ensure_capacity without growing: PIC_E_CAPACITY when the
// next step could need more room than the slot holds.
void check_capacity(const Slot& sl, const Counters& c) {
  if (!sl.ionizing) return;
  if ((uint64_t)c.next_id + 2ull * c.count[0] > 0xFFFFFFFFull)
    throw Err(PIC_E_CAPACITY, "particle ids exhausted: the next step could need ids beyond 2^32 - 1");
  if (!room_for_step(c.count[0], c.count[1], c.next_id, (uint64_t)sl.cap[0], (uint64_t)sl.cap[1], sl.birth_cap))
    throw Err(PIC_E_CAPACITY, "the next step needs more particle room than the slot holds (pic_step grows it)");
}

template <class T>
void sort_species(Ctx& C, Slot& sl, int sp) {
  InstDev<T> I = make_dev<T>(sl);
  check_sort_target(sl, sp);
  const int other = 1 - sl.cur[sp];
  PBuf& d = sl.pb[sp][other];
  SortDst<T> dst{(T*)d.s[0], (T*)d.s[1], (T*)d.v[0], (T*)d.v[1], (T*)d.v[2], d.w, d.id, d.cell, (T*)d.s[2],
                 (T*)d.acc};
  const uint32_t ncell = sl.d.dim == 1 ? sort_bins_1d(sl) : sl.nleaves;
  hip_check(launch_sort<T>(I, sp, ncell, sl.off, sl.scan_tmp, dst, grid_for(sl.cap[sp]), C.stream), "sort");
  sl.cur[sp] = other;
}

void sort_slot(Ctx& C, Slot& sl) {
  for (int sp = 0; sp < sl.d.nspecies; ++sp) {
    if (!sl.pb[sp][0].base) continue;
    if (sl.prec == 32) sort_species<float>(C, sl, sp); else sort_species<double>(C, sl, sp);
  }
  upload_dev(C, sl);
}

}  // namespace pic

namespace pic {
template InstDev<float> make_dev<float>(const Slot&);
template InstDev<double> make_dev<double>(const Slot&);
template SpeciesK<float> to_dev<float>(const HostK&);
template SpeciesK<double> to_dev<double>(const HostK&);
}  // namespace pic
