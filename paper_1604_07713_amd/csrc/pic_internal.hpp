// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pic.h"

namespace pic {

constexpr int kBlock = 256;          // threads per workgroup of the particle kernels
constexpr int kKeyBits = 16;         // quadtree keys: Morton code of 16-bit coordinates

// Per-instance device counters.  Updated only by kernels, so a sequence of
// steps (or a captured graph) runs without host round trips.
struct Counters {
  uint32_t count[2];     // particle slots in use per species (live + holes)
  uint32_t next_id;
  uint32_t nbirths;      // staged births of the current step
  uint32_t flags;        // kFlag* bits
  uint32_t step;         // global index of the next step
  uint32_t vstep0;       // step index of v_table[0]
  uint32_t done;         // workgroups finished in the current launch
  unsigned long long stats[12];
};
// kFlagNeedRoom: a step found less room than its worst case of births needs
// and was not run (nor any later one, until the host clears the flag): the
// instance stays at its last committed step.  The other flags mark overflows
// that this check rules out; they remain as a guard.
enum : uint32_t { kFlagBirthOverflow = 1u, kFlagIdOverflow = 2u, kFlagSplitOverflow = 4u, kFlagNeedRoom = 8u };
enum StatIdx {
  kStAlive0 = 0, kStAlive1, kStAbs0, kStAbs1, kStElastic, kStIonization, kStCx, kStBirths,
  kStViol0, kStViol1, kStLostReflect, kStUnused
};

template <class T>
struct SpeciesK {
  T qm_dt, hqm_dt, dt_L;
  T a_el, a_iz, v_iz2, mu2, vmax2, v_thg, a_cx, gmax;
  uint32_t tcand;
  int mcc;
};

template <class T>
struct Births {          // staging of one step's ionization births (SoA)
  uint32_t* parent;
  uint32_t* rank;        // rank of the parent id among the staged ones (kept zero between steps)
  uint32_t* bin;         // [kBirthBins] staged parents per id bin (kept zero between steps)
  uint32_t* bin_off;     // [kBirthBins + 1] first position of each bin in 'sorted'
  uint32_t* cursor;      // [kBirthBins] fill positions
  uint32_t* sorted;      // staged parent ids grouped by bin
  uint32_t* cell;
  uint32_t* w;
  T* s[3];
  T* ve[3];
  T* vi[3];
};

// Kernel-side view of one instance.
template <class T>
struct InstDev {
  int dim, N, particle_bc, nspecies;
  uint32_t key0, key1;           // Philox key
  SpeciesK<T> sk[2];
  T* s[2][3];                    // [species][axis] (axis 2: 3D only)
  T* v[2][3];
  uint32_t* w[2];
  uint32_t* id[2];
  uint32_t* cell[2];
  T* acc[2];                     // direct implicit: (dt/2) x filtered acceleration (else null)
  uint32_t cap[2];
  const T* E;                    // 1D node E [N+1]; 2D corner E [nleaves][4][2]; 3D corner E [nleaves][8][3]
  const uint32_t* leaf_key;
  const uint32_t* leaf_xy;       // 2D: (x0 << 16) | y0 in 16-bit units; 3D: x0 | y0 << 10 | z0 << 20 in 10-bit units
  const uint8_t* leaf_lv;
  const uint32_t* lut;           // leaf containing each level-lut_level cell's low corner
  int lut_level;
  int lut_direct;                // no leaf finer than lut_level
  uint32_t nleaves;
  unsigned long long* Q;         // [2 parity][2 species][nq]
  uint32_t nq;
  Births<T> br;
  uint32_t birth_cap;
  Counters* ctr;
  const double* v_table;         // 1D drive potential per step (solve on device)
  uint32_t v_len;
  unsigned long long* part;      // per-block partial stats [nparts][kNStat]
  uint32_t nparts;
  // FP64 field data
  double kappa[2];               // charge-sum -> Poisson right-hand side factor per species
  double inv2dx;                 // 1D: 1 / (2 dx)
  int dipic;                     // 1D direct implicit step (D1 scheme)
  uint32_t sort_shift;           // 1D: particles are kept ordered by bins of 2^sort_shift cells
  double chi[2];                 // direct implicit: charge-sum -> susceptibility factor per species
  unsigned long long* Qp;        // direct implicit: charge at the predicted positions [2][N+1]
  double* dws;                   // direct implicit solve scratch [3][N+1] (meshes beyond one LDS chunk)
  int cell_e;                    // 1D energy-conserving coupling: E holds cell values, gathered without interpolation
  int cic_amr;                   // 2D cloud-in-cell coupling: deposit and gather through the particle's cloud
  const T* cellE;                // 2D cloud-in-cell: cell-centred E [nleaves][2]
  int births_binned;             // births ranked through id bins (else pairwise)
  double* phi64;                 // 1D: node potential; 2D: cell potential
  double* e64;                   // 1D: node E; 2D: corner E [nleaves][8]
};
constexpr int kNStat = 12;

// Room for one step of an ionizing instance: every electron alive at the
// start of the step can ionize at most once, so a step appends at most
// count[0] electrons and as many ions, stages as many births and uses twice
// as many ids.  A step without that room is not started (every workgroup of
// every launch of the step sees the same counters and decides alike), so
// the instance is never left part-way through a step.
__host__ __device__ inline bool room_for_step(uint32_t count0, uint32_t count1, uint32_t next_id, uint64_t cap0,
                                              uint64_t cap1, uint64_t birth_cap) {
  const uint64_t c0 = count0, c1 = count1;
  return 2u * c0 <= cap0 && c1 + c0 <= cap1 && c0 <= birth_cap && (uint64_t)next_id + 2u * c0 <= 0xFFFFFFFFull;
}
template <class T>
__device__ __forceinline__ bool step_blocked(const InstDev<T>& I) {
  const Counters* c = I.ctr;
  if (c->flags & kFlagNeedRoom) return true;
  if (I.nspecies < 2 || I.sk[0].mcc != PIC_MCC_ELECTRON) return false;   // no births
  return !room_for_step(c->count[0], c->count[1], c->next_id, I.cap[0], I.cap[1], I.birth_cap);
}

// Births per step above which the ranking goes through id bins (pairwise
// ranking work grows as the square of the births).
constexpr double kBinnedBirthsPerStep = 2048.0;

// Work item of the batched (persistent) launches.
struct WorkItem {
  uint32_t inst, species, begin, end;
};

// ---- launchers (k_step.hip) ----
// commit != 0: the last workgroup advances the step index (no births kernel
// or field solve follows in this step).
// t0 / t1, when given, receive the step kernel's own start and end (timing).
template <class T> hipError_t launch_step(const InstDev<T>& I, hipStream_t s, int grid, bool mcc, int commit,
                                          hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
template <class T> int step_resident_grid(int dim, bool mcc, bool direct);
template <class T> hipError_t launch_step1d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                                    unsigned long long* bpart, hipStream_t s, int grid, bool mcc);
template <class T> hipError_t launch_step2d_batched(const InstDev<T>* I, const WorkItem* items, uint32_t nitems,
                                                    unsigned long long* bpart, hipStream_t s, int grid, bool mcc);
// Births of one step: rank the staged births by parent id, append the pairs.
// binned: rank through id bins (work ~ births x births per bin) instead of
// comparing every pair (work ~ births^2); the host picks it for many births.
constexpr uint32_t kBirthBins = 4096;
template <class T> hipError_t launch_births(const InstDev<T>& I, hipStream_t s, bool binned);
// pair_births / bin_births: the most births per step expected of an
// instance ranked pairwise / through id bins (its births_binned flag); they
// size the grids, and a negative value means no instance ranks that way
template <class T> hipError_t launch_births_batched(const InstDev<T>* I, int ninst, hipStream_t s,
                                                    double pair_births, double bin_births);
template <class T> hipError_t launch_commit(const InstDev<T>& I, hipStream_t s);
template <class T> hipError_t launch_commit_batched(const InstDev<T>* I, int ninst, hipStream_t s);
template <class T> hipError_t launch_stats_reduce(const InstDev<T>* I, int ninst, unsigned long long* rows,
                                                  const uint32_t* row_begin, uint32_t nrows_plain, hipStream_t s);
template <class T> hipError_t launch_deposit(const InstDev<T>& I, hipStream_t s, int grid);
// cell-centred E table [nleaves][2] of the cloud-in-cell coupling from the
// FP64 corner table [nleaves][8]
template <class T> hipError_t launch_cell_e(const double* corner_e64, uint32_t nleaves, T* cellE, hipStream_t s);
// the field the step's gather gives at n device points pts[n*dim] -> out[n*dim]
template <class T> hipError_t launch_gather_points(const InstDev<T>& I, const double* pts, int64_t n, double* out,
                                                   hipStream_t s);
template <class T> hipError_t launch_leapfrog_start(const InstDev<T>& I, hipStream_t s, int grid);
template <class T> hipError_t launch_relocate(const InstDev<T>& I, int species, hipStream_t s, int grid);
// 1D direct implicit step: predictor (grid workgroups), field (one
// workgroup), corrector (grid workgroups); births and commit follow.
template <class T> hipError_t launch_dipic_predict(const InstDev<T>& I, hipStream_t s, int grid);
template <class T> hipError_t launch_dipic_field(const InstDev<T>& I, hipStream_t s);
template <class T> hipError_t launch_dipic_correct(const InstDev<T>& I, hipStream_t s, int grid, bool mcc);

// ---- field (k_field.hip) ----
// mode 0: solve from the latest deposit with phi(0) = phi_left[inst];
// mode 1: after a step: solve from this step's deposit with phi(0) from the
//         drive table, then commit the step (rows: partial-stats rows).
template <class T> hipError_t launch_field1d(const InstDev<T>* insts, int ninst, int max_n, int mode,
                                             const double* phi_left, hipStream_t s);
template <class T> hipError_t launch_node_e_1d(const InstDev<T>& I, const double* data, int is_phi, hipStream_t s);
// charge density per node (1D, lv = NULL) or leaf (2D) from Q[species][nq];
// shift = 16 (+ F in 1D)
// charge density per cell: 1D (lv null) over dx; 2D over h^2 depth_z; 3D
// (cube != 0) over h^3
hipError_t launch_rho(const unsigned long long* Q, uint32_t nq, int nspecies, double qw0_0, double qw0_1, int shift,
                      double dx, const uint8_t* lv, double length, double depth_z, int cube, double* rho,
                      hipStream_t s);
struct Mesh2D {
  const uint32_t* key;
  const uint32_t* xy;
  const uint8_t* lv;
  const uint32_t* lut;
  int lut_level;
  uint32_t nleaves;
  double length;
  int field_bc[4];
  double wall_phi[4];
};
template <class T> hipError_t launch_corner_field(const Mesh2D& m, const double* corner_phi, double* grad,
                                                  double* corner_e64, T* corner_e, hipStream_t s);
// octree (the mesh view carries the packed 10-bit corners in xy): corner
// potentials [leaf][8] -> gradients [leaf][8][3] -> nodal E [leaf][8][3]
template <class T> hipError_t launch_corner_field3(const Mesh2D& m, const double* corner_phi, double* grad,
                                                   double* corner_e64, T* corner_e, hipStream_t s);
hipError_t launch_cell_to_corner_phi(const Mesh2D& m, const double* cell_phi, double* corner_phi, hipStream_t s);
template <class T> hipError_t launch_round_table(const double* src, T* dst, int64_t n, hipStream_t s);
struct Stencil2D {
  uint32_t* nbr;     // [nleaves][8]; unused entries point at the leaf itself
  // [nleaves + 1]: 2 bits per neighbour entry k (bits 2k, 2k+1): 0 unused,
  // 1 face coefficient 1 (same level), 2 coefficient 2/3 (levels one apart);
  // the last word is set when a face between leaves more than one level
  // apart was found (not a 2:1 tree)
  uint32_t* code;
  double* diag;      // [nleaves]
  double* bnd;       // [nleaves] Dirichlet contribution to the right-hand side
};
hipError_t launch_build_stencil(const Mesh2D& m, const Stencil2D& st, hipStream_t s);
// CG work vectors, block partials and scalars live in 'ws' (layout in
// k_field.hip); the scalars sit at cg_scalars_offset(nleaves) doubles.
struct CgScal {
  double gam[2];   // r.u of the last two iterations (by parity)
  double alf[2];   // alpha of the last two iterations (by parity)
  double rr, bb;   // r.r of the last iteration checked, b.b
  uint32_t it;     // iterations done when the stopping test was last checked
  uint32_t done;   // stopping test met: later launches return at once
};
hipError_t launch_cg_setup(const Mesh2D& m, const Stencil2D& st, const unsigned long long* Q, int nspecies,
                           const double* kappa, double* x, double* ws, hipStream_t s);
// iteration k = 0, 1, 2, ... in order after the setup; the launch of k = maxit
// only checks and stops
hipError_t launch_cg_iter(const Mesh2D& m, const Stencil2D& st, double* x, double* ws, uint32_t k, double rtol2,
                          uint32_t maxit, hipStream_t s);
int cg_ws_doubles(uint32_t nleaves);
int cg_grid(uint32_t nleaves);
size_t cg_scalars_offset(uint32_t nleaves);

// ---- mesh (k_mesh.hip) ----
hipError_t launch_build_lut(const uint32_t* key, const uint8_t* lv, uint32_t nleaves, uint32_t* lut, int lut_level,
                            hipStream_t s);
// dst[l] = src[old leaf holding the centre of new leaf l]
hipError_t launch_remap_cells(const uint32_t* nxy, const uint8_t* nlv, uint32_t n, const uint32_t* okey,
                              const uint8_t* olv, const uint32_t* olut, int olut_level, const double* src, double* dst,
                              hipStream_t s);
hipError_t launch_leaf_xy(const uint32_t* key, const uint8_t* lv, uint32_t nleaves, uint32_t* xy, hipStream_t s);
// octree: packed 10-bit corner coordinates of each leaf, and the lookup
// table at level L (8^L + 1 entries)
hipError_t launch_leaf_xyz(const uint32_t* key, uint32_t nleaves, uint32_t* xyz, hipStream_t s);
hipError_t launch_build_lut3(const uint32_t* key, uint32_t nleaves, uint32_t* lut, int lut_level, hipStream_t s);
__host__ __device__ inline uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

}  // namespace pic
