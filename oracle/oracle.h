/*
 * Plain CPU oracle for the electrostatic PIC step on a uniform 1D mesh and
 * on a cell-based quadtree (Kolobov & Arslanbekov, "Electrostatic PIC with
 * adaptive Cartesian mesh", arXiv:1604.07713).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library; the two meet only in the
 * seeded input generators, which hold none of the method's arithmetic.
 *
 * Every routine is a straight loop over particles in id order (or over
 * leaves in Morton order) in the precision T the instance asks for: FP64, or
 * FP32 as an IEEE "mirror" of the GPU's FP32 path (same operations in the
 * same order, no contraction).
 *
 * Section references are to the paper:  Sec. 3 (MCC, multigrid Poisson at
 * cell centres, NGP scatter, bilinear gather from nodal E, explicit PIC with
 * dx < 3 lambda_D, dt < 1/omega_p, CIC on a uniform mesh), Sec. 3.1 (quadtree
 * cell lists, reassignment of particles on refine/coarsen, no per-level
 * weights, ghost cells at +-1 level for direct and diagonal neighbours),
 * Sec. 4.3 (splitting one particle into four in 2D; merging; AMR keeping the
 * particles-per-cell count steady while particles multiply).
 *
 * Parity status of each part is listed in the header comment of oracle.cpp.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_E_ARG = -1, OR_E_CAPACITY = -3, OR_E_STATE = -5 };
enum { OR_MCC_NONE = 0, OR_MCC_ELECTRON = 1, OR_MCC_ION_CX = 2 };
enum { OR_WALL_NEUMANN = 0, OR_WALL_DIRICHLET = 1 };
enum { OR_ABSORB = 0, OR_REFLECT = 1 };
/* particle-field coupling: 1D CIC to nodes, momentum- or energy-conserving
   (Sec. 3); 2D NGP scatter with bilinear gather of nodal E (OR_FIELD_CIC_EM,
   Sec. 3) or the cloud-in-cell on the quadtree with ghost cells at +-1 level
   and the same shape function for scatter and gather (OR_FIELD_CIC_AMR,
   Sec. 3.1) */
enum { OR_FIELD_CIC_EM = 0, OR_FIELD_CIC_EC = 1, OR_FIELD_CIC_AMR = 2,
       /* 1D direct implicit PIC (Sec. 3: DIPIC, the Poisson solve extended
          with the implicit susceptibility), D1 time integration; CIC to the
          nodes with the linear gather; steps only with the field solve */
       OR_FIELD_DIPIC = 3 };
/* field kinds for or_field_set.  OR_NODE_E_1D is for the momentum-conserving
   1D coupling (N+1 node values), OR_CELL_E_1D for the energy-conserving one
   (N cell values); each is refused on the other coupling. */
enum { OR_NODE_E_1D = 0, OR_NODE_PHI_1D = 1, OR_CORNER_PHI_2D = 2, OR_CORNER_E_2D = 3, OR_CELL_PHI_2D = 4,
       OR_CELL_E_1D = 5, OR_CELL_E_2D = 6 /* [leaf][2], cloud-in-cell slots only */,
       /* 3D octree: potentials at each leaf's 8 corners [leaf][8], or E at
          them [leaf][8][3]; corner c = a + 2b + 4e with a, b, e in {0, 1}
          the sides along x, y, z */
       OR_CORNER_PHI_3D = 7, OR_CORNER_E_3D = 8 };

typedef struct {
  double charge;     /* C */
  double mass;       /* kg */
  double w0;         /* real particles carried by w_units = 2^16 (1D: per m^2) */
  int mcc;           /* OR_MCC_* */
  double sigma_el, sigma_iz, eps_iz;  /* electron: m^2, m^2, eV */
  double sigma_cx;                    /* ion charge exchange, m^2 */
  double eps_max;                     /* eV; sets nu_max of the null-collision method */
} or_species;

typedef struct {
  int dim;           /* 1, 2 or 3 (3: static octree, field given at the nodes) */
  int precision;     /* 32 or 64 (particle arithmetic); field solve is FP64 */
  double length;     /* 1D gap / 2D square side, m */
  double dt;         /* s */
  int ncells;        /* 1D uniform cells */
  int min_level, max_level, base_level;        /* 2D (levels <= 14), 3D (levels <= 10) */
  int refine_disk; double disk_cx, disk_cy, disk_r; int disk_level;  /* 2D disk / 3D ball refinement */
  int field_bc[4]; double wall_phi[4];        /* 2D walls x0,x1,y0,y1 */
  int particle_bc;   /* OR_ABSORB / OR_REFLECT */
  double depth_z;    /* 2D out-of-plane length, m */
  double gas_density, gas_temperature, gas_mass;
  uint64_t seed; uint32_t instance_key;
  int nspecies;      /* 1 or 2: [0] electrons, [1] ions */
  or_species species[2];
  int field_scheme;  /* 1D: OR_FIELD_CIC_EM (node E, linear gather) or
                        OR_FIELD_CIC_EC (cell E, the particle's cell value) */
  /* 2D explicit tree (nleaves > 0): leaves in Morton order, key = Morton code
     of the leaf's low corner in 16-bit units (x in the even bits), level per
     leaf.  They must tile the square, lie within [min_level, max_level] and be
     2:1 balanced across faces and corners, else or_create fails.  base_level
     and the disk refinement are then ignored. */
  const uint32_t* leaf_keys;
  const uint8_t* leaf_levels;
  int64_t nleaves;
  double disk_cz;    /* 3D: z of the refined ball's centre (x, y: disk_cx, disk_cy) */
} or_desc;

typedef struct {
  int64_t alive_start[2];
  int64_t absorbed[2];
  int64_t elastic, ionization, cx, births;
  int64_t numax_violations[2];
  int64_t lost_reflect;   /* reflected particle still outside: absorbed */
} or_stats;

typedef struct {
  int64_t refined, coarsened, balance_refined;
  int64_t split_parents, merged_pairs;
  int64_t nleaves;
  double merge_energy_change;   /* J-equivalent in (w_units * v^2) units */
} or_adapt_stats;

void* or_create(const or_desc* d);
void or_destroy(void* h);
int or_load(void* h, int species, int64_t n, const double* s, const double* v,
            const uint32_t* w, const uint32_t* id);
int64_t or_count(void* h, int species);
uint32_t or_next_id(void* h);
int or_read(void* h, int species, double* s, double* v, uint32_t* w, uint32_t* id, uint32_t* cell);
int64_t or_nleaves(void* h);
int or_leaves(void* h, uint32_t* keys, uint8_t* levels);
int64_t or_nq(void* h);   /* nodes (1D) or leaves (2D) */
int or_deposit(void* h, uint64_t* q_out);
/* charge density of the latest deposit per node (1D, C/m^3: the node sum over
   dx) or per leaf (2D, C/m^3: the leaf sum over h^2 depth_z) */
int or_rho(void* h, double* rho_out);
/* corner potentials [leaf][4] behind the current 2D field table (after a
   CORNER_PHI / CELL_PHI field set or a 2D solve) */
int or_corner_phi(void* h, double* out);
/* set the next id handed to births and split copies; OR_E_ARG if an id in use
   is not below it */
int or_set_next_id(void* h, uint32_t next_id);
int or_field_set(void* h, int kind, const double* data);
int or_field_table(void* h, double* out);
int or_field_solve_1d(void* h, double phi_left, double* phi_out, double* e_out);
/* direct implicit slots (test hook): deposit the particles as they are and
   solve the implicit Poisson equation with phi(0) = phi_left, phi(L) = 0;
   phi_out[N+1] the node potentials, chi_out[N+1] the node susceptibility;
   the E table is set from them */
int or_dipic_field(void* h, double phi_left, double* phi_out, double* chi_out);
int or_field_solve_2d(void* h, const double* phi_init, double rtol, int maxit,
                      double* phi_out, int* iters, double* relres);
int64_t or_assemble_2d(void* h, int32_t* rows, int32_t* cols, double* vals, double* rhs);
int or_leapfrog_start(void* h);
int or_step(void* h, int64_t step0, int nsteps, const double* v_next, int solve_1d, or_stats* st);
int or_adapt(void* h, int n_lo, int n_hi, or_adapt_stats* st);
int or_locate(void* h, int64_t n, const double* s, uint32_t* leaf);
/* the field the step's gather gives at n positions s[n*dim] (the current
   table, the slot's coupling): out[n*dim] (test helper) */
int or_gather(void* h, int64_t n, const double* s, double* out);
void or_derived(void* h, int species, double* out);
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
