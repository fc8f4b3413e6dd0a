/*
 * pic.h — C ABI of the MI355X (gfx950) ES-PIC particle-loop library.
 *
 * Method: Kolobov & Arslanbekov, "Electrostatic PIC with adaptive Cartesian
 * mesh" (arXiv:1604.07713).  The library advances charged super-particles of
 * one or more independent instances ("slots") on a uniform 1D mesh or on a
 * cell-based quadtree.  Every step runs on the GPU in hand-written HIP
 * kernels:
 *   gather E at the particle (Sec. 3: bilinear interpolation of nodal E;
 *     linear on the uniform 1D mesh), explicit leapfrog push (Sec. 3),
 *   wall rule, locate the leaf cell that holds the particle (Sec. 3.1),
 *   null-collision Monte Carlo collisions with the background gas and
 *     ionization births (Sec. 3 MCC; Sec. 4.3 exponential multiplication),
 *   charge deposit (Sec. 3: NGP to quadtree leaves, CIC to the nodes of the
 *     uniform mesh; no per-level volume weighting, Sec. 3.1),
 *   quadtree adaptation to the particle count with particle split/merge
 *     (Sec. 3.1 reassignment on refine/coarsen; Sec. 4.3 splitting 1 -> 4).
 * The Poisson solves (FP64 Thomas in 1D; FP64 cell-centred finite volumes
 * with Jacobi-preconditioned CG in 2D, standing in for the paper's multigrid
 * of Sec. 3) also run in kernels of this library.
 *
 * Conventions common to all calls:
 *  - Every call returns an int status (PIC_OK or a negative PIC_E_*); no
 *    exception crosses the ABI.  pic_last_error() gives a per-context text.
 *  - Host arrays passed in are copied; the caller keeps ownership.  Output
 *    arrays are caller-allocated host buffers of the stated size.
 *  - Positions are normalised to the domain: s = x / length in [0, 1)^dim.
 *    Velocities are in m/s (three components in 1D and 2D).  Particle weight
 *    is an integer w_units; w_units = 2^16 carries species.w0 real particles.
 *  - Particle ids are unique u32 per instance across species.
 *  - All device work is enqueued on the stream given to pic_mesh_build (or
 *    pic_set_stream); a context is not thread-safe.  Calls that return data
 *    to the host synchronise that stream.
 *  - Particle storage order on the device is unspecified; results (ids,
 *    states, deposits) do not depend on it.  Reads return particles sorted by
 *    id.
 *  - A device-side capacity overflow (births or split copies beyond the
 *    reserved slots, or u32 id exhaustion) returns PIC_E_CAPACITY; the
 *    instance is then in an error state (PIC_E_STATE on further steps).
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 2

typedef struct pic_ctx_s* pic_ctx;

enum pic_status {
  PIC_OK = 0,
  PIC_E_ARG = -1,        /* invalid argument or descriptor */
  PIC_E_NOMEM = -2,      /* device allocation failed */
  PIC_E_CAPACITY = -3,   /* births / split copies / ids exceeded capacity */
  PIC_E_HIP = -4,        /* a HIP runtime call failed */
  PIC_E_STATE = -5,      /* call not valid in the instance's state */
  PIC_E_NUMERIC = -6     /* field solve did not converge */
};

enum { PIC_MCC_NONE = 0, PIC_MCC_ELECTRON = 1, PIC_MCC_ION_CX = 2 };
enum { PIC_WALL_NEUMANN = 0, PIC_WALL_DIRICHLET = 1 };
enum { PIC_ABSORB = 0, PIC_REFLECT = 1 };
/* Particle-field coupling on the uniform 1D mesh (Sec. 3), both with CIC
 * charge assignment to the nodes: momentum-conserving (the particle's E is
 * interpolated linearly between its cell's node E values) or energy-
 * conserving (the particle takes its cell's E, the difference of the cell's
 * two node potentials over dx; the field table then holds N cell values). */
enum { PIC_FIELD_CIC_EM = 0, PIC_FIELD_CIC_EC = 1 };
enum { PIC_FP32 = 32, PIC_FP64 = 64 };
/* field kinds for pic_field_set */
enum {
  PIC_NODE_E_1D = 0,     /* double[ncells+1]: E at the nodes, V/m            */
  PIC_NODE_PHI_1D = 1,   /* double[ncells+1]: potential at the nodes, V      */
  PIC_CORNER_PHI_2D = 2, /* double[nleaves][4]: potential at leaf corners     */
  PIC_CORNER_E_2D = 3,   /* double[nleaves][4][2]: nodal E at leaf corners    */
  PIC_CELL_PHI_2D = 4    /* double[nleaves]: cell-centre potential            */
};
/* corner order of a leaf: 0 = (x0,y0), 1 = (x1,y0), 2 = (x0,y1), 3 = (x1,y1) */

typedef struct {
  double charge;        /* C */
  double mass;          /* kg */
  double w0;            /* real particles carried by w_units = 2^16 (1D: per m^2) */
  int mcc;              /* PIC_MCC_*: electron elastic+ionization, or ion charge exchange */
  double sigma_el;      /* m^2, electron elastic (constant)                      */
  double sigma_iz;      /* m^2, electron-impact ionization above eps_iz          */
  double eps_iz;        /* eV                                                     */
  double sigma_cx;      /* m^2, ion charge exchange                              */
  double eps_max;       /* eV, sets the null-collision frequency bound           */
} pic_species_desc;

typedef struct {
  int dim;              /* 1 (uniform mesh) or 2 (quadtree)                      */
  int precision;        /* PIC_FP32 or PIC_FP64: particle arithmetic             */
  double length;        /* m: 1D gap, or side of the 2D square                   */
  double dt;            /* s                                                      */
  int ncells;           /* 1D: uniform cells (2 .. 1<<20)                        */
  int min_level, max_level, base_level;   /* 2D levels, 0 .. 14                 */
  int refine_disk;      /* 2D: refine leaves whose closed box meets the disk ... */
  double disk_cx, disk_cy, disk_r;        /* ... (normalised centre, radius)    */
  int disk_level;       /* ... up to this level, then 2:1 balance               */
  int field_bc[4];      /* 2D walls x=0, x=1, y=0, y=1: PIC_WALL_*               */
  double wall_phi[4];   /* Dirichlet wall potentials, V                          */
  int particle_bc;      /* PIC_ABSORB or PIC_REFLECT                             */
  double depth_z;       /* 2D: out-of-plane length for the charge density, m     */
  double gas_density, gas_temperature, gas_mass;   /* m^-3, K, kg               */
  uint64_t seed;        /* Philox key = (seed_lo, seed_hi ^ instance_key)        */
  uint32_t instance_key;
  int nspecies;         /* 1 or 2: [0] electrons, [1] ions (births need both)    */
  pic_species_desc species[2];
  int64_t capacity[2];  /* particle slots per species; 0 = sized from the load
                           (3x the loaded count + 4096 when ionizing); grows to
                           2x the projected need between chunks of steps       */
  int field_scheme;     /* 1D: PIC_FIELD_CIC_EM or PIC_FIELD_CIC_EC; 2D: must be
                           PIC_FIELD_CIC_EM (NGP deposit, bilinear gather)      */
} pic_instance_desc;

typedef struct {
  int64_t alive_start[2];       /* particle-updates: particles alive at step start */
  int64_t absorbed[2];
  int64_t elastic, ionization, cx, births;
  int64_t numax_violations[2];  /* speed above the null-collision bound (should be 0) */
  int64_t lost_reflect;         /* reflected but still outside: removed        */
  double loop_ms;               /* summed duration of the timed particle-loop launches (timing != 0) */
  double step_ms;               /* wall duration of the call on the stream (timing != 0) */
  int64_t loop_launches;        /* particle-loop launches timed in loop_ms               */
} pic_step_stats;

typedef struct {
  int64_t step0;        /* global index of the first step (Philox counter word 1); */
                        /* < 0: every slot continues from its own step index      */
  int nsteps;
  int solve_field;      /* 1D: after each step solve Poisson on the device with   */
  const double* v_next; /* ... phi(0) = v_next[k*ninst_sel + j] for step k, slot j */
  int sort_every;       /* re-sort particles by cell every n steps (0 = never)    */
  int batched;          /* 0: launches per slot; > 0: one persistent launch over   */
                        /* all selected 1D slots of one precision, with this many  */
                        /* particles per work item (1 = 4096)                      */
  int grid;             /* workgroups of the particle kernel: persistent grid of the
                           batched launch (0 = 2048), or grid of the per-slot launch
                           (0 = one workgroup per 256 particles, at most 2048);
                           at most 8192                                         */
  int graph_steps;      /* batched only: capture this many steps into a HIP graph  */
                        /* and replay it (0 = no graph)                            */
  const int* slots;     /* selected slots (NULL = all live slots)                 */
  int nslots;
  int timing;           /* 0: no events; n > 0: record HIP events around the      */
                        /* particle-loop kernel of every n-th step of the call      */
                        /* (per-slot launches; batched launches: every step), and   */
                        /* around the whole call.  PIC_E_ARG if negative.           */
} pic_step_args;

typedef struct {
  int n_lo, n_hi;       /* target particles per leaf and species, e.g. 16 and 64 */
} pic_adapt_args;

typedef struct {
  int64_t refined, coarsened, balance_refined;
  int64_t split_parents, merged_pairs;
  int64_t nleaves;
  double merge_energy_change;   /* sum over merges of w (|v'|^2) - (w1|v1|^2 + w2|v2|^2) */
} pic_adapt_stats;

/* Device memory from the caller (e.g. a framework's caching allocator):
 * alloc(bytes, stream, user) returns device memory usable in stream order on
 * 'stream' (the context's stream) or NULL; free(p, user) gives a block back.
 * The library hands a block back only after its stream has finished every
 * queued use of it. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* p, void* user);
  void* user;
} pic_allocator;

/* Route the particle, mesh, field and adaptation-scratch memory of a context
 * through 'a' (NULL: hipMalloc with the library's own block cache).  Only on
 * a context that holds no instance yet (build with ninst = 0, then
 * pic_admit): else PIC_E_STATE.  The allocator must outlive the context. */
int pic_set_allocator(pic_ctx c, const pic_allocator* a);

/* Build a context holding ninst >= 0 instances (slots 0..ninst-1; more can be
 * admitted later with pic_admit): uniform 1D mesh,
 * or quadtree (uniform at base_level, optional disk refinement, 2:1 balance
 * across faces and corners; Sec. 3.1).  'stream' is a hipStream_t (NULL =
 * default stream).  On success *out owns all device state. */
int pic_mesh_build(const pic_instance_desc* descs, int ninst, void* stream, pic_ctx* out);

/* Replace the particles of one species of one slot with n host particles:
 * s[n*dim] normalised positions in [0,1), v[n*3] m/s, w[n] (NULL: 2^16 each),
 * id[n] (NULL: 0..n-1).  Values are rounded to the slot's precision.
 * PIC_E_ARG if a position is outside [0,1). */
int pic_particles_load(pic_ctx c, int slot, int species, int64_t n, const double* s, const double* v,
                       const uint32_t* w, const uint32_t* id);

/* Set the field table the gather reads (see the PIC_*_1D/2D kinds).  2D nodal
 * E is the mean over the leaves having the node as a corner of their
 * corner gradients (Sec. 3, bilinear gather from nodal E). */
int pic_field_set(pic_ctx c, int slot, int kind, const double* data);

/* v <- v - (q dt / 2m) E(x): start the leapfrog from the current field. */
int pic_leapfrog_start(pic_ctx c, int slot);

/* Advance nsteps steps: gather, push, walls, locate, MCC with births, deposit
 * (Sec. 3, 3.1, 4.3) for the selected slots; stats are summed over slots. */
int pic_step(pic_ctx c, const pic_step_args* a, pic_step_stats* stats);

/* Deposit the current particles (CIC to nodes in 1D, NGP to leaves in 2D) and
 * copy the per-species integer charge sums to q_out[2][nq] (may be NULL).  1D
 * units: w_units * 2^F (F = 24 FP32, 32 FP64); 2D: w_units. */
int pic_deposit(pic_ctx c, int slot, uint64_t* q_out);

/* How a slot ranks the staged births of a step by parent id (Sec. 4.3
 * births; the ranks fix the newborn ids): 0 (default) pairwise while recent
 * steps had up to 16384 births each, binned above; 1 always pairwise
 * (work ~ births^2); 2 always binned (parent ids grouped in 4096 id bins,
 * work ~ births x births per bin).  Both give the same ranks.  PIC_E_ARG for
 * another method. */
int pic_set_births_ranking(pic_ctx c, int slot, int method);

/* Copy the latest per-species integer charge sums to q_out[2][nq] without
 * depositing again: after pic_step, the sums the last step's particle loop
 * accumulated (its survivors and births); after pic_deposit or pic_adapt,
 * theirs.  Units as pic_deposit.  PIC_E_ARG if q_out is NULL. */
int pic_deposit_read(pic_ctx c, int slot, uint64_t* q_out);

/* Poisson from the latest deposit.  1D: Thomas with phi(0) = phi_left,
 * phi(L) = 0; outputs phi_out/e_out[ncells+1] (nullable).  2D: FV +
 * Jacobi CG from phi_init (nullable) to rtol, at most maxit iterations;
 * phi_out[nleaves]; e_out[nleaves*8] corner E (nullable).  Either sets the
 * gather table.  PIC_E_NUMERIC if CG did not reach rtol. */
int pic_field_solve(pic_ctx c, int slot, double phi_left, const double* phi_init, double rtol, int maxit,
                    double* phi_out, double* e_out, int* iters, double* relres);

/* Adapt the quadtree of a 2D slot to the particle count (Sec. 3.1, 4.3):
 * coarsen sibling groups holding at most n_hi with a child below n_lo, refine
 * leaves above n_hi (repeatedly), 2:1 balance, reassign particles by
 * position, split particles 1 -> 4 in leaves below n_lo, merge pairs in
 * leaves above n_hi at max_level.  Ends with a fresh deposit. */
int pic_adapt(pic_ctx c, int slot, const pic_adapt_args* a, pic_adapt_stats* s);

/* ---- helpers ---- */
int64_t pic_count(pic_ctx c, int slot, int species);          /* live particles, or < 0 on error */
uint32_t pic_next_id(pic_ctx c, int slot);
/* copy one species sorted by id: s[n*dim], v[n*3], w[n], id[n], cell[n] (all nullable) */
int pic_particles_read(pic_ctx c, int slot, int species, double* s, double* v, uint32_t* w, uint32_t* id,
                       uint32_t* cell);
int64_t pic_nleaves(pic_ctx c, int slot);
int pic_leaves_read(pic_ctx c, int slot, uint32_t* keys, uint8_t* levels);   /* Morton order */
int64_t pic_nq(pic_ctx c, int slot);                           /* nodes (1D) or leaves (2D) */
int pic_field_read(pic_ctx c, int slot, double* out);          /* gather table, as double */
int pic_sort(pic_ctx c, int slot);                             /* drop holes, order by cell */
int pic_locate(pic_ctx c, int slot, int64_t n, const double* s, uint32_t* leaf);
int pic_derived(pic_ctx c, int slot, int species, double* out12);
int pic_philox(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out);  /* ctr[n*4] */
int pic_set_stream(pic_ctx c, void* stream);
int pic_sync(pic_ctx c);
int pic_num_slots(pic_ctx c);
/* Serving: put a new instance into a free slot (allocating its state), or
 * free a slot.  Slots are independent; pic_step over many slots batches them. */
int pic_admit(pic_ctx c, const pic_instance_desc* d, int* slot);
int pic_retire(pic_ctx c, int slot);
int64_t pic_slot_bytes(pic_ctx c, int slot);                   /* device bytes held by a slot */
const char* pic_last_error(pic_ctx c);
void pic_destroy(pic_ctx c);
int pic_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
