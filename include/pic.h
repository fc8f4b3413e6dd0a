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
 * The Poisson solves (1D: the exact solution of the node system by the
 * closed-form inverse of the tridiagonal operator, integer prefix sums
 * rounded once; 2D: FP64 cell-centred finite volumes
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
 *  - Capacity (Sec. 4.3: ionization multiplies the particles
 *    exponentially).  A step of an ionizing instance starts only with room
 *    for its worst case of births (every electron alive ionizing once); a
 *    step without that room is not run, so the instance stays at its last
 *    committed step.  pic_step then grows the buffers on the host and goes
 *    on from there: the draws depend only on (particle id, step), so the
 *    result is bit-identical to a run that never stopped.  When the room
 *    cannot be made (the slot's memory limit, the 4 GiB per-array limit,
 *    device memory, u32 particle ids), pic_step returns PIC_E_CAPACITY (or
 *    PIC_E_NOMEM) with every slot at its last committed step
 *    (pic_step_index tells which); the caller may free memory or raise the
 *    limit and call again with step0 = -1 for the remaining steps.
 *    PIC_E_STATE marks a slot whose device-side overflow guard fired
 *    anyway (not expected: the room check rules it out).
 *  - Failed slots.  A call that fails part-way through changing a slot's
 *    device tables (pic_adapt for lack of device memory, or any runtime
 *    error in pic_adapt or pic_particles_load) marks the slot failed; so
 *    does the overflow guard above.  Every later call on a failed slot
 *    returns PIC_E_STATE, except pic_count, pic_next_id, pic_step_index,
 *    pic_nleaves, pic_nq, pic_slot_bytes and pic_retire; the context's other
 *    slots are unaffected.  Device memory running out in pic_step,
 *    pic_particles_load or pic_field_solve leaves the slot usable (see
 *    above and below).
 *  - Launch checks: with PIC_CHECK_LAUNCHES=1 in the environment, every
 *    kernel-side view of a slot is checked on the host against the slot's
 *    live device blocks before it is used (each array inside one block with
 *    the extent its count implies; particle arrays below 4 GiB); a failed
 *    check returns PIC_E_STATE instead of launching.
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 4

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
/* On the quadtree: NGP scatter to the leaves with bilinear gather of nodal E
 * (PIC_FIELD_CIC_EM, the default, Sec. 3), or the cloud-in-cell on the
 * quadtree (Sec. 3.1, Fig. 2): a particle's square cloud of its leaf's size
 * covers its leaf and the direct and diagonal neighbours on its side, through
 * ghost cells at +-1 level where the neighbours differ in level (a ghost cell
 * inside a coarser leaf belongs to it, one over finer leaves is shared by
 * area, one outside the domain folds back), with the same shape function for
 * the scatter (charge in fixed point, F/2 bits per axis: exactly conserved)
 * and for the gather of the cell-centred E (the mean of each leaf's nodal E,
 * or PIC_CELL_E_2D). */
enum { PIC_FIELD_CIC_AMR = 2 };
/* 1D only: the direct implicit step (Sec. 3, the D1 scheme; the Poisson
 * solve carries the implicit susceptibility).  Each particle keeps b =
 * (dt/2) abar, abar its time-filtered acceleration (set by
 * pic_leapfrog_start to (dt/2) a(x_0), zero at load and at birth).  A step:
 *   predictor  v~ = v + b, x~ = x + dt v~ (wall rule);
 *   field      -d/dx[(1 + chi) dphi/dx] = rho~/eps0 with phi(0) = the next
 *              drive value, phi(L) = 0; rho~ and chi = sum_s (q_s/m_s)
 *              (dt^2/2) rho~_s/eps0 from the CIC charge of the predicted
 *              positions (a wall node's charge over its half cell), face
 *              coefficients 1 + (chi_i + chi_i+1)/2, solved by forward
 *              elimination and back substitution in FP64; node E as for
 *              PIC_FIELD_CIC_EM;
 *   corrector  dv = (q dt / 2m) E_n+1(x~): v = v~ + dv, x = x~ + dt dv,
 *              b = (b + dv)/2 (wall rule), then collisions, births and
 *              the deposit.
 * Such a slot steps only with solve_field set (the field is part of the
 * step) and not in batched or no-allocation calls. */
enum { PIC_FIELD_DIPIC = 3 };
enum { PIC_FP32 = 32, PIC_FP64 = 64 };
/* field kinds for pic_field_set (Sec. 3: potential at cell centres or nodes,
 * E at the nodes for the gather) */
enum {
  PIC_NODE_E_1D = 0,     /* double[ncells+1]: E at the nodes, V/m (momentum-conserving slots only) */
  PIC_NODE_PHI_1D = 1,   /* double[ncells+1]: potential at the nodes, V      */
  PIC_CORNER_PHI_2D = 2, /* double[nleaves][4]: potential at leaf corners     */
  PIC_CORNER_E_2D = 3,   /* double[nleaves][4][2]: nodal E at leaf corners    */
  PIC_CELL_PHI_2D = 4,   /* double[nleaves]: cell-centre potential            */
  PIC_CELL_E_1D = 5,     /* double[ncells]: E of each cell, V/m (energy-conserving slots only) */
  PIC_CELL_E_2D = 6,     /* double[nleaves][2]: cell-centred E, V/m (cloud-in-cell slots only) */
  PIC_CORNER_PHI_3D = 7, /* double[nleaves][8]: potential at octree leaf corners, V */
  PIC_CORNER_E_3D = 8    /* double[nleaves][8][3]: nodal E at octree leaf corners, V/m */
};
/* corner order of a quadtree leaf: 0 = (x0,y0), 1 = (x1,y0), 2 = (x0,y1),
 * 3 = (x1,y1); of an octree leaf: c = a + 2b + 4e with a, b, e in {0, 1} the
 * lower / upper side along x, y, z.  On the octree (Sec. 3.1 quad/octree,
 * cubic cells) the nodal E of a node is the mean, over the leaves having it
 * as a corner, of their trilinear-potential gradients there (taken in octant
 * order: below the node in x first, then y, then z), the gather is the
 * trilinear interpolation of the leaf's corner E and the deposit is NGP to
 * the leaf. */

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
  int dim;              /* 1 (uniform mesh), 2 (quadtree) or 3 (static octree:
                           field given at the nodes; no pic_adapt, no
                           pic_field_solve, no batched steps)                 */
  int precision;        /* PIC_FP32 or PIC_FP64: particle arithmetic             */
  double length;        /* m: 1D gap, or side of the 2D square                   */
  double dt;            /* s                                                      */
  int ncells;           /* 1D: uniform cells (2 .. 1<<20)                        */
  int min_level, max_level, base_level;   /* 2D levels, 0 .. 14; 3D, 0 .. 10   */
  int refine_disk;      /* 2D / 3D: refine leaves whose closed box meets the
                           disk / ball ...                                      */
  double disk_cx, disk_cy, disk_r;        /* ... (normalised centre, radius;
                                             3D: centre z in disk_cz)          */
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
  int64_t capacity[2];  /* particle slots per species at load: this many (at
                           least the loaded count, rounded up to 256), or 0 =
                           3x the loaded count + 4096 when ionizing, else the
                           count; pic_step grows them as births need room     */
  int field_scheme;     /* 1D: PIC_FIELD_CIC_EM or PIC_FIELD_CIC_EC; 2D:
                           PIC_FIELD_CIC_EM (NGP deposit, bilinear gather) or
                           PIC_FIELD_CIC_AMR (cloud-in-cell on the tree)       */
  /* 2D explicit tree (Sec. 3.1: cell-based quadtree; nleaves > 0 selects it,
     base_level and the disk refinement are then ignored): leaf_keys[nleaves]
     the Morton code of each leaf's low corner in 16-bit units (x in the even
     bits), leaf_levels[nleaves] its level, in Morton order.  The leaves must
     tile the square, lie within [min_level, max_level] and be 2:1 balanced
     across faces and corners (ghost cells at +-1 level, Sec. 3.1), else
     PIC_E_ARG.  Host arrays, read only during the call that builds the slot. */
  const uint32_t* leaf_keys;
  const uint8_t* leaf_levels;
  int64_t nleaves;
  double disk_cz;       /* 3D: normalised z of the refined ball's centre        */
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
  int64_t room_stops;           /* times a slot stopped for want of room and was grown   */
} pic_step_stats;

typedef struct {
  int64_t step0;        /* global index of the first step (Philox counter word 1); */
                        /* < 0: every slot continues from its own step index      */
  int nsteps;
  int solve_field;      /* 1D: after each step solve Poisson on the device with   */
  const double* v_next; /* ... phi(0) = v_next[k*ninst_sel + j] for step k, slot j */
                        /* (a direct implicit slot solves within the step, at the */
                        /* same drive value, and needs both)                        */
  int sort_every;       /* re-sort particles by cell every n steps (0 = never; 1D: by bins of cells) */
  int batched;          /* 0: launches per slot; > 0: one persistent launch over   */
                        /* all selected slots of one dimension and precision, with */
                        /* this many particles per work item (1 = 4096); quadtree  */
                        /* slots with the cloud-in-cell coupling, octree slots and */
                        /* direct implicit slots are refused (PIC_E_ARG)           */
  int grid;             /* workgroups of the particle kernel: persistent grid of the
                           batched launch (0 = 2048), or grid of the per-slot launch
                           (0 = one workgroup per 256 particles, at most 2048);
                           at most 8192                                         */
  int graph_steps;      /* batched only: capture this many steps into a HIP graph  */
                        /* and replay it (0 = no graph)                            */
  const int* slots;     /* selected slots (NULL = all live slots)                 */
  int nslots;
  int timing;           /* 0: no events; n > 0: time the particle loop of every    */
                        /* n-th step of the call (per-slot launches: the step       */
                        /* kernel's own start and end, or to after the births      */
                        /* kernels when they follow; direct implicit: predictor to */
                        /* births; batched launches: every step, around the launch */
                        /* and its births kernels), and the whole call.  PIC_E_ARG */
                        /* if negative.                                             */
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

/* ---- the five calls of the particle loop ---- */

/* Build a context holding ninst >= 0 instances (slots 0..ninst-1; more can be
 * admitted later with pic_admit).  Mesh (Sec. 3.1: one cell-based grid for
 * particle movement, collisions and output): a uniform 1D mesh of ncells, or
 * a quadtree uniform at base_level with optional disk refinement and 2:1
 * balance across faces and corners (ghost cells at +-1 level for direct and
 * diagonal neighbours, Sec. 3.1), or an explicit tree (leaf_keys).
 * descs[ninst] are host structs, read during the call.  'stream' is a
 * hipStream_t (NULL = default stream).  On success *out owns all device
 * state (free it with pic_destroy).  Errors: PIC_E_ARG for an invalid
 * descriptor (levels, explicit tree, species), PIC_E_NOMEM, PIC_E_HIP. */
int pic_mesh_build(const pic_instance_desc* descs, int ninst, void* stream, pic_ctx* out);

/* Replace the particles of one species of one slot (Sec. 3: super-particles
 * of the species; Sec. 3.1: each is kept in the leaf that contains it) with
 * n host particles: s[n*dim] normalised positions in [0,1), v[n*3] m/s, w[n]
 * (NULL: 2^16 each, i.e. w0 real particles), id[n] (NULL: 0..n-1).  Values
 * are rounded to the slot's precision; the arrays are copied.  PIC_E_ARG if
 * a position is outside [0,1) or a weight is 0.  PIC_E_NOMEM (the room is
 * allocated before the old particles are touched) leaves the slot as it
 * was. */
int pic_particles_load(pic_ctx c, int slot, int species, int64_t n, const double* s, const double* v,
                       const uint32_t* w, const uint32_t* id);

/* Advance nsteps steps of the selected slots (Sec. 3 explicit PIC with MCC,
 * Sec. 3.1 particle tracking on the tree, Sec. 4.3 ionization births): per
 * particle gather E, leapfrog push, wall rule, locate the cell, null-
 * collision MCC with births, deposit to the charge sums.  a (host struct,
 * read during the call) selects slots, launch shape, field solve and
 * timing; stats (nullable) receives counts summed over the slots.  Capacity
 * as in the conventions above (PIC_E_CAPACITY / PIC_E_NOMEM leave every
 * slot at its last committed step).  PIC_E_ARG for bad arguments,
 * PIC_E_STATE for a slot without particles or in an error state. */
int pic_step(pic_ctx c, const pic_step_args* a, pic_step_stats* stats);

/* Deposit the current particles (Sec. 3: CIC to the nodes of the uniform 1D
 * mesh, NGP to the leaf cells of the quadtree; Sec. 3.1: the cloud-in-cell on
 * the quadtree, and no per-level volume weighting) and copy out, each
 * nullable:
 *   q_out[2][nq]  per-species integer charge sums, in weight units (NGP:
 *                 w_units; 1D and the 2D cloud: w_units * 2^F, F = 24 FP32,
 *                 32 FP64);
 *   rho_out[nq]   charge density, C/m^3: sum over species of
 *                 q w0 2^-16 (2^-F with a cloud) sums over dx (1D, per unit
 *                 area) or over h^2 depth_z (2D, h the leaf side).
 * nq = pic_nq (nodes in 1D, leaves in 2D); host buffers of the caller. */
int pic_deposit(pic_ctx c, int slot, uint64_t* q_out, double* rho_out);

/* Adapt the quadtree of a 2D slot to the particle count (Sec. 3.1: cells
 * refined and coarsened, particles reassigned by position; Sec. 4.3: AMR
 * keeps particles per cell steady, splitting 1 -> 4 and merging as the
 * fallback): coarsen sibling groups holding at most n_hi with a child below
 * n_lo (and no touching leaf two levels finer), refine leaves above n_hi
 * (repeatedly), 2:1 balance, reassign particles, split particles 1 -> 4 in
 * leaves below n_lo, merge pairs in leaves above n_hi at max_level.  Ends
 * with a fresh deposit.  s (nullable) receives what was done.  PIC_E_ARG for
 * a 1D slot; PIC_E_CAPACITY, after a complete adaptation, if split copies
 * would exhaust the u32 ids or the per-array limit (the particles are then
 * not split) or a leaf at max_level holds more particles than one merge
 * round sorts (that leaf is not merged); PIC_E_NOMEM marks the slot failed
 * (the conventions above). */
int pic_adapt(pic_ctx c, int slot, const pic_adapt_args* a, pic_adapt_stats* s);

/* For callers that cannot allocate device memory (code between graph
 * captures, tight serving loops, harnesses that forbid allocation): pic_step
 * without any device allocation.  Batched launches only (a->batched > 0,
 * graph_steps = 0, timing = 0; else PIC_E_ARG).  Its launch tables (work
 * items, instance table, per-item partial statistics, sort jobs, drive
 * tables) live in a 16 MiB device workspace of the library, one per device,
 * held until the process ends; a call whose tables do not fit returns
 * PIC_E_ARG before any step runs.  It never grows particle buffers: when a
 * step needs more room it returns PIC_E_CAPACITY with every slot at its last
 * committed step (pic_step grows them).  The workspace is shared by every
 * call on the device and keeps the last call's contents: calls that overlap
 * on one device (two threads, two streams) race and must not be made.
 * Results equal pic_step's with the same arguments. */
int pic_step_noalloc(pic_ctx c, const pic_step_args* a, pic_step_stats* stats);

/* ---- field feed (Sec. 3: Poisson for the potential, E at the nodes) ---- */

/* Set the field table the gather reads, from host data of the given kind
 * (PIC_* field kinds above; the sizes are stated there).  2D nodal E is the
 * mean, over the leaves having the node as a corner, of their corner
 * gradients (Sec. 3: bilinear gather from nodal E).  PIC_E_ARG for a kind
 * that does not fit the slot (dimension or 1D coupling). */
int pic_field_set(pic_ctx c, int slot, int kind, const double* data);

/* Poisson from the latest deposit (Sec. 3, potential at cell centres; the
 * paper's multigrid is replaced by direct / CG solves in FP64).  1D: exact
 * solution of the node system with phi(0) = phi_left, phi(L) = 0; outputs phi_out/e_out[ncells+1]
 * (nullable).  2D: cell-centred finite volumes, two-point fluxes, Jacobi CG
 * from phi_init[nleaves] (nullable: the slot's last solution) to rtol, at
 * most maxit iterations; phi_out[nleaves], e_out[nleaves*8] corner E
 * (nullable); iters, relres nullable.  Either sets the gather table.
 * PIC_E_NUMERIC if CG did not reach rtol; PIC_E_STATE if the tree is not
 * 2:1 balanced. */
int pic_field_solve(pic_ctx c, int slot, double phi_left, const double* phi_init, double rtol, int maxit,
                    double* phi_out, double* e_out, int* iters, double* relres);

/* v <- v - (q dt / 2m) E(x) for every particle of the slot: start the
 * leapfrog from the current field table (Sec. 3, explicit PIC). */
int pic_leapfrog_start(pic_ctx c, int slot);

/* Copy the latest per-species integer charge sums to q_out[2][nq] (host,
 * not NULL) without depositing again (Sec. 3 charge assignment): after
 * pic_step, the sums the last step's particle loop accumulated (its
 * survivors and births); after pic_deposit or pic_adapt, theirs.  Units as
 * pic_deposit.  PIC_E_ARG if q_out is NULL. */
int pic_deposit_read(pic_ctx c, int slot, uint64_t* q_out);

/* ---- configuration ---- */

/* Route the particle, mesh, field and adaptation-scratch memory of a context
 * through 'a' (NULL: hipMalloc with the library's own block cache).  Only on
 * a context that holds no instance yet (build with ninst = 0, then
 * pic_admit): else PIC_E_STATE.  The allocator must outlive the context.
 * (Infrastructure; no passage of the paper.) */
int pic_set_allocator(pic_ctx c, const pic_allocator* a);

/* How a slot ranks the staged births of a step by parent id (Sec. 4.3
 * births; the ranks fix the newborn ids): 0 (default) pairwise while recent
 * steps had up to 16384 births each, binned above; 1 always pairwise
 * (work ~ births^2); 2 always binned (parent ids grouped in 4096 id bins,
 * work ~ births x births per bin).  Both give the same ranks.  PIC_E_ARG for
 * another method. */
int pic_set_births_ranking(pic_ctx c, int slot, int method);

/* Device bytes the slot may hold once its particle and births buffers grow
 * (Sec. 4.3: exponential growth of the particle count; serving admits jobs
 * by projected memory).  0 = no limit.  Growth that would pass the limit
 * returns PIC_E_CAPACITY from pic_step with the slot at its last committed
 * step.  PIC_E_ARG if negative. */
int pic_set_slot_limit(pic_ctx c, int slot, int64_t max_bytes);

/* Serving: put a new instance into a free slot (allocating its state, as
 * pic_mesh_build does for one descriptor), or free a slot.  Slots are
 * independent; pic_step over many slots batches them.  *slot receives the
 * slot index.  (Infrastructure around the method; no passage of the paper.) */
int pic_admit(pic_ctx c, const pic_instance_desc* d, int* slot);
int pic_retire(pic_ctx c, int slot);

/* Make all later work of the context go to another hipStream_t (after
 * finishing the queued work); pic_sync waits for the context's stream. */
int pic_set_stream(pic_ctx c, void* stream);
int pic_sync(pic_ctx c);

/* ---- readers and helpers (host buffers of the caller, sizes as stated) ---- */

/* live particles of a species (Sec. 3 super-particles), or < 0 on error */
int64_t pic_count(pic_ctx c, int slot, int species);
/* next particle id the slot hands to births and split copies (Sec. 4.3); 0 on error */
uint32_t pic_next_id(pic_ctx c, int slot);
/* global index of the slot's next step (its last committed step + 1), or < 0 */
int64_t pic_step_index(pic_ctx c, int slot);
/* one species sorted by id: s[n*dim], v[n*3], w[n], id[n], cell[n] (all
 * nullable; n = pic_count); cell = leaf index (2D, Sec. 3.1) or 1D cell */
int pic_particles_read(pic_ctx c, int slot, int species, double* s, double* v, uint32_t* w, uint32_t* id,
                       uint32_t* cell);
/* quadtree leaves (Sec. 3.1): count, then keys[n] / levels[n] in Morton order */
int64_t pic_nleaves(pic_ctx c, int slot);
int pic_leaves_read(pic_ctx c, int slot, uint32_t* keys, uint8_t* levels);
/* entries of the charge sums and densities: nodes (1D) or leaves (2D) */
int64_t pic_nq(pic_ctx c, int slot);
/* the gather table as double: 1D [ncells+1] node E (cell E for energy-
 * conserving slots, last entry 0); 2D [nleaves][4][2] corner E (Sec. 3), or
 * [nleaves][2] cell E for cloud-in-cell slots (Sec. 3.1) */
int pic_field_read(pic_ctx c, int slot, double* out);
/* the field E the step's gather gives at n points s[n*dim] (normalised, in
 * [0,1)): out[n*dim], V/m (Sec. 3 / 3.1 gather); PIC_E_ARG for a point outside */
int pic_gather(pic_ctx c, int slot, int64_t n, const double* s, double* out);
/* drop holes and order the particles by cell (Sec. 3.1 cell-based lists; in
 * 1D by bins of consecutive cells, at most 64 bins; the results of later
 * steps do not depend on it) */
int pic_sort(pic_ctx c, int slot);
/* leaf[n] containing each point s[n*2] in [0,1)^2 (Sec. 3.1 location on the
 * tree); PIC_E_ARG for a point outside */
int pic_locate(pic_ctx c, int slot, int64_t n, const double* s, uint32_t* leaf);
/* the slot's derived per-species constants out12[12], rounded to its
 * precision: q dt/m, dt/L, candidate threshold, a_el, a_iz, v_iz^2, 2m/M,
 * v_max^2, gas thermal speed, a_cx, g_max, q dt/2m (Sec. 3 MCC) */
int pic_derived(pic_ctx c, int slot, int species, double* out12);
/* Philox4x32-10 blocks (the counter-based generator behind the MCC draws):
 * out[n*4] for counters ctr[n*4] under key[2] */
int pic_philox(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out);
int pic_num_slots(pic_ctx c);
int64_t pic_slot_bytes(pic_ctx c, int slot);                   /* device bytes held by a slot */
const char* pic_last_error(pic_ctx c);                         /* NULL ctx: this thread's last error */
void pic_destroy(pic_ctx c);
int pic_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
