/*
 * sbfem.h -- C ABI of the MI355X explicit octree-SBFEM time stepper.
 *
 * The library advances  M u'' + C u' + K u = P(t) b  with the central
 * difference method on a lumped (diagonal) mass (eq. DnMdiag, Sec. 3.3),
 * computing the internal force element by element (eq. Rinte) as
 * R_int = sum_e s_e R_e^T K_p R_e u_e, where K_p is the stiffness of the
 * unit master cell of pattern p (eq. Rintep), R_e the signed permutation that
 * maps the cell onto its master (Sec. 3.2.2), and s_e = E_e h_e (eq. KM_scale).
 *
 * Conventions shared by every call:
 *  - Every call returns sbfem_status; 0 is success.  On failure the message
 *    is available from sbfem_last_error() (per calling thread).
 *  - Pointers named "host" point to host memory; the library copies what it
 *    needs before returning and never keeps a caller pointer.  Device memory
 *    is owned by the library and released by the matching destroy call.
 *  - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *    Work is enqueued on it; read_state blocks until its copy is complete.
 *  - Calls on one mesh handle are not thread-safe; different handles are
 *    independent.  A pattern library must outlive the meshes created from it.
 *  - dof numbering is node-major: dof = 3*node + axis.
 */
#ifndef SBFEM_H
#define SBFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBFEM_OK = 0,
  SBFEM_EINVAL = -1,     /* malformed argument or mesh */
  SBFEM_ENOMEM = -2,     /* device allocation failed or over the memory budget */
  SBFEM_EDEVICE = -3,    /* a HIP runtime call failed */
  SBFEM_EUNSTABLE = -4,  /* non-finite displacement detected (time step too large) */
  SBFEM_EBUSY = -5,
  SBFEM_ENOTCONV = -6    /* an iterative solve did not reach its tolerance */
} sbfem_status;

/* Precision of the element product K_p u_e.  FP32/FP16/BF16 accumulate in FP32. */
typedef enum { SBFEM_PROD_FP64 = 0, SBFEM_PROD_FP32 = 1, SBFEM_PROD_FP16 = 2, SBFEM_PROD_BF16 = 3 } sbfem_prod;
/* Storage of the displacement history u_n, u_{n-1}. */
typedef enum { SBFEM_STATE_FP64 = 0, SBFEM_STATE_FP32 = 1, SBFEM_STATE_KAHAN32 = 2 } sbfem_state;
/*
 * Assembly of R_int:
 *  ATOMIC  element forces scattered with floating-point atomics, separate update pass;
 *  COLOUR  cells processed colour by colour (no two cells of a colour share a node),
 *          plain read-modify-write, bitwise reproducible, separate update pass;
 *  TILED   owner tiles: each block owns a run of nodes, sums the rows of every regular
 *          8-node cell touching them in on-chip memory and updates them in the same
 *          pass; the hanging-node cells are computed once each in a pass before it,
 *          whose row forces the owning blocks add (no atomics outside on-chip memory).
 */
typedef enum { SBFEM_ASM_ATOMIC = 0, SBFEM_ASM_COLOUR = 1, SBFEM_ASM_TILED = 2 } sbfem_asm;
/* Load-time function P(t) (Sec. 5, eqs. Ricker, Triangle, Lamb), or a table of P(t_n) per step
   (R_ext evaluated at t_n = n dt, Alg. 1). */
typedef enum {
  SBFEM_LOAD_RICKER = 0,
  SBFEM_LOAD_TRIANGLE = 1,
  SBFEM_LOAD_SINE_BURST = 2,
  SBFEM_LOAD_TABLE = 3
} sbfem_load_kind;

typedef struct sbfem_patterns sbfem_patterns;  /* opaque: uploaded master-cell library */
typedef struct sbfem_mesh sbfem_mesh;          /* opaque: one simulation's resident state */

/*
 * Orientation code of a cell (0..47), the signed permutation Q with
 * u_master[k][a] = s_a * u_cell[conn[k]][pi(a)]  (Sec. 3.2.2, transformation
 * of u and back-transformation of the force with Q^-1 = Q^T):
 *   code = 8*perm + signs, perm indexes pi in the order
 *   (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0), and bit a of signs set
 *   means s_a = -1.
 */

typedef struct {
  int64_t n_nodes;              /* number of nodes N (3N dofs) */
  int64_t n_cells;              /* number of cells */
  double h0;                    /* edge of a level-0 cell; h_e = h0 * 2^-level[e] */
  const int32_t* conn;          /* host: node ids per cell in master order of its pattern,
                                   concatenated in cell order; ndof(pattern)/3 entries per cell */
  const uint16_t* pattern;      /* host [n_cells]: pattern id (index into the uploaded library) */
  const uint8_t* orient;        /* host [n_cells]: orientation code, see above */
  const uint8_t* level;         /* host [n_cells]: octree level */
  const uint8_t* material;      /* host [n_cells]: material id < n_materials */
  int32_t n_materials;
  const double* E;              /* host [n_materials]: Young's modulus relative to the library's */
  const double* rho;            /* host [n_materials]: density */
  const uint8_t* fixed_dof;     /* host [3N]: 1 = Dirichlet dof (held at zero), may be NULL */
  int64_t load_nnz;             /* entries of the nodal load vector b (Gamma_N) */
  const int64_t* load_dof;      /* host [load_nnz]: dof index */
  const double* load_val;       /* host [load_nnz]: value; f_ext(t) = P(t) b */
  int32_t load_kind;            /* sbfem_load_kind */
  double load_t1, load_P0;      /* parameters t1 and P0 of P(t) */
  int32_t load_cycles;          /* cycles of the sine burst */
  double dt;                    /* time step (> 0) */
  double alpha;                 /* mass-proportional damping C = alpha M (eq. C) */
  int32_t prod;                 /* sbfem_prod */
  int32_t state;                /* sbfem_state */
  int32_t assembly;             /* sbfem_asm */
  const double* u0;             /* host [3N] initial displacement, NULL = zero */
  const double* v0;             /* host [3N] initial velocity, NULL = zero */
  /* owner-tile shape (TILED assembly); 0 = library default.  tile_nodes: nodes owned by one
     block (halved automatically until the block's on-chip memory fits); block_threads:
     threads per block of the owner-tile pass (regular 8-node cells and the update),
     block_threads_mixed per block of the hanging-node cell pass (one wave per item of up
     to 64 cells of one pattern); multiples of 64, at most 512. */
  int32_t tile_nodes;
  int32_t block_threads;
  int32_t block_threads_mixed;
  /* SBFEM_LOAD_TABLE: P(t_n) = load_table[n] for 0 <= n < load_table_n, 0 from then on
     (host [load_table_n], copied to the device by create_mesh; 8 B per entry in the
     footprint).  Ignored by the other load kinds. */
  int64_t load_table_n;
  const double* load_table;
} sbfem_mesh_desc;

/*
 * Upload the master-cell library (Table "Data structure": K_e and M_e of the
 * unique patterns, unit edge, unit modulus and density, one Poisson ratio).
 *   ndof      host [n_patterns]: 3 * nodes of each pattern (24..78)
 *   K         host: row-major ndof x ndof blocks, concatenated in pattern order
 *   m         host: lumped diagonal masses (ndof each), concatenated
 *   omega     host [n_patterns]: largest circular frequency of K phi = w^2 m phi
 * Fails with SBFEM_EINVAL for ndof outside 24..78 or not a multiple of 3, or a
 * non-positive mass.
 */
sbfem_status sbfem_upload_patterns(sbfem_patterns** out, int32_t n_patterns, const int32_t* ndof,
                                   const double* K, const double* m, const double* omega,
                                   void* hip_stream);
void sbfem_destroy_patterns(sbfem_patterns* p);

/*
 * Device bytes create_mesh allocates for this descriptor (admission control): the sum of the
 * sizes of the mesh's device buffers, from the same host set-up that create_mesh runs (so it
 * costs as much host time).  A mesh of the owner-tile assembly created without u0 allocates
 * 8 B per dof more the first time its internal force is read (read_state which = 2).
 * Errors: those of create_mesh's validation.
 */
sbfem_status sbfem_mesh_footprint(const sbfem_patterns* p, const sbfem_mesh_desc* d, int64_t* bytes);

/*
 * The same host set-up split from the upload, for callers that admit a mesh by its
 * footprint before creating it (a serving loop): sbfem_plan_mesh runs create_mesh's host
 * set-up (validation, renumbering, tiling, mass; Alg. 1 initialisation) into a host plan and
 * returns the device bytes sbfem_mesh_footprint would; sbfem_create_mesh_planned then makes
 * the mesh from the plan without repeating it.  The plan keeps the pointers p and d: both
 * must stay valid and unchanged until sbfem_create_mesh_planned returns.  A plan serves one
 * create (SBFEM_EINVAL after that) and is freed by sbfem_destroy_plan, used or not.
 * Errors: those of sbfem_create_mesh.
 */
typedef struct sbfem_plan sbfem_plan;
sbfem_status sbfem_plan_mesh(sbfem_plan** out, const sbfem_patterns* p, const sbfem_mesh_desc* d,
                             int64_t* device_bytes);
sbfem_status sbfem_create_mesh_planned(sbfem_mesh** out, sbfem_plan* plan, void* hip_stream);
void sbfem_destroy_plan(sbfem_plan* plan);

/* Smallest element limit 2/omega_max,e over the cells (eqs. tcr, tcr_scale). */
sbfem_status sbfem_critical_dt(const sbfem_patterns* p, const sbfem_mesh_desc* d, double* dt_cr);

/*
 * Build a resident simulation: validates the mesh (node ids in range, pattern
 * ids in range, orientation < 48, material < n_materials, dt > 0, every free
 * dof with positive lumped mass), sorts cells by pattern, assembles the lumped
 * diagonal mass (Alg. 1 set-up), and sets u_0 and the start-up point
 * u_-1 = u_0 - dt v_0 + dt^2/2 M^-1 (P(0) b - K u_0) - alpha dt^2/2 v_0 (eq. D0).
 * The step counter starts at 0.
 */
sbfem_status sbfem_create_mesh(sbfem_mesh** out, const sbfem_patterns* p, const sbfem_mesh_desc* d,
                               void* hip_stream);
void sbfem_destroy_mesh(sbfem_mesh* m);

/*
 * Advance n_steps central-difference steps (Alg. 1 time loop):
 *   R_int = sum_e s_e R_e^T K_p R_e u_e,  r = P(t_n) b - R_int,  t_n = n dt,
 *   u_{n+1} = (dt^2 M^-1 r + 2 u_n - (1 - alpha dt/2) u_{n-1}) / (1 + alpha dt/2).
 * Every step's update checks the values it writes; the first step whose u_{n+1} is not finite
 * (time step above the stability limit) is recorded on the device.  The call is asynchronous,
 * so that record is examined by the next call on the mesh (step_n, step_batch, read_state),
 * which then returns SBFEM_EUNSTABLE naming the step.
 */
sbfem_status sbfem_step_n(sbfem_mesh* m, int64_t n_steps, void* hip_stream);

/*
 * With steps > 0, step_n launches its steps in chunks of `steps` and, after each chunk, waits
 * for it and examines the non-finite record: a chunk that produced a non-finite u_{n+1} makes
 * that step_n return SBFEM_EUNSTABLE at once (the mesh's step is then the end of that chunk,
 * no further chunk is launched).  The call then blocks once per chunk; steps = 0 (the
 * default) restores the asynchronous behaviour above.  Errors: SBFEM_EINVAL (steps < 0).
 */
sbfem_status sbfem_set_check_interval(sbfem_mesh* m, int64_t steps);

/*
 * Advance several meshes in one stream: mesh i takes n_steps[i] steps (a mesh
 * may appear once; n_steps[i] >= 0).  Owner-tile meshes that share a pattern
 * library, product precision, state storage and block shape advance together:
 * each launch covers the tiles (and hanging-cell items) of every such mesh that
 * still has steps to take.  Other meshes are stepped in turn.  Returns after the
 * work of the batched groups has completed.  A repeated mesh or a negative count:
 * SBFEM_EINVAL, nothing stepped.
 */
sbfem_status sbfem_step_batch(sbfem_mesh* const* ms, int32_t n, const int64_t* n_steps, void* hip_stream);

/*
 * sbfem_step_batch for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same arguments, results
 * and errors as sbfem_step_batch, except:
 *  - the work lists of the batched launches (mesh refs, (mesh, tile) and (mesh, item) lists)
 *    go into a static buffer of SBFEM_NOALLOC_SCRATCH_BYTES per device, which the library
 *    holds until the process ends; nothing is allocated or freed (no hipMalloc, no graphs);
 *  - a batch whose lists exceed the buffer (24 B per mesh and 16 B per owner tile and per
 *    hanging-cell item of its largest group, 256-byte aligned parts) fails with SBFEM_EINVAL
 *    before any step is taken;
 *  - all meshes must live on one device.
 * Every call on a device shares that device's buffer, and each segment rewrites it before
 * use (nothing in it needs to start at zero); calls that overlap on one device (other
 * threads or streams) race on it.  The call returns after its work has completed, like
 * sbfem_step_batch.
 */
#define SBFEM_NOALLOC_SCRATCH_BYTES (8u << 20)
sbfem_status sbfem_step_batch_noalloc(sbfem_mesh* const* ms, int32_t n, const int64_t* n_steps, void* hip_stream);

/*
 * Step loops in HIP graphs (owner-tile assembly only; the time loop of Alg. 1
 * replayed from a captured graph instead of launched step by step).  With
 * steps > 0, step_n runs every whole chunk of `steps` steps as one replay of a
 * graph captured on first use (its launches read the step number from device
 * memory, so one graph serves every chunk); sbfem_step_batch does the same for
 * a group whose meshes all have steps > 0 (the smallest value is used), with
 * the graph and work lists of each set of active meshes cached between calls
 * (at most 16 sets; a mesh's entries go when it is destroyed or its value
 * changes).  0 (the default) launches every step.  Not used while profiling is
 * on.  Results equal those of direct launches (same kernels, same order).
 * steps outside [0, 4096], or > 0 on another assembly: SBFEM_EINVAL.
 */
sbfem_status sbfem_set_graph_steps(sbfem_mesh* m, int32_t steps);

/*
 * Copy state to host memory host_out [3N] (FP64):
 *   which = 0: u_n, 1: u_{n-1}, 2: R_int(u_n) = sum_e s_e R_e^T K_p R_e u_e (in the mesh's
 *   product precision), 3: the lumped diagonal mass M (Sec. 3.3; FP64, fixed dofs included).
 * Reduced state storage is widened to FP64 (a compensated pair as hi + lo).
 * *step (may be NULL) receives n.  Blocks until the copy has landed.
 */
sbfem_status sbfem_read_state(sbfem_mesh* m, int32_t which, double* host_out, int64_t* step,
                              void* hip_stream);

/* Replace u_n, u_{n-1} (host [3N] each) and the step counter (checkpoint restore). */
sbfem_status sbfem_write_state(sbfem_mesh* m, const double* u_n, const double* u_nm1, int64_t step,
                               void* hip_stream);

/* Device bytes held by a mesh, and the number of cells per pattern-size class (diagnostics). */
sbfem_status sbfem_mesh_info(const sbfem_mesh* m, int64_t* device_bytes, int64_t* n_dof, int32_t* n_colours);

/*
 * Probe time histories (displacement at a point, Sec. 5.2; acceleration history, Sec. 5.3):
 * from the mesh's current step on, the update of every step n records, for each of the
 * n_probes dofs (host, caller numbering), u_{n+1} and the central-difference acceleration
 * (u_{n+1} - 2 u_n + u_{n-1}) / dt^2 into row n - n_0 of a device history of `capacity` rows
 * (n_0: the step at this call); later steps are not recorded.  A dof may appear more than once.
 * n_probes = 0 removes the probes.  Device memory: 16 B per probe and row, allocated here (not
 * part of sbfem_mesh_footprint).  Owner-tile assembly only.  Waits for the stream's work.
 * Errors: SBFEM_EINVAL (bad dof, negative count or capacity, other assembly), SBFEM_ENOMEM.
 */
sbfem_status sbfem_set_probes(sbfem_mesh* m, int32_t n_probes, const int64_t* dofs, int64_t capacity,
                              void* hip_stream);

/*
 * The recorded rows: *rows = min(capacity, steps taken since sbfem_set_probes), *step0 = n_0;
 * host_u and host_a [rows][n_probes] (row-major; either may be NULL, both NULL to query the
 * count).  Blocks until the copies have landed.
 */
sbfem_status sbfem_read_probes(sbfem_mesh* m, double* host_u, double* host_a, int64_t* rows, int64_t* step0,
                               void* hip_stream);

/*
 * Lowest eigenfrequencies of the free vibration K phi = omega^2 M phi with the lumped mass
 * (Sec. 5.1): the k smallest omega over the free dofs, ascending, into host_omega [k], and the
 * relative residuals |A x - theta x| / theta of the Ritz pairs into host_resid [k] (may be NULL),
 * where A = M^-1/2 K M^-1/2 and theta = omega^2.  Chebyshev-filtered subspace iteration with
 * a block of `block` vectors (0: k + max(16, k/2)) and filters of degree `degree` (0: 20)
 * damping [largest Ritz value, max over cells of omega_max,e^2]; K is applied element by
 * element by the owner-tile pass to the whole block in one launch; Rayleigh-Ritz with the
 * block's Gram matrix every iteration.  Stops when every wanted residual is <= tol, or after
 * max_iter iterations (*iterations receives the count; may be NULL).  The eigenvalues of
 * A must be positive (Dirichlet conditions that remove the rigid modes).  Needs the owner-tile
 * assembly with FP64 products and state.  Device memory: 6 blocks of 3N x block FP64 values
 * plus the hanging-cell rows of every column, allocated for the call and freed before it returns.
 * Errors: SBFEM_EINVAL (assembly or precision, k < 1, block outside [k, min(free dofs, 512)],
 * max_iter < 1, tol <= 0), SBFEM_ENOMEM, SBFEM_EDEVICE, SBFEM_ENOTCONV (host_omega then holds
 * the last estimates).  The step state of the mesh is not touched.
 */
sbfem_status sbfem_eigen_lowest(sbfem_mesh* m, int32_t k, int32_t block, int32_t degree, int32_t max_iter, double tol,
                                double* host_omega, double* host_resid, int32_t* iterations, void* hip_stream);

/*
 * Kernel timing for diagnostics.  With profiling enabled, every kernel launch
 * of step_n / step_batch on this mesh is bracketed by HIP events recorded on
 * the launch stream.  profile_read waits for the recorded work, returns the
 * summed milliseconds and launch counts per kernel class, and clears them.
 * Classes: 0 load, 1 element kernel of 8-node cells (TILED: the owner-tile pass,
 * which also applies the update), 2 element kernel of larger cells (TILED: the
 * hanging-node cell pass), 3 central-difference update.
 */
#define SBFEM_N_KERNEL_CLASSES 4
sbfem_status sbfem_profile(sbfem_mesh* m, int32_t enable);
sbfem_status sbfem_profile_read(sbfem_mesh* m, double* ms, int64_t* launches);

/*
 * Layout statistics (diagnostics): vals[0..n_vals) receives, in order,
 *  0 owner tiles that own no node of a hanging-node cell, 1 the other owner
 *  tiles, 2 cell items of regular 8-node cells, 3 local node entries over all
 *  tiles, 4 cell entries (regular cells once per tile they touch, plus the
 *  hanging-node cells once each), 5 nodes owned per tile, 6 and 7 algorithmic
 *  bytes per step of the owner-tile pass and of the hanging-node cell pass:
 *  32 B per dof (u_n, u_{n-1}, M^-1 read, u_{n+1} written) and 16 B per load
 *  entry in the owner-tile pass (eq. DnMdiag, Alg. 1 time loop), 4 B per node id
 *  + 3 B per cell in the pass that computes the cell, 8 the largest number of
 *  local nodes of a tile, 9 the on-chip memory of an owner-tile block (bytes).
 *  Entries not available for the mesh's assembly are 0.
 */
sbfem_status sbfem_mesh_layout(const sbfem_mesh* m, int64_t* vals, int32_t n_vals);

/*
 * Device memory of objects created from now on (pattern libraries, meshes, and the work lists
 * of sbfem_step_batch) comes from alloc(bytes, user) and goes back through release(ptr, user),
 * e.g. a framework's caching allocator; both NULL restores hipMalloc/hipFree.  alloc must
 * return device memory of the current device aligned to at least 256 bytes, or NULL (the
 * creating call then fails with SBFEM_ENOMEM).  Each object keeps the pair it was created
 * with and releases through it when destroyed, so the pair must stay callable until then.
 * Process-wide setting, not synchronised with concurrent creation calls.
 * Errors: SBFEM_EINVAL if exactly one of alloc, release is NULL.
 */
sbfem_status sbfem_set_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                                 void* user);

/* Last error message of the calling thread ("" if none). */
const char* sbfem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBFEM_H */
