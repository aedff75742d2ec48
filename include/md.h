/*
 * md.h -- C ABI of the MI355X (gfx950) short-range molecular-dynamics hot path.
 *
 * The library advances periodic boxes of a binary (up to 4 species)
 * Lennard-Jones or soft-sphere mixture with velocity Verlet, following
 * Allsopp, Ruocco, Fratalocchi, arXiv:1105.5613:
 *   - pair potential Eq. (1) (Lennard-Jones) or Eq. (2) (soft sphere), each
 *     truncated in the shifted-force form Eq. (3) ("Interaction potential");
 *   - cubic cells of side >= cutoff holding many particles each, searched
 *     over neighbouring cells only (Fig. 1, "Grid-search method"); here the
 *     cells feed a full neighbour list with a skin that is rebuilt when some
 *     particle has moved more than half the skin;
 *   - velocity-Verlet time marching ("Parallel force calculation");
 *   - fixed-temperature (canonical) runs by isokinetic velocity rescaling and
 *     linear temperature ramps (scaling-results and glass sections).
 *
 * One context holds `nrep` independent replicas (a single system is
 * nrep = 1).  Replica r owns particles [off_r, off_r + n[r]) of every
 * caller array, where off_r = n[0] + ... + n[r-1].
 *
 * Conventions
 *   - Every call returns md_status: MD_OK (0) or a negative error code.
 *     md_last_error(ctx) gives a message for the last failure.
 *   - Per-particle caller arrays are in the caller's particle order
 *     ("original id" order); vectors are [Ntot][3] row-major.
 *   - Pointers documented as DEVICE must be HIP device memory (e.g. torch
 *     CUDA tensors on ROCm); HOST pointers are ordinary process memory.
 *     Arrays are borrowed for the duration of the call only.
 *   - All device work is enqueued on the hip stream given to md_init.
 *     Calls that return data to the host synchronise that stream and report
 *     device-side errors latched since the last such call.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - The context owns its device buffers (sorted state, cells, lists,
 *     partials).  md_init takes them from hipMalloc; md_init_alloc from a
 *     caller-supplied allocator (e.g. a framework's caching allocator).
 *     They are released in md_destroy.
 */
#ifndef MD_H
#define MD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx_s* md_ctx;
typedef int32_t md_status;

enum {
  MD_OK = 0,
  MD_EINVAL = -1,     /* invalid argument (shape, range, non-finite input) */
  MD_ENOMEM = -2,     /* device allocation failed */
  MD_EBOX = -3,       /* box side L < 2 (max rc + skin) */
  MD_EOVERFLOW = -4,  /* a neighbour row longer than the capacity.  md_build_cells
                         and md_step grow the capacity and finish the call
                         themselves (see there); returned only when growing
                         cannot help: the staged path's 16383 LDS slots per row
                         tile, or repeated growth within one call */
  MD_ENONFINITE = -5, /* a non-finite force or a particle that left the box by
                         more than one box length between rebuilds */
  MD_EHIP = -6,       /* a HIP runtime call failed */
  MD_ESTATE = -7      /* call order (e.g. md_forces before md_set_state) */
};

enum { MD_POT_LJ = 0, MD_POT_SOFT = 1 };
enum { MD_TRUNC_SHIFTED_FORCE = 0, MD_TRUNC_SHIFT = 1 };
enum { MD_FP64 = 0, MD_MIXED = 1 };
/* Kernel path.  GATHER: one thread group per particle gathers neighbour
 * positions from global memory; list entries are 32-bit indices with a
 * periodic-image code; works for any box.  STAGED: one block per row tile
 * of cells (about 128 home particles) copies the tile's 27-piece
 * neighbourhood, with periodic shifts applied, into LDS once per force
 * launch, and list entries are 16-bit LDS slots; needs >= 3 cells per box
 * side.  CELLS: the paper's list-free linked-cell evaluation ("Grid-search
 * method", Fig. 1): no neighbour list at all, every force launch searches
 * the 27-cell stencil of each particle (cells rebuilt by the skin rule);
 * needs >= 3 cells per box side; md_get_neighbors and md_list_stats return
 * MD_ESTATE.  AUTO is GATHER. */
enum { MD_PATH_AUTO = 0, MD_PATH_GATHER = 1, MD_PATH_STAGED = 2, MD_PATH_CELLS = 3 };
#define MD_MAXT 4

/* Physical and numerical parameters, shared by all replicas of a context. */
typedef struct {
  int32_t ntypes;     /* number of species, 1..4 */
  int32_t potential;  /* MD_POT_LJ: Eq. (1); MD_POT_SOFT: Eq. (2) */
  int32_t trunc;      /* MD_TRUNC_SHIFTED_FORCE: Eq. (3); MD_TRUNC_SHIFT: V(r)-V(rc) */
  int32_t precision;  /* MD_FP64: all FP64.  MD_MIXED: pair forces in FP32 with
                         FP32 accumulation from an FP64 displacement; positions,
                         velocities, the skin check and energy/virial totals FP64 */
  double eps[16];     /* eps[a*4+b], symmetric, a,b < ntypes */
  double sig[16];     /* sigma[a*4+b], symmetric, > 0 */
  double rc[16];      /* cutoff per species pair, > 0 */
  double mass[4];     /* mass per species, > 0 */
  double skin;        /* neighbour-list skin >= 0 (0 rebuilds every step) */
  double dt;          /* time step */
  int32_t max_neighbors; /* neighbour capacity per particle; 0 = from density */
  int32_t graph_steps;   /* steps per captured hipGraph in md_step; 0 = direct */
  int32_t tpp;           /* lanes per particle in the force kernel (1,2,4,8; staged
                            path 1,2,4); 0 = auto */
  int32_t unroll;        /* list slots gathered per pipelined chunk in the force
                            kernel (1,2,4,8); 0 = auto */
  int32_t path;          /* MD_PATH_AUTO, MD_PATH_GATHER, MD_PATH_STAGED or MD_PATH_CELLS */
  int32_t tile_cells;    /* staged path: cells per row tile (1..64); 0 = auto */
  int32_t stage_slots;   /* staged path: LDS slots per tile (>= 64); slots beyond are
                            read from global memory; 0 = auto */
  int32_t split_kick;    /* 0 = auto: in directly launched NVE steps of a one-replica
                            context on the gather path, the force launch of a step also
                            applies the next step's first half kick and drift (same
                            arithmetic and results, one pass over the particles fewer per
                            step; never on the last step of an md_step call, so the state
                            it leaves is complete); 1 = always a separate kick/drift
                            launch */
  int32_t small_box;     /* 0 = auto: a context of one box of at most 8,192 particles
                            (and 4,096 cells) rebuilds its cells in one block, and one of
                            at most 16,384 particles with >= 3 cells per side searches
                            its list (gather path) with 32 lanes per particle: the same
                            cells and lists bit for bit, with fewer launches and less
                            latency at these sizes; 1 = always the general kernels */
} md_params;

/* Per-replica observables after the last completed step. */
typedef struct {
  double ke;        /* kinetic energy 1/2 sum m v^2 (after any rescale) */
  double pe;        /* potential energy sum over pairs of V*(r) */
  double virial;    /* W = sum over pairs of r f(r), f = -d(V*)/dr */
  double T;         /* 2 ke / (3 n - 3) */
  double P;         /* (2 ke + W) / (3 V) */
  double E;         /* ke + pe */
  double max_disp;  /* largest |x - x_ref| after this step's drift (x_ref: positions at
                       the last list build), before any rebuild it triggers */
  double T_target;  /* thermostat target of the step (0 for NVE) */
  int64_t step;     /* steps taken since md_set_state */
  int64_t n_rebuild;/* list builds since md_set_state */
} md_obs;

/* Create a context for nrep replicas: n [nrep] particles (HOST, each >= 2),
 * L [nrep] cubic box sides (HOST).  hip_stream: a hipStream_t (NULL = the
 * null stream).  Fails with MD_EBOX if some L < 2 (max rc + skin).
 * The total particle count must be below 2^26 (list entries carry a 26-bit
 * index and a 6-bit periodic-image code). */
md_status md_init(md_ctx* out, const md_params* p, int32_t nrep,
                  const int64_t* n, const double* L, void* hip_stream);

/* Caller-supplied device allocator.  alloc(u, bytes, stream) returns at
 * least `bytes` bytes of device memory, aligned to 256 bytes, usable in
 * stream order on `stream` (the context's stream), or NULL on failure (the
 * call then fails with MD_ENOMEM).  free(u, ptr, stream) takes back a
 * pointer alloc returned; the library has synchronised the stream before
 * calling it, so no queued work still uses ptr.  u is passed through.  The
 * callbacks run on the thread that calls the library: in md_init_alloc,
 * when a call grows a buffer (neighbour capacity, logs, analysis scratch)
 * and in md_destroy. */
typedef struct {
  void* (*alloc)(void* u, size_t bytes, void* stream);
  void (*free)(void* u, void* ptr, void* stream);
  void* u;
} md_allocator;

/* md_init with every device buffer of the context taken from *alloc
 * (alloc = NULL: hipMalloc, as md_init).  *alloc is copied; u must stay
 * valid until md_destroy. */
md_status md_init_alloc(md_ctx* out, const md_params* p, int32_t nrep, const int64_t* n,
                        const double* L, void* hip_stream, const md_allocator* alloc);

/* Release every device buffer; ctx becomes invalid.  NULL is a no-op. */
md_status md_destroy(md_ctx ctx);

/* Message for the last failure on ctx (ctx = NULL: last md_init failure). */
const char* md_last_error(md_ctx ctx);

/* Upload a state (DEVICE pointers, original id order): x, v [Ntot][3]
 * doubles, type [Ntot] int32 in [0, ntypes).  The particle record of the
 * paper's data structure (position, velocity, species; "Grid-search
 * method").  Positions must lie in [-L, 2L) per coordinate.  Resets step and
 * rebuild counters and image counters; the next md_build_cells / md_forces /
 * md_step rebuilds.  The arrays are copied; the caller keeps ownership.
 * Errors: MD_EINVAL for a NULL array or a species outside [0, ntypes),
 * MD_ENONFINITE for a non-finite value (this call synchronises). */
md_status md_set_state(md_ctx ctx, const double* x, const double* v,
                       const int32_t* type);

/* Download the state (DEVICE pointers, original id order, any may be NULL):
 * x [Ntot][3] positions as stored (wrapped into the periodic box at the last
 * list build, "Grid-search method", and drifted since), v [Ntot][3], img
 * [Ntot][3] int32 periodic image counters (unwrapped position = x + img * L,
 * the displacement behind the glass section's mean-squared displacement).
 * The caller owns the buffers.  Synchronises; MD_ESTATE before a state is
 * set; reports errors latched by earlier asynchronous calls. */
md_status md_get_state(md_ctx ctx, double* x, double* v, int32_t* img);

/* The grid search ("Grid-search method", Fig. 1): wrap positions into
 * [0, L), bin them into cubic cells of side L/nc >= max rc + skin with
 * nc = floor(L / (max rc + skin)) (nc < 3 -> one cell), order particles by
 * (cell, original id) and build the full neighbour list: j is listed for i
 * iff r_ij^2 < (rc_ab + skin)^2 over the 27-cell stencil (the skin, the
 * list and its reuse between builds are this library's, not the paper's).
 * Synchronises; when a row overflows the capacity it grows the capacity and
 * rebuilds once (MD_EOVERFLOW only when that cannot help). */
md_status md_build_cells(md_ctx ctx);

/* Evaluate forces, potential energy and virial on the current state
 * (building the list first when needed): the truncated pair potential of
 * Eq. (1) or Eq. (2) in the shifted-force form Eq. (3) ("Interaction
 * potential"), F_i = sum_j f(r_ij) (x_i - x_j) / r_ij over the pairs within
 * rc_ab.  Forces stay in the context (md_get_forces).  Asynchronous;
 * MD_ESTATE before a state is set. */
md_status md_forces(md_ctx ctx);

/* Copy the forces of the last md_forces / md_step (Eq. (3) summed over the
 * pairs, "Interaction potential") to F (DEVICE pointer, caller-owned,
 * original id order, [Ntot][3]) as doubles (MD_FP64) or floats
 * (MD_MIXED).  Synchronises; MD_ESTATE before any force evaluation. */
md_status md_get_forces(md_ctx ctx, void* F);

/* Advance every replica by nsteps velocity-Verlet steps of length dt
 * ("Parallel force calculation": half kick, drift, forces, half kick), with
 * the cells and lists rebuilt whenever some particle of a replica moved more
 * than skin/2 since its last build.
 * T0, T1: HOST [nrep] thermostat targets or NULL for NVE; the k-th step of
 * this call (k = 1..nsteps) rescales velocities to
 * T_target = T0 + (T1 - T0) min(k / ramp_steps, 1)  (ramp_steps <= 0: T0):
 * the canonical runs of the scaling section and the linear cooling ramp of
 * the glass section, by isokinetic rescaling (the paper names no mechanism).
 * log: HOST [nsteps / log_every][nrep] observables of every log_every-th
 * step, or NULL.  Synchronises at the end and reports latched errors.
 * Capacity overflow: a rebuild whose longest row exceeds the neighbour
 * capacity halts the steps queued after it; this call then grows the
 * capacity, rebuilds that step's lists on its state and finishes the call,
 * so the result is the one a context with enough capacity computes (bit for
 * bit).  If growing cannot help, MD_EOVERFLOW is returned with the state of
 * the interrupted step (drifted and re-sorted, forces not yet evaluated).
 * Forces, kinetic energy and T are formed every step; the pair sums behind
 * pe, virial, P and E only on the logged steps and the last step of the
 * call (inside a hipGraph chunk: also its last step, and every step when
 * log_every does not divide graph_steps), so the observables after md_step
 * and every log record are complete. */
md_status md_step(md_ctx ctx, int32_t nsteps, const double* T0,
                  const double* T1, int64_t ramp_steps, md_obs* log,
                  int32_t log_every);

/* Observables of every replica (HOST [nrep], caller-owned): kinetic and
 * potential energy, virial, temperature, pressure and total energy (the
 * per-rank quantities the paper reduces globally, "Parallel force
 * calculation"; the potential energy of the glass section's caloric curve).
 * Synchronises and reports errors latched by earlier asynchronous calls. */
md_status md_observables(md_ctx ctx, md_obs* out);

/* Parity hook, HOST pointers: cell_start [nc^3 + 1] (offsets local to the
 * replica) and order_ids [n] (replica-local original ids in cell order) of
 * replica rep as built by the last list build.  Synchronises. */
md_status md_get_cells(md_ctx ctx, int32_t rep, int32_t* cell_start,
                       int32_t* order_ids);

/* Parity hook, HOST pointers: for each particle of replica rep (local
 * original id order) count [n] and up to cap neighbour ids [n][cap]
 * (replica-local original ids, list order unspecified).  Synchronises. */
md_status md_get_neighbors(md_ctx ctx, int32_t rep, int32_t* count,
                           int32_t* ids, int32_t cap);

/* Geometry of replica rep: cells per side, 1/cell side, particle count and
 * offset, and the neighbour capacity in use. */
md_status md_replica_info(md_ctx ctx, int32_t rep, int32_t* nc, double* inv_cell,
                          int64_t* n, int64_t* offset, int32_t* max_neighbors);

/* Kernel timing (not part of the method; for roofline measurement).
 * md_profile(ctx, every): from now on, in md_step the force kernel launch of
 * every `every`-th step (0 = off) is bracketed by two hipEvents recorded on
 * the context stream; earlier records are discarded.  While profiling is on,
 * md_step launches every step directly (graph_steps is ignored: events
 * recorded by a replayed graph cannot be timed).
 * md_profile_read: synchronises and returns the number of bracketed force
 * launches and their summed duration in milliseconds. */
typedef struct {
  int64_t force_launches;
  double force_ms;
} md_prof;
md_status md_profile(md_ctx ctx, int32_t every);
md_status md_profile_read(md_ctx ctx, md_prof* out);

/* Autotuner: times every force-kernel variant of the context's path (lanes
 * per particle x unroll) on
 * the current state, `reps` launches each, with hipEvents on the context
 * stream, keeps the fastest and recomputes forces and observables with it.
 * Positions and velocities are not changed.  Synchronises. */
typedef struct {
  int32_t tpp, unroll;   /* chosen variant */
  double force_ms;       /* its mean force-kernel time */
  int32_t ntried;
  int32_t tried_tpp[16], tried_unroll[16];
  double tried_ms[16];
} md_tune;
md_status md_autotune(md_ctx ctx, int32_t reps, md_tune* out);

/* Mean-squared displacement (glass section observables).  md_msd_reference
 * stores the current unwrapped positions x + img L as the reference;
 * md_msd returns, per replica (HOST [nrep]), the mean over its particles of
 * |u - u_ref|^2.  md_msd fails with MD_ESTATE before a reference is set.
 * Synchronises. */
md_status md_msd_reference(md_ctx ctx);
md_status md_msd(md_ctx ctx, double* out);

/* Radial distribution function of replica rep (glass section):
 * g[b] = 2V/N^2 * (number of pairs i < j with b dr <= r_ij < (b+1) dr) / shell
 * volume of bin b, dr = rmax / nbins, minimum image, exact FP64 distances.
 * With rmax <= cell side - skin (and >= 3 cells per side) the pairs come
 * from the cell grid (any replica size; builds the cells first if needed);
 * otherwise all pairs are visited and the replica may hold at most 262144
 * particles.  rmax <= L/2, nbins <= 8192.  g HOST [nbins].  Synchronises. */
md_status md_rdf(md_ctx ctx, int32_t rep, double rmax, int32_t nbins, double* g);

/* md_rdf for callers that cannot allocate device memory (tight serving or
 * analysis loops, harnesses that forbid hipMalloc): the same g(r), bit for
 * bit, with the pair histogram in a fixed 64 KiB device array (8192 64-bit
 * counters) that each GPU holds for the life of the process instead of a
 * buffer allocated per call.  Allocates nothing and builds nothing: the
 * cell sweep (rmax <= cell side - skin) needs cells built by an earlier
 * md_build_cells / md_forces / md_step, else MD_ESTATE.  nbins > 8192 ->
 * MD_EINVAL.  Every call on one GPU shares that array and clears it first,
 * so calls that overlap on the same GPU (other host threads, other
 * contexts' streams) race and must be serialised by the caller.
 * Synchronises, so it cannot itself be captured in a graph. */
md_status md_rdf_static(md_ctx ctx, int32_t rep, double rmax, int32_t nbins, double* g);

/* Neighbour-list statistics of replica rep (rep = -1: all replicas) at the
 * last list build: mean and maximum entries per particle.  Synchronises. */
md_status md_list_stats(md_ctx ctx, int32_t rep, double* mean, int32_t* max);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
