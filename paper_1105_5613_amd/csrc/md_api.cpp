// md_api.cpp -- the C ABI declared in include/md.h: validation, derived
// constants, device buffers, the per-step launch sequence and error latch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "md_internal.h"
#include "stage.h"

using namespace mdk;

// Pair-distance histogram of md_rdf_static: a fixed device array, so that
// call allocates nothing.  Every GPU the library runs on holds its own copy
// (64 KiB) until the process ends; host code addresses it only through the
// per-device pointer hipGetSymbolAddress returns (scratch_dev).
constexpr int32_t kStaticBins = 8192;
static __device__ __align__(256) unsigned long long scratch[kStaticBins];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_dev[kMaxDevices] = {};

// Look up this device's copy of scratch once (the device must be current).
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[dev] = (unsigned long long*)ptr;
  return hipSuccess;
}

unsigned long long* scratch_dev(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev >= 0 && dev < kMaxDevices ? g_scratch_dev[dev] : nullptr;
}
}  // namespace

struct md_ctx_s {
  md_params p{};
  int32_t device = 0;  // the device current at md_init
  int32_t nrep = 0, ntot = 0, stride = 0, ncells = 0, ntiles = 0, cap = 0, tpp = 1, unroll = 4;
  int32_t mixed = 0;
  // staged path (row tiles with LDS-staged neighbourhoods)
  int32_t staged = 0, nrt = 0, lcap_f = 0;
  int32_t cells = 0;  // list-free cell path (row tiles, no neighbour list)
  int32_t any_single = 0, any_multi = 0;  // replicas with one cell / with >= 3 per side
  bool small_chain = false;  // one small replica: the one-block rebuild chain
  bool small_list = false;   // ... and the 32-lanes-per-particle list build
  std::vector<RowTile> rtiles_h;
  RowTile* rtiles = nullptr;
  uint16_t* nbr16 = nullptr;
  int32_t* cell_tile = nullptr;  // staged path: row tile of each cell
  hipStream_t stream = nullptr;
  std::vector<RepDesc> reps_h;
  std::vector<Tile> tiles_h;
  // device buffers
  RepDesc* reps = nullptr;
  Tile* tiles = nullptr;
  PairTab* tab = nullptr;
  int32_t thr_form = 4;  // form of the list thresholds in the neighbour search (fma_pair_form)
  int32_t rc2_form = 4;  // form of the force cutoffs on the list-free path
  int32_t nmax_rep = 0;  // particles of the largest replica
  DevState* st = nullptr;
  int32_t *cell_rep = nullptr, *counts = nullptr, *cell_start = nullptr, *bsum = nullptr;
  int32_t *cell_of = nullptr, *slot = nullptr, *tmp_src = nullptr;
  double4 *pos = nullptr, *pos_tmp = nullptr;
  int4* pos16 = nullptr;  // mixed form, gather path: cell-relative FP32 records
  double *vel = nullptr, *vel_tmp = nullptr, *xref = nullptr;
  void* frc = nullptr;
  int32_t *id = nullptr, *id_tmp = nullptr, *img = nullptr;
  uint32_t* nbr = nullptr;
  int32_t* ncount = nullptr;
  double* part = nullptr;
  int32_t* rebuild = nullptr;
  double* dmax = nullptr;   // [ntiles] per-tile max of the last drift
  // fused NVE steps (force mode 2): the drifted positions go to the other
  // buffer of a pair, pos <-> pos_tmp (pos_tmp is scratch of the rebuild
  // chain otherwise) and pos16 <-> pos16_alt; dpend [nrep] holds the drift
  // maximum measured for the next step
  int4* pos16_alt = nullptr;
  double* dpend = nullptr;
  // two-level reduction of the force partials (large replicas only)
  std::vector<RedChunk> chunks_h;
  RedChunk* chunks = nullptr;
  int32_t nchunks = 0, max_chunks = 0;
  double* part2 = nullptr;
  md_obs* obs = nullptr;
  int64_t* kcall = nullptr;
  double* lam = nullptr;
  double* therm = nullptr;  // T0 [nrep], T1 [nrep]
  double* u0 = nullptr;     // MSD reference, original id order [N][3]
  double* msd_part = nullptr;
  double* msd_out = nullptr;
  md_obs* log_dev = nullptr;
  int64_t log_cap = 0;
  std::vector<void*> owned;
  md_allocator alloc{};  // alloc.alloc == nullptr: hipMalloc / hipFree
  // captured K-step graphs (md_params.graph_steps)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t gkey[15] = {0};
  int32_t prof_epoch = 0;
  // force-kernel timing
  int32_t prof_every = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  bool has_state = false, built = false, forces_valid = false;
  std::string err;
};

namespace {

std::string g_init_error;

md_status fail(md_ctx c, md_status code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_init_error = msg;
  return code;
}

#define HIPCHECK(c, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(c, MD_EHIP, std::string(#call " failed: ") + hipGetErrorString(e_));     \
  } while (0)

template <typename T>
md_status dalloc(md_ctx c, T** ptr, size_t count) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (c->alloc.alloc) {
    p = c->alloc.alloc(c->alloc.u, bytes, (void*)c->stream);
    if (!p) return fail(c, MD_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, MD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->owned.push_back(p);
  *ptr = (T*)p;
  return MD_OK;
}

void dfree(md_ctx c, void* p) {
  if (!p) return;
  auto it = std::find(c->owned.begin(), c->owned.end(), p);
  if (it != c->owned.end()) c->owned.erase(it);
  if (c->alloc.alloc) {
    (void)hipStreamSynchronize(c->stream);  // nothing queued may still use p
    c->alloc.free(c->alloc.u, p, (void*)c->stream);
  } else {
    (void)hipFree(p);
  }
}

double max_rc(const md_params& p) {
  double m = 0.0;
  for (int a = 0; a < p.ntypes; ++a)
    for (int b = 0; b < p.ntypes; ++b) m = std::max(m, p.rc[a * MD_MAXT + b]);
  return m;
}

// Untruncated pair potential (Eq. (1) / Eq. (2)) and dV/dr at r, for the
// host-side shift constants of Eq. (3).
void plain_v(const md_params& p, int ab, double r, double* v, double* dv) {
  double s = p.sig[ab] / r;
  double s6 = s * s * s * s * s * s, s12 = s6 * s6;
  double e = p.eps[ab];
  if (p.potential == MD_POT_SOFT) {
    *v = 4.0 * e * s12;
    *dv = -48.0 * e * s12 / r;
  } else {
    *v = 4.0 * e * (s12 - s6);
    *dv = -4.0 * e * (12.0 * s12 - 6.0 * s6) / r;
  }
}

md_status validate(const md_params* p, std::string* why) {
  if (!p) return *why = "params is NULL", MD_EINVAL;
  if (p->ntypes < 1 || p->ntypes > MD_MAXT) return *why = "ntypes must be 1..4", MD_EINVAL;
  if (p->potential != MD_POT_LJ && p->potential != MD_POT_SOFT)
    return *why = "unknown potential", MD_EINVAL;
  if (p->trunc != MD_TRUNC_SHIFTED_FORCE && p->trunc != MD_TRUNC_SHIFT)
    return *why = "unknown truncation", MD_EINVAL;
  if (p->precision != MD_FP64 && p->precision != MD_MIXED)
    return *why = "unknown precision", MD_EINVAL;
  for (int a = 0; a < p->ntypes; ++a) {
    if (!(p->mass[a] > 0.0) || !std::isfinite(p->mass[a])) return *why = "mass must be > 0", MD_EINVAL;
    for (int b = 0; b < p->ntypes; ++b) {
      int ab = a * MD_MAXT + b, ba = b * MD_MAXT + a;
      if (!(p->sig[ab] > 0.0) || !(p->rc[ab] > 0.0) || !std::isfinite(p->eps[ab]) ||
          !std::isfinite(p->sig[ab]) || !std::isfinite(p->rc[ab]))
        return *why = "sigma and rc must be finite and > 0", MD_EINVAL;
      if (p->eps[ab] != p->eps[ba] || p->sig[ab] != p->sig[ba] || p->rc[ab] != p->rc[ba])
        return *why = "species tables must be symmetric", MD_EINVAL;
    }
  }
  if (!(p->skin >= 0.0) || !std::isfinite(p->skin)) return *why = "skin must be >= 0", MD_EINVAL;
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return *why = "dt must be > 0", MD_EINVAL;
  if (p->max_neighbors < 0) return *why = "max_neighbors must be >= 0", MD_EINVAL;
  if (p->tpp != 0 && p->tpp != 1 && p->tpp != 2 && p->tpp != 4 && p->tpp != 8)
    return *why = "tpp must be 0, 1, 2, 4 or 8", MD_EINVAL;
  if (p->graph_steps < 0) return *why = "graph_steps must be >= 0", MD_EINVAL;
  if (p->unroll != 0 && p->unroll != 1 && p->unroll != 2 && p->unroll != 4 && p->unroll != 8)
    return *why = "unroll must be 0, 1, 2, 4 or 8", MD_EINVAL;
  if (p->path < MD_PATH_AUTO || p->path > MD_PATH_CELLS) return *why = "unknown path", MD_EINVAL;
  if (p->tile_cells < 0 || p->tile_cells > kMaxRowCells)
    return *why = "tile_cells must be 0..64", MD_EINVAL;
  if (p->stage_slots != 0 && p->stage_slots < 64) return *why = "stage_slots must be 0 or >= 64", MD_EINVAL;
  if (p->split_kick != 0 && p->split_kick != 1) return *why = "split_kick must be 0 or 1", MD_EINVAL;
  if (p->small_box != 0 && p->small_box != 1) return *why = "small_box must be 0 or 1", MD_EINVAL;
  return MD_OK;
}

md_status sync_and_check(md_ctx c) {
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  DevState st{};
  HIPCHECK(c, hipMemcpy(&st, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
  if (st.err) {
    DevState z{};
    HIPCHECK(c, hipMemcpy(c->st, &z, sizeof(DevState), hipMemcpyHostToDevice));
    if (st.err & kErrSlots)
      return fail(c, MD_EOVERFLOW,
                  "a staged row tile's neighbourhood exceeds 16383 LDS slots (use smaller "
                  "tile_cells)");
    if (st.err & kErrOverflow)
      return fail(c, MD_EOVERFLOW, "neighbour list capacity exceeded");
    if (st.err & kErrType) return fail(c, MD_EINVAL, "species index out of range");
    if (st.err & kErrStray)
      return fail(c, MD_ENONFINITE, "a position left the box by more than one box length");
    return fail(c, MD_ENONFINITE, "non-finite position, velocity or force");
  }
  return MD_OK;
}

// zeroed: the kick of this step (or the fused force launch of the previous
// step) already cleared the cell histogram (one replica, see
// launch_kick_drift's nzero and FuseOut)
void run_chain(md_ctx c, hipStream_t s, bool zeroed = false) {
  // several replicas rebuild at different steps: spread each one's blocks
  // (bin/scatter: groups of 4 tiles; list build: groups of 32 cells)
  const int32_t spread_t = c->nrep > 1 ? 4 : 0, spread_c = c->nrep > 1 ? 32 : 0;
  if (c->small_chain) {
    // its histogram lives in LDS: nothing to clear
    launch_chain_small(s, c->reps, c->rebuild, c->pos, c->id, c->img, c->cell_start, c->stride,
                       c->vel, c->id_tmp, c->pos_tmp, c->vel_tmp, c->st);
  } else {
    if (!zeroed) launch_zero_counts(s, c->ncells, c->cell_rep, c->rebuild, c->st, c->counts);
    launch_bin(s, c->ntiles, c->tiles, c->reps, c->rebuild, c->pos, c->id, c->img, c->counts,
               c->cell_of, c->slot, c->st, spread_t);
    launch_scan(s, c->ncells, c->counts, c->cell_start, c->bsum, c->st);
    launch_scatter(s, c->ntiles, c->tiles, c->rebuild, c->cell_of, c->slot, c->cell_start,
                   c->tmp_src, c->st, spread_t);
    launch_cell_gather(s, c->ncells, c->cell_rep, c->rebuild, c->cell_start, c->tmp_src,
                       c->stride, c->id, c->pos, c->vel, c->id_tmp, c->pos_tmp, c->vel_tmp,
                       c->st);
  }
  if (c->cells)
    launch_commit_order(s, c->ntiles, c->tiles, c->rebuild, c->stride, c->pos_tmp, c->vel_tmp,
                        c->id_tmp, c->pos, c->vel, c->id, c->xref, c->st);
  else if (c->staged)
    launch_nlist_tiles(s, c->ncells, c->cell_rep, c->reps, c->rebuild, c->tab, c->thr_form,
                       c->cell_start,
                       c->stride, c->cap, c->pos_tmp, c->vel_tmp, c->id_tmp, c->pos, c->vel, c->id,
                       c->xref, c->nbr16, c->ncount, c->st, c->cell_tile, c->rtiles, spread_c);
  else if (c->small_list && c->any_multi)
    launch_nlist_small(s, c->ntot, c->reps, c->rebuild, c->tab, c->cell_start, c->stride, c->cap,
                       c->pos_tmp, c->vel_tmp, c->id_tmp, c->pos, c->vel, c->id, c->xref, c->nbr,
                       c->ncount, c->st, c->pos16);
  else
    launch_nlist(s, c->ntiles, c->tiles, c->reps, c->rebuild, c->tab, c->thr_form, c->cell_start,
                 c->stride, c->cap, c->pos_tmp, c->vel_tmp, c->id_tmp, c->pos, c->vel, c->id,
                 c->xref, c->nbr, c->ncount, c->st, c->ncells, c->cell_rep, c->any_single,
                 c->any_multi, c->pos16, spread_c);
}

// energy: form PE and W (the staged and list-free kernels always do).
// mode 2 (gather path only): the fused NVE step, see FuseOut; the caller
// swaps the position buffers after the launch.
void launch_forces(md_ctx c, int32_t mode, hipStream_t s, int32_t energy = 1,
                   int32_t nzero = 0) {
  if (c->cells)
    launch_force_cells(s, c->mixed, mode, c->rc2_form, c->nrt, c->rtiles, c->reps, c->tab,
                       c->cell_start, c->pos, c->vel, c->frc, c->stride, c->p.dt, c->part,
                       c->st);
  else if (c->staged)
    launch_force_staged(s, c->mixed, mode, c->tpp, c->unroll, c->nrt, c->rtiles, c->reps,
                        c->tab, c->cell_start, c->pos, c->vel, c->frc, c->nbr16, c->ncount,
                        c->stride, c->cap, c->lcap_f, c->p.dt, c->part, c->st);
  else
    launch_force(s, c->mixed, mode, energy,
                 (size_t)c->nmax_rep * c->cap * sizeof(uint32_t) > kStreamListBytes, c->tpp,
                 c->unroll, c->ntiles, c->tiles, c->reps, c->tab, c->pos, c->pos16, c->vel,
                 c->frc, c->nbr, c->ncount, c->stride, c->cap, c->p.dt, c->part, c->st,
                 FuseOut{c->pos_tmp, c->pos16_alt, c->xref, c->counts, nzero});
}

void drop_graph(md_ctx c);

// Grow the neighbour capacity after an overflowed build to the longest row it
// found plus 16 (never below the old capacity).  The rows already built move
// to the new layout (a replica that did not rebuild keeps its list bit for
// bit); the overflowed rows are rebuilt by the caller.  A captured graph
// holds the old list pointer and capacity and is dropped.
md_status grow_capacity(md_ctx c) {
  std::vector<int32_t> cnt(c->ntot);
  HIPCHECK(c, hipMemcpy(cnt.data(), c->ncount, sizeof(int32_t) * c->ntot, hipMemcpyDeviceToHost));
  int32_t m = 0;
  for (int32_t v : cnt) m = std::max(m, v);
  if (m <= c->cap) return fail(c, MD_EOVERFLOW, "overflow flagged with every row within capacity");
  const int32_t cap = std::max(c->cap, ((m + 16 + 7) / 8) * 8);
  const int32_t elem = c->staged ? 2 : 4;
  void* old = c->staged ? (void*)c->nbr16 : (void*)c->nbr;
  md_status rc;
  void* fresh = nullptr;
  if (c->staged) {
    uint16_t* p = nullptr;
    rc = dalloc(c, &p, list_elems(c->ntot, cap));
    fresh = p;
  } else {
    uint32_t* p = nullptr;
    rc = dalloc(c, &p, list_elems(c->ntot, cap));
    fresh = p;
  }
  if (rc) return rc;
  launch_relayout_list(c->stream, c->ntot, c->ncount, c->cap, cap, elem, old, fresh);
  HIPCHECK(c, hipGetLastError());
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  dfree(c, old);
  if (c->staged)
    c->nbr16 = (uint16_t*)fresh;
  else
    c->nbr = (uint32_t*)fresh;
  c->cap = cap;
  drop_graph(c);
  return MD_OK;
}

// Full rebuild of every replica (md_build_cells and the first build after
// md_set_state); grows the neighbour capacity once on overflow.
md_status build_all(md_ctx c) {
  for (int attempt = 0; attempt < 2; ++attempt) {
    launch_mark_rebuild(c->stream, c->nrep, c->rebuild, c->st);
    run_chain(c, c->stream);
    launch_after_build(c->stream, c->nrep, c->rebuild, c->obs, c->st);
    md_status rc = sync_and_check(c);
    if (rc == MD_OK) {
      c->built = true;
      c->forces_valid = false;
      return MD_OK;
    }
    if (rc != MD_EOVERFLOW || attempt == 1) return rc;
    if (c->err.find("LDS slots") != std::string::npos) return rc;  // not a capacity
    rc = grow_capacity(c);
    if (rc) return rc;
  }
  return MD_OK;
}

ThermoArgs no_thermo() {
  ThermoArgs t{};
  return t;
}

void launch_reductions(md_ctx c, hipStream_t s, int32_t step, const ThermoArgs& ta,
                       int32_t energy = 1, int32_t drift_src = 0, int32_t next = 0) {
  if (c->nchunks)
    launch_reduce_chunks(s, c->nchunks, c->chunks, c->part, c->dmax, step, next, c->part2,
                         c->st);
  launch_reduce(s, c->nrep, c->reps, c->part, c->dmax, c->nchunks ? c->part2 : nullptr, step,
                energy, DriftArgs{drift_src, next, c->dpend}, ta, c->kcall, c->lam, c->rebuild,
                c->obs, c->st);
}

// Split every replica's partial blocks [fb0, fb1) (and drift tiles) into
// chunks of about kRedChunk when some replica has more than 16 chunks' worth;
// otherwise the per-replica pass reads the partials directly (one launch
// instead of two: up to 16 partials per thread of its block).  Host side
// only: the caller uploads reps and chunks.
void plan_chunks(md_ctx c) {
  int32_t most = 0;
  for (const RepDesc& d : c->reps_h) most = std::max(most, d.fb1 - d.fb0);
  c->chunks_h.clear();
  if (most <= 16 * kRedChunk) {
    c->nchunks = 0;
    for (RepDesc& d : c->reps_h) d.cb0 = d.cb1 = 0;
    return;
  }
  for (RepDesc& d : c->reps_h) {
    const int64_t nb = d.fb1 - d.fb0, nt = d.tile1 - d.tile0;
    const int64_t nch = std::max<int64_t>(1, (nb + kRedChunk - 1) / kRedChunk);
    d.cb0 = (int32_t)c->chunks_h.size();
    for (int64_t j = 0; j < nch; ++j) {
      RedChunk ch;
      ch.b0 = d.fb0 + (int32_t)(nb * j / nch);
      ch.b1 = d.fb0 + (int32_t)(nb * (j + 1) / nch);
      ch.t0 = d.tile0 + (int32_t)(nt * j / nch);
      ch.t1 = d.tile0 + (int32_t)(nt * (j + 1) / nch);
      c->chunks_h.push_back(ch);
    }
    d.cb1 = (int32_t)c->chunks_h.size();
  }
  c->nchunks = (int32_t)c->chunks_h.size();
}

void launch_forces0(md_ctx c) {
  launch_forces(c, 0, c->stream);
  launch_reductions(c, c->stream, 0, no_thermo());
}


// Directly launched NVE steps of a one-replica gather-path context can fuse
// the next step's kick and drift into the force launch (md_params.split_kick).
bool can_fuse(md_ctx c, int32_t thermo) {
  return !thermo && c->nrep == 1 && !c->cells && !c->staged && c->p.split_kick == 0;
}

// One velocity-Verlet step on stream s (also used while capturing a graph).
// energy: the step forms PE and W (the observables refreshed on it).
// kick: launch this step's first half kick and drift (false when the
// previous step's fused force launch applied them).  fuse: this step's force
// launch applies the next step's kick and drift (force mode 2); the next
// step is then enqueued with kick = false.
// resume: finish a step whose list build overflowed (kHalt): its kick and
// drift are done and its histogram is stale, so the chain clears the counts
// itself; drift_src (0: kick tile maxima, 1: the maximum the previous fused
// force launch stored) is then the one of the interrupted step.
md_status enqueue_step(md_ctx c, hipStream_t s, const ThermoArgs& ta, int32_t thermo, int32_t k,
                       int32_t energy, bool kick = true, bool fuse = false, bool resume = false,
                       int32_t drift_src = -1) {
  // one replica: its histogram is read only inside a rebuild, so the kick
  // (or the fused force launch before it) clears it when its threads cover
  // the cells (not in very dilute boxes) and the chain skips a launch (the
  // one-block chain of a small box keeps its histogram in LDS)
  const bool zero_in_kick = c->nrep == 1 && !c->small_chain &&
                            (int64_t)c->ncells <= (int64_t)c->ntiles * kTile;
  const int32_t nzero = zero_in_kick ? c->ncells : 0;
  if (kick && !resume)
    launch_kick_drift(s, c->mixed, thermo, c->ntiles, c->tiles, c->reps, c->tab, c->pos,
                      c->pos16, c->vel, c->frc, c->xref, c->stride, c->p.dt, c->lam, c->rebuild,
                      c->dmax, c->st, c->counts, nzero);
  run_chain(c, s, zero_in_kick && !resume);
  const bool timed = c->prof_every > 0 && (k + 1) % c->prof_every == 0;
  if (timed) {
    if (c->ev_pool.size() < c->ev_used + 2) return fail(c, MD_EHIP, "event pool exhausted");
    HIPCHECK(c, hipEventRecord(c->ev_pool[c->ev_used], s));
  }
  launch_forces(c, fuse ? 2 : 1, s, energy, fuse ? nzero : 0);
  if (timed) {
    HIPCHECK(c, hipEventRecord(c->ev_pool[c->ev_used + 1], s));
    c->ev_used += 2;
  }
  if (fuse) {
    std::swap(c->pos, c->pos_tmp);
    std::swap(c->pos16, c->pos16_alt);
  }
  launch_reductions(c, s, 1, ta, energy, drift_src >= 0 ? drift_src : (kick ? 0 : 1),
                    fuse ? 1 : 0);
  return MD_OK;
}

// Steps that form PE and W: the logged ones and the last of the run (the
// observables md_observables returns).  Inside a K-step graph: the logged
// steps when the log cadence divides K (the same steps in every replay),
// every step otherwise, and always the graph's last step.
int32_t energy_step(const ThermoArgs& ta, int64_t k, int64_t last) {
  if (k == last) return 1;
  return ta.log_every > 0 && (k + 1) % ta.log_every == 0;
}
int32_t energy_step_graph(const ThermoArgs& ta, int32_t k, int32_t K) {
  if (k == K - 1) return 1;
  if (ta.log_every <= 0) return 0;
  return K % ta.log_every != 0 || (k + 1) % ta.log_every == 0;
}

md_status reserve_events(md_ctx c, int32_t nsteps);

// Directly launched steps [k0, nsteps) of an md_step call whose steps
// [0, kg) ran inside graph replays.  A step launched here after another one
// of this loop had its kick and drift applied by that step's force launch
// when the call can fuse.  resume: step k0 was interrupted by an overflowed
// list build after its kick and drift; its drift maximum is where that kick
// left it (the previous force launch's partials for a fused direct step, the
// kick's tile maxima otherwise).
md_status enqueue_direct(md_ctx c, hipStream_t s, const ThermoArgs& ta, int32_t thermo,
                         int32_t kg, int32_t k0, int32_t nsteps, bool fusable, bool resume) {
  md_status rc = reserve_events(c, nsteps - k0);
  if (rc) return rc;
  for (int32_t k = k0; k < nsteps; ++k) {
    const bool res = resume && k == k0;
    const bool kick = !res && !(fusable && k > k0);
    const int32_t src = res ? (fusable && k > kg ? 1 : 0) : -1;
    rc = enqueue_step(c, s, ta, thermo, k, energy_step(ta, k, nsteps - 1), kick,
                      fusable && k + 1 < nsteps, res, src);
    if (rc) return rc;
  }
  return MD_OK;
}

md_status reserve_events(md_ctx c, int32_t nsteps) {
  if (c->prof_every <= 0) return MD_OK;
  const size_t need = c->ev_used + 2 * (size_t)(nsteps / c->prof_every + 1);
  while (c->ev_pool.size() < need) {
    hipEvent_t e;
    HIPCHECK(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  return MD_OK;
}

void drop_graph(md_ctx c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
}

// A graph of K steps, captured once per launch configuration and replayed:
// every argument is fixed, the step number lives in device counters.
md_status ensure_graph(md_ctx c, const ThermoArgs& ta, int32_t thermo, int32_t K) {
  const int64_t key[15] = {K, thermo, ta.ramp, ta.log_every, ta.nlog, (int64_t)(intptr_t)ta.log,
                           (int64_t)(intptr_t)c->nbr, (int64_t)(intptr_t)c->nbr16,
                           c->prof_every, c->prof_epoch, (int64_t)(intptr_t)c->pos,
                           c->cap, c->lcap_f, c->tpp, c->unroll};
  if (c->gexec && std::equal(key, key + 15, c->gkey)) return MD_OK;
  drop_graph(c);
  if (!c->cap_stream) HIPCHECK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  md_status rc = reserve_events(c, K);
  if (rc) return rc;
  HIPCHECK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  for (int32_t k = 0; k < K && rc == MD_OK; ++k)
    rc = enqueue_step(c, c->cap_stream, ta, thermo, k, energy_step_graph(ta, k, K));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(c, MD_EHIP, "graph capture failed");
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return fail(c, MD_EHIP, "graph instantiation failed");
  }
  std::copy(key, key + 15, c->gkey);
  return MD_OK;
}

}  // namespace

extern "C" {

const char* md_last_error(md_ctx c) { return c ? c->err.c_str() : g_init_error.c_str(); }

md_status md_init(md_ctx* out, const md_params* p, int32_t nrep, const int64_t* n,
                  const double* L, void* hip_stream) {
  return md_init_alloc(out, p, nrep, n, L, hip_stream, nullptr);
}

md_status md_init_alloc(md_ctx* out, const md_params* p, int32_t nrep, const int64_t* n,
                        const double* L, void* hip_stream, const md_allocator* alloc) {
  if (!out) return fail(nullptr, MD_EINVAL, "out is NULL");
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, MD_EINVAL, "allocator needs both alloc and free");
  *out = nullptr;
  std::string why;
  if (validate(p, &why)) return fail(nullptr, MD_EINVAL, why);
  if (nrep < 1 || !n || !L) return fail(nullptr, MD_EINVAL, "need nrep >= 1 and n, L arrays");
  const double rcmax = max_rc(*p);
  int64_t ntot = 0;
  for (int r = 0; r < nrep; ++r) {
    if (n[r] < 2) return fail(nullptr, MD_EINVAL, "every replica needs at least 2 particles");
    if (!std::isfinite(L[r]) || !(L[r] >= 2.0 * (rcmax + p->skin)))
      return fail(nullptr, MD_EBOX, "box side L must be >= 2 (max rc + skin)");
    ntot += n[r];
  }
  // list entries carry a 26-bit particle index; the list-free path keeps no
  // list and indexes particles with 32-bit integers
  if (p->path != MD_PATH_CELLS && ntot > (int64_t)kIdxMask + 1)
    return fail(nullptr, MD_EINVAL,
                "total particle count must be <= 2^26 on the list paths (the list-free "
                "path takes up to 2^30)");
  // SoA components are addressed as stride + i in 32-bit arithmetic
  if (ntot > (int64_t)1 << 30)
    return fail(nullptr, MD_EINVAL, "total particle count must be <= 2^30");

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, MD_EHIP, "hipGetDevice failed");
  {
    const hipError_t e = scratch_setup(dev);
    if (e != hipSuccess)
      return fail(nullptr, MD_EHIP,
                  std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  }
  md_ctx c = new md_ctx_s();
  c->p = *p;
  c->device = dev;
  c->nrep = nrep;
  c->ntot = (int32_t)ntot;
  c->stride = (int32_t)(((ntot + 63) / 64) * 64);
  c->mixed = p->precision == MD_MIXED;
  c->tpp = p->tpp == 0 ? 2 : p->tpp;
  c->unroll = p->unroll == 0 ? 4 : p->unroll;
  c->stream = (hipStream_t)hip_stream;
  if (alloc) c->alloc = *alloc;
  for (int r = 0; r < nrep; ++r) c->nmax_rep = std::max<int32_t>(c->nmax_rep, (int32_t)n[r]);

  // replica geometry: cells of side >= max rc + skin (nc < 3 -> one cell)
  const double side = rcmax + p->skin;
  int32_t off = 0, coff = 0, tile = 0;
  double rho_max = 0.0;
  for (int r = 0; r < nrep; ++r) {
    RepDesc d{};
    int32_t nc = (int32_t)std::floor(L[r] / side);
    if (nc < 3) nc = 1;
    d.L = L[r];
    d.inv_cell = (double)nc / L[r];
    d.half_skin2 = (0.5 * p->skin) * (0.5 * p->skin);
    d.dof = 3.0 * (double)n[r] - 3.0;
    d.volume = L[r] * L[r] * L[r];
    d.cside = L[r] / nc;
    // mixed records: the largest power of two scale s.t. half a cell side
    // plus the skin plus one unit of drift stays below 2^30 fixed-point units
    d.qs = 1.0;
    while ((0.5 * d.cside + p->skin + 1.0) * (2.0 * d.qs) <= 1073741824.0) d.qs *= 2.0;
    d.qinv = 1.0 / d.qs;
    d.off = off;
    d.n = (int32_t)n[r];
    d.coff = coff;
    d.nc = nc;
    d.tile0 = tile;
    for (int32_t s0 = off; s0 < off + d.n; s0 += kTile) {
      Tile t{};
      t.rep = r;
      t.start = s0;
      t.end = std::min(s0 + kTile, off + d.n);
      c->tiles_h.push_back(t);
      ++tile;
    }
    d.tile1 = tile;
    c->reps_h.push_back(d);
    off += d.n;
    int64_t cells = (int64_t)nc * nc * nc;
    if ((int64_t)coff + cells > (int64_t)0x7fffffff) {
      delete c;
      return fail(nullptr, MD_EINVAL, "too many cells");
    }
    coff += (int32_t)cells;
    rho_max = std::max(rho_max, (double)n[r] / d.volume);
  }
  c->ncells = coff;
  c->ntiles = tile;
  c->small_chain = p->small_box == 0 && nrep == 1 && ntot <= kSmallN && c->ncells <= kSmallCells;
  c->small_list = p->small_box == 0 && nrep == 1 && ntot <= kSmallListN;

  // kernel path: the staged path needs >= 3 cells per side in every replica
  bool all3 = true;
  for (const RepDesc& d : c->reps_h) {
    all3 = all3 && d.nc >= 3;
    if (d.nc == 1) c->any_single = 1;
    else c->any_multi = 1;
  }
  if ((p->path == MD_PATH_STAGED || p->path == MD_PATH_CELLS) && !all3) {
    delete c;
    return fail(nullptr, MD_EINVAL, "the staged and cell paths need >= 3 cells per box side");
  }
  c->staged = p->path == MD_PATH_STAGED;
  c->cells = p->path == MD_PATH_CELLS;
  if (c->mixed && !c->staged && !c->cells)
    for (const RepDesc& d : c->reps_h)
      if (d.nc > 1023) {
        delete c;
        return fail(nullptr, MD_EINVAL,
                    "mixed precision on the gather path supports up to 1023 cells per side");
      }
  int32_t lds_max = 65536;
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      lds_max = v;
    (void)hipGetLastError();
    lds_max = std::min(lds_max, 65536);  // stay within the default per-block limit
  }
  if (c->staged || c->cells) {
    if (c->staged && c->tpp == 8) {
      delete c;
      return fail(nullptr, MD_EINVAL, "the staged path takes tpp 1, 2 or 4");
    }
    // row tiles of about 128 home particles; on the staged path LDS holds the
    // tile's 9 x (nx + 2) cells with 30 % headroom (denser tiles spill to
    // global memory)
    const int32_t homes = c->cells ? cells_homes_per_block() : staged_homes_per_group();
    double need = 0.0;
    for (int r = 0; r < nrep; ++r) {
      RepDesc& d = c->reps_h[r];
      const int32_t nc = d.nc;
      const double ppc = (double)d.n / ((double)nc * nc * nc);
      int32_t cpt = p->tile_cells;
      if (cpt <= 0) cpt = (int32_t)std::floor(0.85 * homes / ppc);
      cpt = std::max(1, std::min(cpt, std::min(nc, (int32_t)kMaxRowCells)));
      const int32_t ntr = (nc + cpt - 1) / cpt;
      d.fb0 = (int32_t)c->rtiles_h.size();
      int32_t nxmax = 0;
      for (int32_t row = 0; row < nc * nc; ++row)
        for (int32_t t = 0; t < ntr; ++t) {
          RowTile rt{};
          rt.rep = r;
          rt.row = row;
          rt.a = (int32_t)((int64_t)t * nc / ntr);
          rt.nx = (int32_t)((int64_t)(t + 1) * nc / ntr) - rt.a;
          nxmax = std::max(nxmax, rt.nx);
          c->rtiles_h.push_back(rt);
        }
      d.fb1 = (int32_t)c->rtiles_h.size();
      need = std::max(need, 9.0 * (nxmax + 2) * ppc);
    }
    c->nrt = (int32_t)c->rtiles_h.size();
    const int32_t want = (int32_t)((int64_t)std::ceil(1.3 * need + 64) / 64 * 64);
    const int32_t room = lds_max - 8192;  // static LDS of the kernel
    c->lcap_f = std::max(64, std::min(want, (int32_t)(room / 24)));
    if (p->stage_slots > 0) c->lcap_f = std::min(c->lcap_f, p->stage_slots);
  } else {
    for (RepDesc& d : c->reps_h) {
      d.fb0 = d.tile0 * c->tpp;
      d.fb1 = d.tile1 * c->tpp;
    }
  }
  if (p->max_neighbors > 0) {
    c->cap = p->max_neighbors;
  } else {
    const double expect = rho_max * 4.0 / 3.0 * M_PI * side * side * side;
    c->cap = (int32_t)(((int64_t)std::ceil(1.5 * expect) + 16 + 7) / 8 * 8);
  }

  // pair table: shift constants of Eq. (3) computed on the host in FP64
  PairTab tab{};
  for (int a = 0; a < MD_MAXT; ++a)
    for (int b = 0; b < MD_MAXT; ++b) {
      const int ab = a * MD_MAXT + b;
      if (a >= p->ntypes || b >= p->ntypes) {
        tab.rc2[ab] = 0.0;  // never used
        tab.thr[ab] = 0.0;
        tab.sig2[ab] = 1.0;
        continue;
      }
      const double rc = p->rc[ab];
      const double t = rc + p->skin;
      tab.rc2[ab] = rc * rc;
      tab.thr[ab] = t * t;
      tab.sig2[ab] = p->sig[ab] * p->sig[ab];
      const double e = p->eps[ab];
      tab.c12[ab] = 4.0 * e;
      tab.c6[ab] = p->potential == MD_POT_SOFT ? 0.0 : -4.0 * e;
      tab.f12[ab] = 48.0 * e;
      tab.f6[ab] = p->potential == MD_POT_SOFT ? 0.0 : -24.0 * e;
      double vc, dvc;
      plain_v(*p, ab, rc, &vc, &dvc);
      tab.vc[ab] = vc;
      tab.fs[ab] = p->trunc == MD_TRUNC_SHIFTED_FORCE ? dvc : 0.0;
      tab.rc[ab] = rc;
    }
  for (int a = 0; a < MD_MAXT; ++a) {
    tab.mass[a] = a < p->ntypes ? p->mass[a] : 1.0;
    tab.inv_mass[a] = 1.0 / tab.mass[a];
  }
  c->thr_form = fma_pair_form(tab.thr, p->ntypes);
  c->rc2_form = fma_pair_form(tab.rc2, p->ntypes);

  std::vector<int32_t> cell_rep(c->ncells);
  for (int r = 0; r < nrep; ++r) {
    const RepDesc& d = c->reps_h[r];
    std::fill(cell_rep.begin() + d.coff, cell_rep.begin() + d.coff + d.nc * d.nc * d.nc, r);
  }

  const size_t N = c->ntot, S = c->stride;
  md_status rc = MD_OK;
#define ALLOC(ptr, count)                       \
  if ((rc = dalloc(c, &(ptr), (count))) != 0) { \
    std::string m_ = c->err;                    \
    md_destroy(c);                              \
    return fail(nullptr, rc, m_);               \
  }
  ALLOC(c->reps, (size_t)nrep);
  ALLOC(c->tiles, (size_t)c->ntiles);
  ALLOC(c->tab, 1);
  ALLOC(c->st, 1);
  ALLOC(c->cell_rep, (size_t)c->ncells);
  ALLOC(c->counts, (size_t)c->ncells);
  ALLOC(c->cell_start, (size_t)c->ncells + 1);
  ALLOC(c->bsum, scan_bsum_elems(c->ncells));
  ALLOC(c->cell_of, N);
  ALLOC(c->slot, N);
  ALLOC(c->tmp_src, N);
  ALLOC(c->pos, N);
  ALLOC(c->pos_tmp, N);
  ALLOC(c->vel, 3 * S);
  ALLOC(c->vel_tmp, 3 * S);
  ALLOC(c->xref, 3 * S);
  if (c->mixed) {
    float* f = nullptr;
    ALLOC(f, 3 * S);
    c->frc = f;
  } else {
    double* f = nullptr;
    ALLOC(f, 3 * S);
    c->frc = f;
  }
  if (c->mixed && !c->staged && !c->cells) {
    ALLOC(c->pos16, S);
    ALLOC(c->pos16_alt, S);
  }
  ALLOC(c->id, N);
  ALLOC(c->id_tmp, N);
  ALLOC(c->img, 3 * N);
  if (c->cells) {
    ALLOC(c->rtiles, (size_t)c->nrt);
  } else if (c->staged) {
    ALLOC(c->nbr16, list_elems(c->ntot, c->cap));
    ALLOC(c->cell_tile, (size_t)c->ncells);
    ALLOC(c->rtiles, (size_t)c->nrt);
  } else {
    ALLOC(c->nbr, list_elems(c->ntot, c->cap));
  }
  if (!c->cells) ALLOC(c->ncount, N);  // list lengths (the list-free path has none)
  ALLOC(c->part, 4 * std::max((size_t)c->ntiles * 8, (size_t)c->nrt));
  ALLOC(c->rebuild, (size_t)nrep);
  ALLOC(c->dmax, (size_t)c->ntiles);
  plan_chunks(c);
  c->max_chunks =
      (int32_t)((std::max((size_t)c->ntiles * 8, (size_t)c->nrt) + kRedChunk - 1) / kRedChunk) +
      nrep;
  ALLOC(c->chunks, (size_t)c->max_chunks);
  ALLOC(c->part2, (size_t)kPart2 * c->max_chunks);
  ALLOC(c->dpend, (size_t)nrep);
  ALLOC(c->obs, (size_t)nrep);
  ALLOC(c->kcall, (size_t)nrep);
  ALLOC(c->lam, (size_t)nrep);
  ALLOC(c->therm, 2 * (size_t)nrep);
#undef ALLOC
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  std::vector<double> ones(nrep, 1.0);
  std::vector<int32_t> cell_tile;
  if (c->staged) {
    cell_tile.assign(c->ncells, 0);
    for (int32_t t = 0; t < c->nrt; ++t) {
      const RowTile& rt = c->rtiles_h[t];
      const RepDesc& d = c->reps_h[rt.rep];
      for (int32_t x = rt.a; x < rt.a + rt.nx; ++x) cell_tile[d.coff + rt.row * d.nc + x] = t;
    }
  }
  bool ok = up(c->reps, c->reps_h.data(), sizeof(RepDesc) * nrep) &&
            up(c->tiles, c->tiles_h.data(), sizeof(Tile) * c->ntiles) &&
            up(c->tab, &tab, sizeof(PairTab)) &&
            up(c->cell_rep, cell_rep.data(), sizeof(int32_t) * c->ncells) &&
            up(c->lam, ones.data(), sizeof(double) * nrep) &&
            (!(c->staged || c->cells) ||
             up(c->rtiles, c->rtiles_h.data(), sizeof(RowTile) * c->nrt)) &&
            (!c->nchunks || up(c->chunks, c->chunks_h.data(), sizeof(RedChunk) * c->nchunks)) &&
            (!c->staged ||
             up(c->cell_tile, cell_tile.data(), sizeof(int32_t) * (size_t)c->ncells)) &&
            hipMemset(c->st, 0, sizeof(DevState)) == hipSuccess &&
            hipMemset(c->counts, 0, sizeof(int32_t) * c->ncells) == hipSuccess &&
            hipMemset(c->rebuild, 0, sizeof(int32_t) * nrep) == hipSuccess &&
            hipMemset(c->obs, 0, sizeof(md_obs) * nrep) == hipSuccess &&
            hipMemset(c->kcall, 0, sizeof(int64_t) * nrep) == hipSuccess &&
            hipMemset(c->dpend, 0, sizeof(double) * nrep) == hipSuccess &&
            hipMemset(c->frc, 0, (c->mixed ? 4 : 8) * 3 * S) == hipSuccess;
  if (!ok) {
    md_destroy(c);
    return fail(nullptr, MD_EHIP, "uploading context tables failed");
  }
  *out = c;
  return MD_OK;
}

md_status md_destroy(md_ctx c) {
  if (!c) return MD_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (void* p : c->owned) {
    if (c->alloc.alloc)
      c->alloc.free(c->alloc.u, p, (void*)c->stream);
    else
      (void)hipFree(p);
  }
  c->owned.clear();
  delete c;
  return MD_OK;
}

md_status md_set_state(md_ctx c, const double* x, const double* v, const int32_t* type) {
  if (!c) return MD_EINVAL;
  if (!x || !v || !type) return fail(c, MD_EINVAL, "x, v and type are required");
  launch_set_state(c->stream, c->ntot, c->stride, x, v, type, c->p.ntypes, c->pos, c->vel, c->id,
                   c->img, c->st);
  HIPCHECK(c, hipMemsetAsync(c->obs, 0, sizeof(md_obs) * c->nrep, c->stream));
  HIPCHECK(c, hipMemsetAsync(c->frc, 0, (c->mixed ? 4 : 8) * 3 * (size_t)c->stride, c->stream));
  md_status rc = sync_and_check(c);
  // positions are checked against the box at the first wrap
  c->has_state = rc == MD_OK;
  c->built = false;
  c->forces_valid = false;
  return rc;
}

md_status md_get_state(md_ctx c, double* x, double* v, int32_t* img) {
  if (!c) return MD_EINVAL;
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  if (x || v) launch_get_state(c->stream, c->ntot, c->stride, c->pos, c->vel, c->id, x, v);
  if (img)
    HIPCHECK(c, hipMemcpyAsync(img, c->img, sizeof(int32_t) * 3 * (size_t)c->ntot,
                               hipMemcpyDeviceToDevice, c->stream));
  return sync_and_check(c);
}

md_status md_build_cells(md_ctx c) {
  if (!c) return MD_EINVAL;
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  return build_all(c);
}

md_status md_forces(md_ctx c) {
  if (!c) return MD_EINVAL;
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  if (!c->built) {
    md_status rc = build_all(c);
    if (rc) return rc;
  }
  launch_forces0(c);
  c->forces_valid = true;
  return MD_OK;
}

md_status md_get_forces(md_ctx c, void* F) {
  if (!c) return MD_EINVAL;
  if (!F) return fail(c, MD_EINVAL, "F is NULL");
  if (!c->forces_valid) return fail(c, MD_ESTATE, "no forces computed");
  launch_get_forces(c->stream, c->ntot, c->stride, c->frc, c->mixed, c->id, F);
  return sync_and_check(c);
}

md_status md_step(md_ctx c, int32_t nsteps, const double* T0, const double* T1,
                  int64_t ramp_steps, md_obs* log, int32_t log_every) {
  if (!c) return MD_EINVAL;
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  if (nsteps < 0) return fail(c, MD_EINVAL, "nsteps must be >= 0");
  if (log && log_every <= 0) return fail(c, MD_EINVAL, "log needs log_every > 0");
  const int32_t thermo = T0 != nullptr;
  if (thermo) {
    for (int r = 0; r < c->nrep; ++r) {
      const double t1 = T1 ? T1[r] : T0[r];
      if (!(T0[r] > 0.0) || !(t1 > 0.0) || !std::isfinite(T0[r]) || !std::isfinite(t1))
        return fail(c, MD_EINVAL, "thermostat targets must be finite and > 0");
    }
  }
  if (!c->built) {
    md_status rc = build_all(c);
    if (rc) return rc;
  }
  if (!c->forces_valid) {
    launch_forces0(c);
    c->forces_valid = true;
  }
  ThermoArgs ta{};
  if (thermo) {
    std::vector<double> th(2 * c->nrep);
    for (int r = 0; r < c->nrep; ++r) {
      th[r] = T0[r];
      th[c->nrep + r] = T1 ? T1[r] : T0[r];
    }
    HIPCHECK(c, hipMemcpyAsync(c->therm, th.data(), sizeof(double) * th.size(),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));  // th is a local buffer
    ta.T0 = c->therm;
    ta.T1 = c->therm + c->nrep;
    ta.ramp = ramp_steps;
    ta.thermo = 1;
  }
  int64_t nlog = 0;
  if (log) {
    nlog = nsteps / log_every;
    if (nlog * c->nrep > c->log_cap) {
      dfree(c, c->log_dev);
      c->log_dev = nullptr;
      c->log_cap = 0;
      md_status rc = dalloc(c, &c->log_dev, (size_t)std::max<int64_t>(nlog * c->nrep, 1));
      if (rc) return rc;
      c->log_cap = nlog * c->nrep;
    }
    ta.log_every = log_every;
    ta.log = c->log_dev;
    ta.nlog = (int32_t)nlog;
  }
  hipStream_t s = c->stream;
  launch_begin_call(s, c->nrep, c->kcall, c->lam);
  int32_t k = 0;
  // events recorded inside a captured graph cannot be timed, so profiled
  // steps are launched directly
  const int32_t K = c->prof_every > 0 ? 0 : c->p.graph_steps;
  if (K > 0 && nsteps >= K) {
    md_status rc = ensure_graph(c, ta, thermo, K);
    if (rc) return rc;
    for (; k + K <= nsteps; k += K) HIPCHECK(c, hipGraphLaunch(c->gexec, s));
  }
  const int32_t kg = k;  // steps [0, kg) ran inside graph replays
  // the last step of a call is never fused: the state it leaves (positions,
  // velocities, forces) is complete
  const bool fusable = can_fuse(c, thermo);
  md_status rc = enqueue_direct(c, s, ta, thermo, kg, kg, nsteps, fusable, false);
  if (rc) return rc;
  if (thermo) launch_apply_lambda(s, c->ntiles, c->tiles, c->stride, c->vel, c->lam, c->nrep, c->st);
  HIPCHECK(c, hipGetLastError());
  // a list build that overflowed halted the queued steps (kHalt): grow the
  // capacity, rebuild the interrupted step's lists on its state and finish
  // the call from there -- the trajectory of a context with enough capacity
  for (int attempt = 0;; ++attempt) {
    HIPCHECK(c, hipStreamSynchronize(s));
    DevState st{};
    HIPCHECK(c, hipMemcpy(&st, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (!(st.err & kErrOverflow) || (st.err & ~kErrOverflow) || attempt == 8) break;
    int64_t done = 0;
    HIPCHECK(c, hipMemcpy(&done, c->kcall, sizeof(int64_t), hipMemcpyDeviceToHost));
    rc = grow_capacity(c);
    if (rc) {
      c->built = false;
      c->forces_valid = false;
      return rc;
    }
    st.err = 0;
    st.any_rebuild = 1;  // the interrupted step's rebuild flags are still set
    HIPCHECK(c, hipMemcpy(c->st, &st, sizeof(DevState), hipMemcpyHostToDevice));
    rc = enqueue_direct(c, s, ta, thermo, kg, (int32_t)done, nsteps, fusable, true);
    if (rc) return rc;
    if (thermo)
      launch_apply_lambda(s, c->ntiles, c->tiles, c->stride, c->vel, c->lam, c->nrep, c->st);
    HIPCHECK(c, hipGetLastError());
  }
  rc = sync_and_check(c);
  if (rc == MD_EOVERFLOW) {
    // not recoverable by growing the list (staged tile slots, or repeated
    // growth): the state is the interrupted step's
    c->built = false;
    c->forces_valid = false;
    return rc;
  }
  if (rc) return rc;
  if (log && nlog > 0)
    HIPCHECK(c, hipMemcpy(log, c->log_dev, sizeof(md_obs) * nlog * c->nrep,
                          hipMemcpyDeviceToHost));
  return MD_OK;
}

md_status md_observables(md_ctx c, md_obs* out) {
  if (!c) return MD_EINVAL;
  if (!out) return fail(c, MD_EINVAL, "out is NULL");
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  HIPCHECK(c, hipMemcpy(out, c->obs, sizeof(md_obs) * c->nrep, hipMemcpyDeviceToHost));
  return MD_OK;
}

md_status md_get_cells(md_ctx c, int32_t rep, int32_t* cell_start, int32_t* order_ids) {
  if (!c) return MD_EINVAL;
  if (rep < 0 || rep >= c->nrep) return fail(c, MD_EINVAL, "replica index out of range");
  if (!c->built) return fail(c, MD_ESTATE, "cells not built");
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  const RepDesc& d = c->reps_h[rep];
  const int64_t ncell = (int64_t)d.nc * d.nc * d.nc;
  if (cell_start) {
    HIPCHECK(c, hipMemcpy(cell_start, c->cell_start + d.coff, sizeof(int32_t) * (ncell + 1),
                          hipMemcpyDeviceToHost));
    for (int64_t k = 0; k <= ncell; ++k) cell_start[k] -= d.off;
  }
  if (order_ids) {
    HIPCHECK(c, hipMemcpy(order_ids, c->id + d.off, sizeof(int32_t) * d.n,
                          hipMemcpyDeviceToHost));
    for (int32_t k = 0; k < d.n; ++k) order_ids[k] -= d.off;
  }
  return MD_OK;
}

md_status md_get_neighbors(md_ctx c, int32_t rep, int32_t* count, int32_t* ids, int32_t cap) {
  if (!c) return MD_EINVAL;
  if (c->cells) return fail(c, MD_ESTATE, "the cell path keeps no neighbour list");
  if (rep < 0 || rep >= c->nrep) return fail(c, MD_EINVAL, "replica index out of range");
  if (!c->built) return fail(c, MD_ESTATE, "list not built");
  if (!count || (cap > 0 && !ids) || cap < 0) return fail(c, MD_EINVAL, "bad output buffers");
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  const RepDesc& d = c->reps_h[rep];
  std::vector<int32_t> cnt(d.n), idv(c->ntot);
  HIPCHECK(c, hipMemcpy(cnt.data(), c->ncount + d.off, sizeof(int32_t) * d.n,
                        hipMemcpyDeviceToHost));
  HIPCHECK(c, hipMemcpy(idv.data(), c->id, sizeof(int32_t) * c->ntot, hipMemcpyDeviceToHost));
  // the list slices that hold the replica's particles, one contiguous block
  const int32_t s0 = (int32_t)(d.off / kSlice), s1 = (int32_t)((d.off + d.n - 1) / kSlice);
  const size_t lo = (size_t)s0 * kSlice * c->cap, nel = (size_t)(s1 - s0 + 1) * kSlice * c->cap;
  std::vector<uint32_t> sl(cap > 0 && d.n > 0 ? nel : 1);
  if (cap > 0 && d.n > 0) {
    const uint32_t* src = c->nbr;
    uint32_t* tmp = nullptr;
    if (c->staged) {
      // staged entries are LDS slots of the home tile: decode to particle indices
      md_status a_rc = dalloc(c, &tmp, list_elems(c->ntot, c->cap));
      if (a_rc) return a_rc;
      launch_decode_staged(c->stream, c->nrt, c->rtiles, c->reps, c->cell_start, c->cap,
                           c->nbr16, c->ncount, tmp);
      src = tmp;
    }
    hipError_t e = hipMemcpy(sl.data(), src + lo, sizeof(uint32_t) * nel, hipMemcpyDeviceToHost);
    if (tmp) dfree(c, tmp);
    if (e != hipSuccess) return fail(c, MD_EHIP, "copying the neighbour list failed");
  }
  for (int32_t i = 0; i < d.n; ++i) {
    const int32_t g = (int32_t)d.off + i;
    const int32_t orig = idv[g] - d.off;
    count[orig] = cnt[i];
    const int32_t m = std::min(std::min(cnt[i], c->cap), cap);
    const size_t b = list_base(g, c->cap) - lo;
    for (int32_t k = 0; k < m; ++k) {
      const uint32_t e = sl[b + (size_t)k * kSlice];
      ids[(size_t)orig * cap + k] = idv[e & kIdxMask] - d.off;
    }
  }
  return MD_OK;
}

md_status md_replica_info(md_ctx c, int32_t rep, int32_t* nc, double* inv_cell, int64_t* n,
                          int64_t* offset, int32_t* max_neighbors) {
  if (!c) return MD_EINVAL;
  if (rep < 0 || rep >= c->nrep) return fail(c, MD_EINVAL, "replica index out of range");
  const RepDesc& d = c->reps_h[rep];
  if (nc) *nc = d.nc;
  if (inv_cell) *inv_cell = d.inv_cell;
  if (n) *n = d.n;
  if (offset) *offset = d.off;
  if (max_neighbors) *max_neighbors = c->cap;
  return MD_OK;
}

md_status md_profile(md_ctx c, int32_t every) {
  if (!c) return MD_EINVAL;
  if (every < 0) return fail(c, MD_EINVAL, "every must be >= 0");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->prof_every = every;
  c->ev_used = 0;
  c->prof_epoch += 1;  // captured graphs hold events of the previous setting
  return MD_OK;
}

md_status md_profile_read(md_ctx c, md_prof* out) {
  if (!c) return MD_EINVAL;
  if (!out) return fail(c, MD_EINVAL, "out is NULL");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  out->force_launches = (int64_t)(c->ev_used / 2);
  out->force_ms = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.0f;
    HIPCHECK(c, hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
    out->force_ms += ms;
  }
  return MD_OK;
}

md_status md_autotune(md_ctx c, int32_t reps, md_tune* out) {
  if (!c) return MD_EINVAL;
  if (!out || reps < 1) return fail(c, MD_EINVAL, "need out and reps >= 1");
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  if (!c->built) {
    md_status rc = build_all(c);
    if (rc) return rc;
  }
  std::vector<std::pair<int32_t, int32_t>> cand;
  if (c->cells)
    cand = {{1, 1}};  // one kernel variant: nothing to choose
  else if (c->staged)
    cand = {{1, 4}, {1, 8}, {2, 2}, {2, 4}, {2, 8}, {4, 2}};
  else
    cand = {{1, 4}, {1, 8}, {2, 2}, {2, 4}, {4, 1}, {4, 2}, {8, 1}};
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  HIPCHECK(c, hipEventCreate(&e1));
  *out = md_tune{};
  double best = 1e300;
  int32_t btpp = c->tpp, bun = c->unroll;
  for (auto& tu : cand) {
    c->tpp = tu.first;
    c->unroll = tu.second;
    launch_forces(c, 0, c->stream);  // warm
    HIPCHECK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) launch_forces(c, 0, c->stream);
    HIPCHECK(c, hipEventRecord(e1, c->stream));
    HIPCHECK(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHECK(c, hipEventElapsedTime(&ms, e0, e1));
    const double avg = ms / reps;
    if (out->ntried < 16) {
      out->tried_tpp[out->ntried] = tu.first;
      out->tried_unroll[out->ntried] = tu.second;
      out->tried_ms[out->ntried] = avg;
      out->ntried += 1;
    }
    if (avg < best) {
      best = avg;
      btpp = tu.first;
      bun = tu.second;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tpp = btpp;
  c->unroll = bun;
  if (!c->staged && !c->cells) {
    // partial-sum blocks per replica follow the lanes per particle
    for (RepDesc& d : c->reps_h) {
      d.fb0 = d.tile0 * c->tpp;
      d.fb1 = d.tile1 * c->tpp;
    }
    plan_chunks(c);
    if (c->nchunks)
      HIPCHECK(c, hipMemcpyAsync(c->chunks, c->chunks_h.data(), sizeof(RedChunk) * c->nchunks,
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->reps, c->reps_h.data(), sizeof(RepDesc) * c->nrep,
                               hipMemcpyHostToDevice, c->stream));
    // the host vectors are re-planned only here, after the copies finished
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  drop_graph(c);
  launch_forces0(c);
  c->forces_valid = true;
  out->tpp = btpp;
  out->unroll = bun;
  out->force_ms = best;
  return sync_and_check(c);
}

md_status md_msd_reference(md_ctx c) {
  if (!c) return MD_EINVAL;
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  if (!c->u0) {
    md_status rc = dalloc(c, &c->u0, 3 * (size_t)c->ntot);
    if (!rc) rc = dalloc(c, &c->msd_part, (size_t)c->ntiles);
    if (!rc) rc = dalloc(c, &c->msd_out, (size_t)c->nrep);
    if (rc) return rc;
  }
  launch_msd_ref(c->stream, c->ntiles, c->tiles, c->reps, c->pos, c->id, c->img, c->u0);
  return sync_and_check(c);
}

md_status md_msd(md_ctx c, double* out) {
  if (!c) return MD_EINVAL;
  if (!out) return fail(c, MD_EINVAL, "out is NULL");
  if (!c->u0) return fail(c, MD_ESTATE, "no MSD reference set");
  launch_msd(c->stream, c->ntiles, c->nrep, c->tiles, c->reps, c->pos, c->id, c->img, c->u0,
             c->msd_part, c->msd_out);
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  HIPCHECK(c, hipMemcpy(out, c->msd_out, sizeof(double) * c->nrep, hipMemcpyDeviceToHost));
  return MD_OK;
}

namespace {
// g(r) of replica rep into g (HOST [nbins]) from the pair histogram hist
// (DEVICE, >= nbins counters, cleared here).  The counts are copied into g's
// own storage (8 bytes each) and normalised in place.  may_build: build the
// cells first when the cell sweep needs them.
md_status rdf_with(md_ctx c, int32_t rep, double rmax, int32_t nbins, double* g,
                   unsigned long long* hist, bool may_build) {
  const RepDesc& d = c->reps_h[rep];
  // the cell sweep covers every pair closer than the cell side minus the
  // skin while the skin rule holds; otherwise all pairs are visited
  const bool by_cells = d.nc >= 3 && rmax <= d.L / d.nc - c->p.skin;
  if (!by_cells && d.n > 262144)
    return fail(c, MD_EINVAL,
                "md_rdf: rmax above the cell side minus the skin needs a replica of at most "
                "262144 particles");
  if (by_cells && !c->built) {
    if (!may_build) return fail(c, MD_ESTATE, "md_rdf_static: cells not built");
    md_status b = build_all(c);
    if (b) return b;
  }
  launch_zero_u64(c->stream, hist, nbins);
  if (by_cells)
    launch_rdf_cells(c->stream, d.coff, d.nc, c->cell_start, c->pos, d.L, rmax, nbins, hist);
  else
    launch_rdf(c->stream, c->pos, d.off, d.n, d.L, rmax, nbins, hist);
  HIPCHECK(c, hipGetLastError());
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  HIPCHECK(c, hipMemcpy(g, hist, sizeof(unsigned long long) * nbins, hipMemcpyDeviceToHost));
  const double dr = rmax / nbins, V = d.L * d.L * d.L, n = (double)d.n;
  const double pi = 3.14159265358979323846;
  for (int32_t b = 0; b < nbins; ++b) {
    unsigned long long h;
    std::memcpy(&h, &g[b], sizeof h);
    const double r0 = b * dr, r1 = (b + 1) * dr;
    const double shell = 4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0);
    g[b] = 2.0 * V * (double)h / (n * n * shell);
  }
  return MD_OK;
}

md_status rdf_args(md_ctx c, int32_t rep, double rmax, int32_t nbins, const double* g) {
  if (rep < 0 || rep >= c->nrep) return fail(c, MD_EINVAL, "replica index out of range");
  if (!c->has_state) return fail(c, MD_ESTATE, "no state set");
  const RepDesc& d = c->reps_h[rep];
  if (!g || nbins < 1 || nbins > kStaticBins || !(rmax > 0.0) || rmax > 0.5 * d.L)
    return fail(c, MD_EINVAL, "need g, 1 <= nbins <= 8192 and 0 < rmax <= L/2");
  return MD_OK;
}
}  // namespace

md_status md_rdf(md_ctx c, int32_t rep, double rmax, int32_t nbins, double* g) {
  if (!c) return MD_EINVAL;
  md_status rc = rdf_args(c, rep, rmax, nbins, g);
  if (rc) return rc;
  unsigned long long* hist = nullptr;
  rc = dalloc(c, &hist, (size_t)nbins);
  if (rc) return rc;
  rc = rdf_with(c, rep, rmax, nbins, g, hist, true);
  dfree(c, hist);
  return rc;
}

md_status md_rdf_static(md_ctx c, int32_t rep, double rmax, int32_t nbins, double* g) {
  if (!c) return MD_EINVAL;
  md_status rc = rdf_args(c, rep, rmax, nbins, g);
  if (rc) return rc;
  unsigned long long* hist = scratch_dev(c->device);
  if (!hist) return fail(c, MD_EHIP, "md_rdf_static: no scratch address for this device");
  return rdf_with(c, rep, rmax, nbins, g, hist, false);
}

md_status md_list_stats(md_ctx c, int32_t rep, double* mean, int32_t* max) {
  if (!c) return MD_EINVAL;
  if (c->cells) return fail(c, MD_ESTATE, "the cell path keeps no neighbour list");
  if (rep < -1 || rep >= c->nrep) return fail(c, MD_EINVAL, "replica index out of range");
  if (!c->built) return fail(c, MD_ESTATE, "list not built");
  md_status rc = sync_and_check(c);
  if (rc) return rc;
  const int32_t off = rep < 0 ? 0 : c->reps_h[rep].off;
  const int32_t n = rep < 0 ? c->ntot : c->reps_h[rep].n;
  std::vector<int32_t> cnt(n);
  HIPCHECK(c, hipMemcpy(cnt.data(), c->ncount + off, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  int64_t sum = 0;
  int32_t m = 0;
  for (int32_t v : cnt) {
    sum += v;
    m = std::max(m, v);
  }
  if (mean) *mean = (double)sum / (double)n;
  if (max) *max = m;
  return MD_OK;
}

}  // extern "C"
