// md_internal.h -- device data layout and kernel launchers of libmd (gfx950).
//
// Layout in HBM (particle arrays are in cell order, "sorted index" i):
//   pos   double4[Ntot]        x, y, z, species (as a double); 32 B records
//                              so one neighbour gather is two 16 B loads
//   vel   double [3][stride]   SoA velocities
//   frc   double or float [3][stride]  SoA forces
//   xref  double [3][stride]   positions at the last list build (skin check)
//   id    int32  [Ntot]        original (caller) index of sorted particle i
//   img   int32  [Ntot][3]     periodic image counters, ORIGINAL id order
//   nbr   uint32 [cap][stride] neighbour list, ELL (slot-major) so that a
//                              wave reading slot k of 64 consecutive
//                              particles touches one 256 B line; an entry is
//                              (sorted j) | (image code << 26)
// Cells: replica r owns cells [coff_r, coff_r + nc_r^3); cell_start holds
// global particle offsets.  Particles of a replica stay in its range.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/md.h"

namespace mdk {

constexpr int kTile = 256;          // particles per tile == threads per block
constexpr int kIdxBits = 26;        // neighbour index bits
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;

// error word bits (latched on the device, read at synchronising calls)
enum : int32_t {
  kErrNonFinite = 1,
  kErrOverflow = 2,   // a neighbour row longer than the list capacity
  kErrStray = 4,
  kErrType = 8,
  kErrSlots = 16,     // staged path: a tile neighbourhood beyond the 14-bit slots
};
// A list build that overflowed halts the rest of the queued step sequence:
// the force, reduction, kick and rescale kernels read this mask first and
// return at once, and the first halted force launch clears any_rebuild so
// the rebuild chains of the later queued steps exit too.  The state is left
// as the overflowing build made it (drifted, wrapped and re-sorted positions,
// half-kicked velocities); the host grows the capacity and finishes the
// interrupted step from there.
constexpr int32_t kHalt = kErrOverflow | kErrSlots;

// Neighbour lists are stored as sliced ELL: slice s holds particles
// [256 s, 256 s + 256) and stores its cap rows one after another, row k
// holding entry k of the slice's 256 particles.  A wave reading entry k of
// consecutive particles reads contiguous memory, and the whole list of a
// slice is one contiguous block (a few pages even for very large systems).
constexpr int32_t kSlice = 256;
__host__ __device__ inline size_t list_base(int32_t i, int32_t cap) {
  return (size_t)(i >> 8) * (size_t)cap * kSlice + (size_t)(i & (kSlice - 1));
}
inline size_t list_elems(int32_t ntot, int32_t cap) {
  return (size_t)((ntot + kSlice - 1) / kSlice) * kSlice * (size_t)cap;
}

struct Tile {          // a run of <= kTile particles of one replica
  int32_t rep;
  int32_t start;
  int32_t end;
  int32_t pad;
};

struct RepDesc {       // per-replica geometry, device resident
  double L;
  double inv_cell;     // nc / L, correctly rounded on the host
  double half_skin2;   // (skin / 2)^2
  double dof;          // 3 n - 3
  double volume;
  int32_t off, n;      // particle range
  int32_t coff, nc;    // first cell, cells per side
  int32_t tile0, tile1;// tiles [tile0, tile1)
  int32_t fb0, fb1;    // force-kernel partial blocks [fb0, fb1) of this replica
  int32_t cb0, cb1;    // reduction chunks [cb0, cb1) (two-level reduction only)
  double cside;        // cell side L / nc
  double qs, qinv;     // mixed records: fixed-point scale 2^s and 2^-s (make_recq)
};

// Mixed form gather record of a particle (16 B): the offsets from the centre
// of the cell it was binned into at the last list build, (c + 1/2) * cside
// formed in FP64, as 32-bit fixed-point integers in units of 2^-s (qinv; s
// per replica so that every offset a record can hold -- half a cell side
// plus the skin and one step's drift -- stays below 2^30 units: 2^-28 =
// 3.7e-9 for the LJ workloads), and a word holding the cell coordinates (10
// bits each, for the record updates of the drift) and the species (bits
// 30-31).  With s the periodic image of a listed pair, x_i - (x_j + s L)
// equals
//   (off_i - off_j) + (c_i - c_j - s nc) * cside
// exactly; mixed lists carry d = c_i - c_j - s nc in {-1, 0, 1}^3, and the
// force kernel forms the displacement in FP64 from the exact integer offset
// difference and d * cside, then does the pair arithmetic in FP32.  (FP32
// offsets rounded the displacement to 6e-8 of the cell side, which the pair
// force's stiffness turned into most of the mixed form's force error.)
__device__ inline uint32_t pack_cell(int32_t cx, int32_t cy, int32_t cz, int32_t t) {
  return (uint32_t)cx | ((uint32_t)cy << 10) | ((uint32_t)cz << 20) | ((uint32_t)t << 30);
}
__device__ inline int32_t to_fixed(double u) {
  // |u| beyond 2^30 units only in a step whose skin check rebuilds the record
  // before any force launch reads it; clamped to stay defined
  u = u > 1073741824.0 ? 1073741824.0 : (u < -1073741824.0 ? -1073741824.0 : u);
  return __double2int_rn(u);
}
__device__ inline int4 make_recq(double x, double y, double z, uint32_t w, double cside,
                                 double qs) {
  const int32_t cx = (int32_t)(w & 1023u), cy = (int32_t)((w >> 10) & 1023u),
                cz = (int32_t)((w >> 20) & 1023u);
  return make_int4(to_fixed((x - ((double)cx + 0.5) * cside) * qs),
                   to_fixed((y - ((double)cy + 0.5) * cside) * qs),
                   to_fixed((z - ((double)cz + 0.5) * cside) * qs), (int32_t)w);
}

// Per species pair ab = a * 4 + b.  The pair function Eq. (3) is written as
//   V*(r) = c12 (s/r)^12 + c6 (s/r)^6 - vc - (r - rc) fs
//   f(r)/r = (f12 (s/r)^12 + f6 (s/r)^6) / r^2 + fs / r
// with c6 = 0 for the soft sphere Eq. (2) and fs = 0 for a plain energy shift.
struct PairTab {
  double rc2[16];      // force cutoff squared
  double thr[16];      // list threshold (rc + skin)^2
  double sig2[16];
  double c12[16], c6[16], f12[16], f6[16];
  double vc[16];       // V(rc)
  double fs[16];       // V'(rc) (shifted force) or 0
  double rc[16];
  double inv_mass[4];
  double mass[4];
};

// The hardware deals consecutive workgroups of a launch round-robin to the 8
// XCDs, each with its own L2.  Renumber blocks so that XCD x runs one
// contiguous run of logical blocks: neighbouring tiles (which gather the same
// neighbour positions) then share an L2.  Bijective for any grid size.
constexpr int kXcd = 8;
__device__ inline int32_t xcd_block(int32_t b, int32_t nb) {
  const int32_t q = nb / kXcd, r = nb % kXcd;
  const int32_t x = b % kXcd, k = b / kXcd;
  return x * q + (x < r ? x : r) + k;
}

// Block order of the rebuild chain in contexts with several replicas: the
// work there is gated per replica, and xcd_block would put a rebuilding
// replica's contiguous block range on one or two XCDs while the others idle.
// Here groups of g consecutive logical blocks are dealt round-robin to the
// XCDs instead (a group still shares an L2).  Bijective on a grid that is a
// multiple of kXcd * g (spread_grid); logical blocks past the real count exit.
__device__ inline int32_t xcd_spread(int32_t b, int32_t g) {
  const int32_t x = b % kXcd, k = b / kXcd;
  return ((k / g) * kXcd + x) * g + (k % g);
}
inline int32_t spread_grid(int32_t nb, int32_t g) {
  const int32_t m = kXcd * g;
  return (nb + m - 1) / m * m;
}

// The force kernel reads the list with non-temporal loads when one replica's
// list (capacity) exceeds this: about 1.5x the 256 MB last-level (Infinity)
// cache, a list that would not stay cached between launches anyway.  Smaller
// lists -- small boxes, short soft-sphere lists, and the replicas of a batch,
// which are processed a few at a time -- are read normally and hit that
// cache from one step to the next (measured both ways: +2 % per step for the
// 1M-particle LJ box with streaming, -3 % for 256 replicas, -12 % for the 1M
// soft-sphere box).
constexpr size_t kStreamListBytes = (size_t)384 << 20;

struct DevState {      // context scalars the kernels update
  int32_t err;
  int32_t any_rebuild;
  int32_t pad[2];
};
__device__ inline bool halted(const DevState* st) { return (st->err & kHalt) != 0; }

// ---- launchers (each file owns its kernels) ----------------------------------
// cells.hip
void launch_set_state(hipStream_t s, int32_t ntot, int32_t stride, const double* x,
                      const double* v, const int32_t* type, int32_t ntypes,
                      double4* pos, double* vel, int32_t* id, int32_t* img, DevState* st);
void launch_get_state(hipStream_t s, int32_t ntot, int32_t stride, const double4* pos,
                      const double* vel, const int32_t* id, double* x, double* v);
void launch_get_forces(hipStream_t s, int32_t ntot, int32_t stride, const void* frc,
                       int32_t mixed, const int32_t* id, void* F);
void launch_mark_rebuild(hipStream_t s, int32_t nrep, int32_t* rebuild, DevState* st);
// Copy every particle's first min(ncount, cap_old) list entries from the
// sliced-ELL layout of capacity cap_old to that of capacity cap_new (elem 2
// or 4 bytes), when the capacity grows.
void launch_relayout_list(hipStream_t s, int32_t ntot, const int32_t* ncount, int32_t cap_old,
                          int32_t cap_new, int32_t elem, const void* src, void* dst);
void launch_zero_counts(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const int32_t* rebuild, const DevState* st, int32_t* counts);
void launch_bin(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                const int32_t* rebuild, double4* pos, const int32_t* id, int32_t* img,
                int32_t* counts, int32_t* cell_of, int32_t* slot, DevState* st, int32_t spread);
void launch_scan(hipStream_t s, int32_t ncells, const int32_t* counts, int32_t* cell_start,
                 int32_t* bsum, const DevState* st);
size_t scan_bsum_elems(int32_t ncells);
void launch_scatter(hipStream_t s, int32_t ntiles, const Tile* tiles, const int32_t* rebuild,
                    const int32_t* cell_of, const int32_t* slot, const int32_t* cell_start,
                    int32_t* tmp_src, const DevState* st, int32_t spread);
// One-block form of the chain above (zero, bin, scan, scatter, gather) for a
// context of one replica with at most kSmallN particles and kSmallCells
// cells; the same cell_start and records, in one launch.  (At 16,384
// particles the block's serial walk over 16 particles per thread already
// cost more than the three launches it saves.)
constexpr int kSmallThreads = 1024;
constexpr int kSmallN = 8192;
constexpr int kSmallCells = 4 * kSmallThreads;  // the scan takes four cells per thread
void launch_chain_small(hipStream_t s, const RepDesc* reps, const int32_t* rebuild,
                        double4* pos, const int32_t* id, int32_t* img, int32_t* cell_start,
                        int32_t stride, const double* vel, int32_t* id_tmp, double4* pos_tmp,
                        double* vel_tmp, DevState* st);
void launch_cell_gather(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const int32_t* rebuild, const int32_t* cell_start,
                        const int32_t* tmp_src, int32_t stride, const int32_t* id,
                        const double4* pos, const double* vel, int32_t* id_tmp,
                        double4* pos_tmp, double* vel_tmp, const DevState* st);
// Form of a symmetric species-pair table t[a * 4 + b] (a, b < ntypes) in the
// cut-off tests: 2 when every entry is t[0][b] + (t[1][b] - t[0][b]) * s_a
// for the species value s_a in {0.0, 1.0} as one FMA, bit for bit -- one
// species, or two whose entries for each b lie within a factor of two (then
// t[1][b] - t[0][b] is exact, Sterbenz); 4 otherwise (a select chain).
inline int32_t fma_pair_form(const double* t, int32_t ntypes) {
  if (ntypes == 1) return 2;  // s_a = 0 only: fma(d, 0, t0) = t0 for any finite d
  if (ntypes > 2) return 4;
  for (int b = 0; b < 2; ++b) {
    const double t0 = t[b], t1 = t[4 + b];
    if (!(t0 * 0.5 <= t1 && t1 <= 2.0 * t0)) return 4;
  }
  return 2;
}
// nlist.hip.  thr_form: fma_pair_form of the list thresholds.  spread: 0, or
// the number of consecutive cells whose blocks share an XCD (see xcd_spread).
void launch_nlist(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                  const int32_t* rebuild, const PairTab* tab, int32_t thr_form,
                  const int32_t* cell_start, int32_t stride, int32_t cap,
                  const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                  double4* pos, double* vel, int32_t* id, double* xref,
                  uint32_t* nbr, int32_t* ncount, DevState* st, int32_t ncells,
                  const int32_t* cell_rep, int32_t any_single, int32_t any_multi,
                  int4* pos16, int32_t spread);
// The gather-path search of a one-replica context with at most
// kSmallListN particles and >= 3 cells per side: the rows of launch_nlist
// bit for bit, 32 lanes per home particle instead of one wave per cell.
// (From ~16,000 particles on the box has cells enough for the one-wave-per-
// cell search to fill the chip: at 32,000 it is the faster one.)
constexpr int kSmallListN = 16384;
void launch_nlist_small(hipStream_t s, int32_t ntot, const RepDesc* reps,
                        const int32_t* rebuild, const PairTab* tab, const int32_t* cell_start,
                        int32_t stride, int32_t cap, const double4* pos_tmp,
                        const double* vel_tmp, const int32_t* id_tmp, double4* pos, double* vel,
                        int32_t* id, double* xref, uint32_t* nbr, int32_t* ncount, DevState* st,
                        int4* pos16);
// force.hip
// mode 0: forces + PE/W + KE of the current v;  mode 1: also the second
// half kick v += dt/2 F/m before KE, and PE/W only when energy != 0;
// mode 2: mode 1, then the next step's half kick and drift (FuseOut).
// unroll: list slots gathered per pipelined chunk (1, 2, 4 or 8).
// stream_list: read the list with non-temporal loads (lists larger than the
// last-level cache; see kStreamListBytes).
// Outputs of the force kernel's mode 2 (the next step's kick and drift
// fused into an NVE step): the drifted positions (the other buffer of the
// position pair), the list-build positions for the skin check, and the cell
// histogram to clear (nzero cells; 0 = none).  Unused by modes 0 and 1.
struct FuseOut {
  double4* pos_out;
  int4* pos16_out;
  const double* xref;
  int32_t* counts;
  int32_t nzero;
};
void launch_force(hipStream_t s, int32_t mixed, int32_t mode, int32_t energy,
                  int32_t stream_list, int32_t tpp,
                  int32_t unroll, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                  const PairTab* tab, const double4* pos, const int4* pos16, double* vel,
                  void* frc, const uint32_t* nbr, const int32_t* ncount, int32_t stride,
                  int32_t cap, double dt, double* part, DevState* st, const FuseOut& fo);
// integrate.hip
void launch_kick_drift(hipStream_t s, int32_t mixed, int32_t thermo, int32_t ntiles,
                       const Tile* tiles, const RepDesc* reps, const PairTab* tab,
                       double4* pos, int4* pos16, double* vel, const void* frc,
                       const double* xref, int32_t stride, double dt, const double* lam,
                       int32_t* rebuild, double* dmax, DevState* st, int32_t* counts,
                       int32_t nzero);
struct ThermoArgs {
  const double* T0;    // [nrep]
  const double* T1;    // [nrep]
  int64_t ramp;
  int32_t thermo;      // 0 = NVE
  int32_t log_every;   // 0 = no log
  md_obs* log;         // [nlog][nrep]
  int32_t nlog;
  int32_t pad;
};
// First level of the two-level reduction (large replicas): chunk c sums the
// partial triples [b0, b1), takes the maximum of the drift tile maxima
// [t0, t1) and, with next = 1, of the fourth partials [b0, b1) (the next
// step's drift measured by a fused force launch) into part2[kPart2 c + k],
// k = 0..4 (pe, w, ke, tile maximum, next maximum).
struct RedChunk {
  int32_t b0, b1, t0, t1;
};
constexpr int32_t kRedChunk = 1024;  // partial blocks per chunk
constexpr int32_t kPart2 = 8;        // doubles per chunk result
void launch_reduce_chunks(hipStream_t s, int32_t nchunks, const RedChunk* ch, const double* part,
                          const double* dmax, int32_t step, int32_t next, double* part2,
                          const DevState* st);
// Where a step's drift maximum comes from and what the reduction does with
// the rebuild flag (one replica per context when next = 1):
// src = 0: the kick/drift tile maxima in dmax; src = 1: pend[r], stored by
// the previous step's reduction.  next = 0: the flag is cleared at the end
// of the step (the next kick sets it again); next = 1: this step's force
// launch drifted the positions of the next step (force mode 2), so the flag
// is set from that drift (pend[r] keeps it for the next step's observables).
struct DriftArgs {
  int32_t src;
  int32_t next;
  double* pend;
};
// step = 0: observables of the current state only; step = 1: end of a step
// part holds one (pe, w, ke, next drift) quadruple per force block; replica
// r owns blocks [fb0, fb1).  dmax holds the kick/drift tile maxima of
// |x - x_ref|^2 (tiles [tile0, tile1) of replica r), read when step = 1 and
// drift.src = 0.  With part2 != NULL the per-replica pass reads the chunk
// results part2[kPart2 c + k], c in [cb0, cb1), instead of part and dmax.
// energy = 0: the step formed no PE/W; pe, virial, P and E keep their last
// values.
void launch_reduce(hipStream_t s, int32_t nrep, const RepDesc* reps, const double* part,
                   const double* dmax, const double* part2, int32_t step, int32_t energy,
                   DriftArgs drift, ThermoArgs ta, int64_t* kcall, double* lam, int32_t* rebuild,
                   md_obs* obs, DevState* st);
void launch_after_build(hipStream_t s, int32_t nrep, int32_t* rebuild, md_obs* obs,
                        DevState* st);
void launch_begin_call(hipStream_t s, int32_t nrep, int64_t* kcall, double* lam);
void launch_apply_lambda(hipStream_t s, int32_t ntiles, const Tile* tiles, int32_t stride,
                         double* vel, double* lam, int32_t nrep, const DevState* st);

// analysis.hip
void launch_msd_ref(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                    const double4* pos, const int32_t* id, const int32_t* img, double* u0);
void launch_msd(hipStream_t s, int32_t ntiles, int32_t nrep, const Tile* tiles,
                const RepDesc* reps, const double4* pos, const int32_t* id, const int32_t* img,
                const double* u0, double* part, double* out);
void launch_rdf(hipStream_t s, const double4* pos, int32_t off, int32_t n, double L, double rmax,
                int32_t nbins, unsigned long long* hist);
// a[0, n) = 0 (a fill kernel rather than hipMemsetAsync, so callers may
// capture it in a graph)
void launch_zero_u64(hipStream_t s, unsigned long long* a, int32_t n);
void launch_rdf_cells(hipStream_t s, int32_t c0, int32_t nc, const int32_t* cell_start,
                      const double4* pos, double L, double rmax, int32_t nbins,
                      unsigned long long* hist);

// staged path (stage.h, nlist.hip tile mode, force_staged.hip)
struct RowTile;
size_t force_staged_lds_bytes(int32_t lcap);
int32_t staged_homes_per_group();
void launch_nlist_tiles(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const RepDesc* reps, const int32_t* rebuild, const PairTab* tab,
                        int32_t thr_form, const int32_t* cell_start, int32_t stride, int32_t cap,
                        const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                        double4* pos, double* vel, int32_t* id, double* xref, uint16_t* nbr16,
                        int32_t* ncount, DevState* st, const int32_t* cell_tile,
                        const RowTile* rtiles, int32_t spread);
void launch_decode_staged(hipStream_t s, int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                          const int32_t* cell_start, int32_t cap, const uint16_t* nbr,
                          const int32_t* ncount, uint32_t* out);
// list-free cell path (force_cells.hip)
int32_t cells_homes_per_block();
// rc2_form: fma_pair_form of the squared force cutoffs.
void launch_force_cells(hipStream_t s, int32_t mixed, int32_t mode, int32_t rc2_form,
                        int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                        const PairTab* tab, const int32_t* cell_start, const double4* pos,
                        double* vel, void* frc, int32_t stride, double dt, double* part,
                        DevState* st);
void launch_commit_order(hipStream_t s, int32_t ntiles, const Tile* tiles,
                         const int32_t* rebuild, int32_t stride, const double4* pos_tmp,
                         const double* vel_tmp, const int32_t* id_tmp, double4* pos,
                         double* vel, int32_t* id, double* xref, const DevState* st);
void launch_force_staged(hipStream_t s, int32_t mixed, int32_t mode, int32_t tpp, int32_t unroll,
                         int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                         const PairTab* tab, const int32_t* cell_start, const double4* pos,
                         double* vel, void* frc, const uint16_t* nbr, const int32_t* ncount,
                         int32_t stride, int32_t cap, int32_t lcap, double dt, double* part,
                         DevState* st);

}  // namespace mdk
