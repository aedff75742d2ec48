// nlist.hip -- cut-off neighbour search over the 27-cell stencil.
//
// The paper finds interacting pairs with a linked-cell grid search over
// neighbouring cubic cells ("Grid-search method", Fig. 1).  Here the same
// search fills a full (both directions) neighbour list with a skin, so the
// force kernel can reuse it for several steps.  The inclusion test must give
// exactly the same set as a plain FP64 evaluation of
//     d = (x_j - x_i) + s L,  r^2 = (dx dx + dy dy) + dz dz  <  (rc_ab + skin)^2
// (exchanging i and j negates every step exactly: the test is symmetric)
// so this file is compiled without FMA contraction (also forced below).
//
// List entry: sorted index j (26 bits) | a 6-bit code, two bits per axis in
// two's complement.  FP64 lists: the periodic image s in {-1, 0, 1} of the
// partner (x_j + s L), so an entry without a shift is the plain index.
// Mixed lists: the cell offset d = c_i - c_j - s nc in {-1, 0, 1} between
// the build-time cells of the pair, which turns the 16-byte cell-relative
// records into the displacement (off_i - off_j) + d * cell side (see
// make_recq) with no further decoding.
#include "stage.h"

#pragma clang fp contract(off)

namespace mdk {
namespace {

__device__ inline void stencil_axis(int32_t q, int32_t o, int32_t nc, int32_t& qn, int32_t& s) {
  int32_t t = q + o;
  s = 0;
  if (t < 0) {
    t += nc;
    s = -1;
  } else if (t >= nc) {
    t -= nc;
    s = 1;
  }
  qn = t;
}

__device__ inline uint32_t image_code(int32_t sx, int32_t sy, int32_t sz) {
  return ((uint32_t)(sx & 3) | ((uint32_t)(sy & 3) << 2) | ((uint32_t)(sz & 3) << 4))
         << kIdxBits;
}

__device__ inline int32_t cell_coord(double c, double inv_cell, int32_t nc) {
  int32_t q = (int32_t)(c * inv_cell);
  return q > nc - 1 ? nc - 1 : q;
}

// One-cell boxes (nc = 1): every other particle of the replica is tested
// with the minimum image  d - L nearbyint(d / L).
__global__ __launch_bounds__(kTile) void k_nlist(
    const Tile* __restrict__ tiles, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ rebuild, const PairTab* __restrict__ tab, int32_t stride,
    int32_t cap, const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref, uint32_t* __restrict__ nbr,
    int32_t* __restrict__ ncount, DevState* st, int32_t dcode, int4* __restrict__ pos16) {
  __shared__ double s_thr[16];
  if (!st->any_rebuild) return;
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  __syncthreads();
  const Tile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
  if (!rebuild[t.rep]) return;
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  const RepDesc R = reps[t.rep];
  if (R.nc != 1) return;  // cell grids: k_nlist_cells
  const double4 p = pos_tmp[i];
  const int32_t ti = (int32_t)p.w;
  const double* thr = &s_thr[ti * 4];
  int32_t cnt = 0;
  uint32_t* out = nbr + list_base(i, cap);
  for (int32_t j = R.off; j < R.off + R.n; ++j) {
    if (j == i) continue;
    const double4 q = pos_tmp[j];
    double ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
    double kx = rint(ex / R.L), ky = rint(ey / R.L), kz = rint(ez / R.L);
    double tx = R.L * kx, ty = R.L * ky, tz = R.L * kz;
    ex = ex - tx;
    ey = ey - ty;
    ez = ez - tz;
    double r2 = (ex * ex + ey * ey) + ez * ez;
    if (r2 < thr[(int32_t)q.w]) {
      // image s = -k; with one cell d = -s nc = k
      const int32_t sx = -(int32_t)kx, sy = -(int32_t)ky, sz = -(int32_t)kz;
      const uint32_t code = dcode ? image_code(-sx, -sy, -sz) : image_code(sx, sy, sz);
      if (cnt < cap) out[(size_t)cnt * kSlice] = (uint32_t)j | code;
      ++cnt;
    }
  }
  ncount[i] = cnt;
  if (cnt > cap) atomicOr(&st->err, kErrOverflow);
  // the new cell order becomes the live state; the list is built on it
  if (pos16) {
    const uint32_t wc = pack_cell(cell_coord(p.x, R.inv_cell, R.nc), cell_coord(p.y, R.inv_cell, R.nc),
                                  cell_coord(p.z, R.inv_cell, R.nc), ti);
    pos16[i] = make_recq(p.x, p.y, p.z, wc, R.cside, R.qs);
  }
  pos[i] = p;
  xref[i] = p.x;
  xref[stride + i] = p.y;
  xref[2 * (size_t)stride + i] = p.z;
  vel[i] = vel_tmp[i];
  vel[stride + i] = vel_tmp[stride + i];
  vel[2 * (size_t)stride + i] = vel_tmp[2 * (size_t)stride + i];
  id[i] = id_tmp[i];
}


// One wave per home cell (nc >= 3), in two phases per group of at most
// kCwGroup home particles.
//
// Test phase: the candidates of the cell -- the 27 stencil cells as single
// contiguous particle ranges (gather path: the home cell, then pairs of
// mirror cells o, -o), or the 9 neighbour rows of one to three
// ranges each (staged path), with their periodic shift -- are packed 64 to a
// chunk, one candidate per lane.
// For every home particle (wave-uniform loop, coordinates through scalar
// loads) each lane tests its candidate.  The ballot of the hits is the whole
// result: its two 32-bit words go to lane h of two registers (one
// v_writelane each) and, once per chunk, to LDS beside the chunk's list
// entries.  Nothing is done per hit.
//
// Write phase: lane h walks the set bits of home h's words in candidate
// order, the t-th bit giving the home's t-th list entry.  The lanes go in
// lock step, so iteration t stores entry t of every home of the group: row t
// of the sliced list, a contiguous segment for the group's consecutive
// particles, written whole in one store.
//
// A neighbourhood of more than kCwChunks * 64 candidates is taken in passes;
// the rows of a later pass start at each home's running count (the stores of
// such a pass are scattered; correct, and rare at the cell sizes used).
// Copying the new order into the live arrays is done here as well.
constexpr int kCwGroup = 32;   // home particles per group (lanes of the write phase)
constexpr int kCwHomes = 4;    // home particles tested per iteration
constexpr int kCwChunks = 12;  // candidate chunks per pass (768 candidates, 6 KB of LDS)
constexpr int kCwWaves = 4;    // waves (cells) per block: a launch with nothing to rebuild
                               // costs its block count; one or two cells per block measured
                               // slower both idle and building
constexpr double kFar = 1.0e300;  // x of the idle lanes of a chunk: r^2 overflows to +inf
static_assert(kCwGroup == 32, "the write phase gives each home two lanes of the wave");
static_assert(kCwHomes == 3 || kCwHomes == 4,
              "the home loop leaves at most one block of 2 and one of 1");

// lo[l + u] = low word of m[u], hi[l + u] = high word, for the wave-uniform
// lane l and u < U: v_writelane with the lane in M0 (the clang in use has no
// builtin for it, and a lane select in another scalar register would break
// the one-scalar-operand limit), M0 stepped between the pairs.  Lanes not
// written keep their values.  The m[u] are usually the scalar results of the
// vector compares just before; the compiler inserts no wait states inside
// inline asm, so the block starts with the longest one a lane operation needs
// after a vector write of a scalar register it reads (one wait for all U).
template <int U>
__device__ inline void write_lanes(uint32_t& lo, uint32_t& hi, const uint64_t (&m)[U], int32_t l) {
#define MDK_WL(a, b) "v_writelane_b32 %0, %" #a ", m0\n\tv_writelane_b32 %1, %" #b ", m0"
#define MDK_S(u) "s"((uint32_t)m[u]), "s"((uint32_t)(m[u] >> 32))
  if constexpr (U == 1) {
    asm volatile("s_nop 4\n\t" MDK_WL(3, 4) : "+v"(lo), "+v"(hi), "+{m0}"(l) : MDK_S(0));
  } else if constexpr (U == 2) {
    asm volatile("s_nop 4\n\t" MDK_WL(3, 4) "\n\ts_add_u32 m0, m0, 1\n\t" MDK_WL(5, 6)
                 : "+v"(lo), "+v"(hi), "+{m0}"(l)
                 : MDK_S(0), MDK_S(1)
                 : "scc");
  } else if constexpr (U == 3) {
    asm volatile("s_nop 4\n\t" MDK_WL(3, 4) "\n\ts_add_u32 m0, m0, 1\n\t" MDK_WL(5, 6)
                 "\n\ts_add_u32 m0, m0, 1\n\t" MDK_WL(7, 8)
                 : "+v"(lo), "+v"(hi), "+{m0}"(l)
                 : MDK_S(0), MDK_S(1), MDK_S(2)
                 : "scc");
  } else {
    static_assert(U == 4, "blocks of 1 to 4 homes");
    asm volatile("s_nop 4\n\t" MDK_WL(3, 4) "\n\ts_add_u32 m0, m0, 1\n\t" MDK_WL(5, 6)
                 "\n\ts_add_u32 m0, m0, 1\n\t" MDK_WL(7, 8) "\n\ts_add_u32 m0, m0, 1\n\t"
                 MDK_WL(9, 10)
                 : "+v"(lo), "+v"(hi), "+{m0}"(l)
                 : MDK_S(0), MDK_S(1), MDK_S(2), MDK_S(3)
                 : "scc");
  }
#undef MDK_S
#undef MDK_WL
}

// LDS written by some lanes of the wave and read by others: order the
// accesses (the LDS unit serves one wave's operations in issue order).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cut-off threshold of the pair (home species a, lane's candidate species b),
// with the home's species value wa (0.0, 1.0, ...) wave-uniform.
// NT = 2: thr = t0 + (t1 - t0) wa as one fused multiply-add.  The launch picks
// this form only when t1 / 2 <= t0 <= 2 t1 for every b, so d = t1 - t0 is
// exact (Sterbenz) and fma(d, 1, t0) = t1, fma(d, 0, t0) = t0 are the
// tabulated values bit for bit.  NT = 4: a select chain on the high word of
// wa (0.0, 1.0, 2.0, 3.0 have distinct high words).
template <int NT>
__device__ inline double pick_thr(double wa, double t0, double d, double t1, double t2,
                                  double t3) {
  if constexpr (NT == 2) {
    return __builtin_fma(d, wa, t0);
  } else {
    const int32_t hi = __double2hiint(wa);
    return hi == 0 ? t0 : (hi == 0x3ff00000 ? t1 : (hi == 0x40000000 ? t2 : t3));
  }
}

// TILE = false: entries are sorted index | image code (uint32, gather path).
// TILE = true: entries are the partner's LDS slot in the staged neighbourhood
// of the row tile holding the home cell (stage.h) | species << 14 (uint16,
// staged path); the slot of a candidate is its piece's first slot in that
// layout plus its offset inside the piece.
template <int HPI, bool TILE, int NT>
__global__ __launch_bounds__(64 * kCwWaves) void k_nlist_cells(
    int32_t ncells, const int32_t* __restrict__ cell_rep, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ rebuild, const PairTab* __restrict__ tab,
    const int32_t* __restrict__ cell_start, int32_t stride, int32_t cap,
    const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref,
    typename std::conditional<TILE, uint16_t, uint32_t>::type* __restrict__ nbr,
    int32_t* __restrict__ ncount, DevState* st, int4* __restrict__ pos16,
    const int32_t* __restrict__ cell_tile, const RowTile* __restrict__ rtiles, int32_t dcode,
    int32_t spread) {
  using E = typename std::conditional<TILE, uint16_t, uint32_t>::type;
  __shared__ double s_thr[16];
  __shared__ int32_t s_pre[kCwWaves][28];    // first packed candidate of piece p
  __shared__ int32_t s_k0[kCwWaves][27];     // first sorted index of piece p
  __shared__ int32_t s_code[kCwWaves][27];   // image code of piece p (shift -1/0/1 per axis)
  __shared__ int32_t s_l0[kCwWaves][27];     // TILE: first LDS slot of piece p in the tile layout
  __shared__ int32_t s_rowsz[kCwWaves][9];   // TILE: slots of tile row q
  __shared__ int32_t s_ecode[kCwWaves][27];  // gather path: entry code of piece p's particles
  __shared__ uint32_t s_ent[kCwWaves][kCwChunks * 64];              // entry of each candidate
  // [word][home] hit bits, and one word more that the write phase's read-ahead
  // may touch past the last word of a full pass (its value is never used)
  __shared__ uint32_t s_hits[kCwWaves][(2 * kCwChunks + 1) * kCwGroup];
  if (!st->any_rebuild) return;  // whole block: one flag load when nothing rebuilds
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  __syncthreads();
  // the wave index is wave-uniform; as a scalar, the per-cell values below are too
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int32_t c =
      (spread ? xcd_spread(blockIdx.x, spread) : xcd_block(blockIdx.x, gridDim.x)) * kCwWaves + w;
  if (c >= ncells) return;
  const int32_t r = cell_rep[c];
  if (!rebuild[r]) return;
  const RepDesc R = reps[r];
  if (R.nc == 1) return;  // minimum-image kernel
  const int32_t nc = R.nc;
  const int32_t lc = c - R.coff;
  const int32_t qx = lc % nc, qy = (lc / nc) % nc, qz = lc / (nc * nc);
  const int32_t h0 = cell_start[c], nh = cell_start[c + 1] - h0;
  uint32_t* const ent = s_ent[w];
  uint32_t* const hits = s_hits[w];

  int32_t own_slot = 13;  // piece holding the home cell's particles
  if constexpr (!TILE) {
    // gather path: the 27 cells as single-cell pieces, the home cell first,
    // then each forward offset o (in (dz, dy, dx) order) followed by its
    // mirror -o; lane q < 27 builds offset q.  A particle's place in its
    // cell moves hits between o and -o but hardly changes their sum, so
    // after every pair the particles of a wave have used about the same
    // number of entries, and the force kernel's gathers at one entry index
    // fall in the same cells more often than with rows in (dz, dy, dx) order.
    if (lane < 27) {
      const int32_t ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
      int32_t nx, sx, ny, sy, nz, sz;
      stencil_axis(qx, ox, nc, nx, sx);
      stencil_axis(qy, oy, nc, ny, sy);
      stencil_axis(qz, oz, nc, nz, sz);
      const int32_t cn = R.coff + (nz * nc + ny) * nc + nx;
      const int32_t slot = lane == 13 ? 0 : (lane > 13 ? 2 * (lane - 13) - 1 : 2 * (13 - lane));
      s_k0[w][slot] = cell_start[cn];
      s_pre[w][slot] = cell_start[cn + 1] - cell_start[cn];  // lengths for now
      const uint32_t code = image_code(sx, sy, sz);
      s_code[w][slot] = (int32_t)code;
      // mixed lists: d = c_i - c_j - s nc = -o
      s_ecode[w][slot] = (int32_t)(dcode ? image_code(-ox, -oy, -oz) : code);
    }
    own_slot = 0;
    wave_lds_sync();
    if (lane == 0) {
      int32_t acc = 0;
      for (int p = 0; p < 27; ++p) {
        const int32_t len = s_pre[w][p];
        s_pre[w][p] = acc;
        acc += len;
      }
      s_pre[w][27] = acc;
    }
    wave_lds_sync();
  } else {
    // staged path: pieces by neighbour rows; lane q < 9 builds neighbour row q
    // (dz = q/3 - 1, dy = q%3 - 1)
    if (lane < 9) {
      int32_t nz, sz, ny, sy;
      stencil_axis(qz, lane / 3 - 1, nc, nz, sz);
      stencil_axis(qy, lane % 3 - 1, nc, ny, sy);
      const int32_t rowbase = R.coff + (nz * nc + ny) * nc;
      const int p = 3 * lane;
      // left wrap, main, right wrap; empty pieces have zero length
      s_k0[w][p] = cell_start[rowbase + nc - 1];
      s_code[w][p] = (int32_t)image_code(-1, sy, sz);
      const int32_t nl = qx - 1 < 0 ? cell_start[rowbase + nc] - cell_start[rowbase + nc - 1] : 0;
      const int32_t lo = qx - 1 < 0 ? 0 : qx - 1, hi = qx + 1 >= nc ? nc - 1 : qx + 1;
      s_k0[w][p + 1] = cell_start[rowbase + lo];
      s_code[w][p + 1] = (int32_t)image_code(0, sy, sz);
      const int32_t nm = cell_start[rowbase + hi + 1] - cell_start[rowbase + lo];
      s_k0[w][p + 2] = cell_start[rowbase];
      s_code[w][p + 2] = (int32_t)image_code(1, sy, sz);
      const int32_t nr = qx + 1 >= nc ? cell_start[rowbase + 1] - cell_start[rowbase] : 0;
      s_pre[w][p] = nl;  // lengths for now
      s_pre[w][p + 1] = nm;
      s_pre[w][p + 2] = nr;
      // the tile's row q: left piece (logical cell a-1 < 0), main cells, right
      // piece (logical cell a+nx >= nc); offsets of this cell's pieces in it
      const RowTile T = rtiles[cell_tile[c]];
      const int32_t tlo = T.a - 1, thi = T.a + T.nx;
      const int32_t mlo = tlo < 0 ? 0 : tlo, mhi = thi >= nc ? nc - 1 : thi;
      const int32_t lsz = tlo < 0 ? cell_start[rowbase + nc] - cell_start[rowbase + nc - 1] : 0;
      const int32_t msz = cell_start[rowbase + mhi + 1] - cell_start[rowbase + mlo];
      const int32_t rsz = thi >= nc ? cell_start[rowbase + 1] - cell_start[rowbase] : 0;
      s_rowsz[w][lane] = lsz + msz + rsz;
      s_l0[w][p] = 0;
      s_l0[w][p + 1] = lsz + (cell_start[rowbase + lo] - cell_start[rowbase + mlo]);
      s_l0[w][p + 2] = lsz + msz;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      int32_t acc = 0;
      for (int p = 0; p < 27; ++p) {
        const int32_t len = s_pre[w][p];
        s_pre[w][p] = acc;
        acc += len;
      }
      s_pre[w][27] = acc;
      int32_t ro = 0;
      for (int q = 0; q < 9; ++q) {
        for (int u = 0; u < 3; ++u) s_l0[w][3 * q + u] += ro;
        ro += s_rowsz[w][q];
      }
      if (ro > kMaxStaged) atomicOr(&st->err, kErrSlots);
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int32_t ncand = s_pre[w][27];

  // groups of at most kCwGroup home particles, of equal size
  const int32_t ngrp = (nh + kCwGroup - 1) / kCwGroup;
  const int32_t gsz = ngrp ? (nh + ngrp - 1) / ngrp : 1;
  // first packed candidate of the cell's own particles (the home cell's
  // piece, or the main piece of the central row: the only candidates that
  // can be a home particle itself)
  const int32_t sv0 = s_pre[w][own_slot] + (h0 - s_k0[w][own_slot]);
  for (int32_t g0 = 0; g0 < nh; g0 += gsz) {
    const int32_t gn = nh - g0 < gsz ? nh - g0 : gsz;
    const int32_t gbase = __builtin_amdgcn_readfirstlane(h0 + g0);  // wave-uniform
    E* const grow = nbr + list_base(gbase, cap);
    const int32_t gs0 = sv0 + g0;  // packed candidates of the group's own particles: [gs0, gs0 + gn)
    int32_t cntv = 0;              // lane h: hits of home gbase + h so far
    for (int32_t pb = 0; pb < ncand; pb += kCwChunks * 64) {
      const int32_t pend = ncand - pb < kCwChunks * 64 ? ncand : pb + kCwChunks * 64;
      const int32_t nwords = 2 * ((pend - pb + 63) >> 6);
      int32_t passv = 0;  // lane h: hits of home gbase + h in this pass
      // ---- test phase ----
      for (int32_t base = pb; base < pend; base += 64) {
        const int32_t ci = (base - pb) >> 6;
        const int32_t v = base + lane;
        const bool valid = v < ncand;
        // piece of candidate v: the last p with s_pre[p] <= v
        int p = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1)
          if (p + step <= 26 && s_pre[w][p + step] <= v) p += step;
        const int32_t k = valid ? s_k0[w][p] + (v - s_pre[w][p]) : h0;
        const uint32_t code = (uint32_t)s_code[w][p];
        const double4 q = pos_tmp[k];
        // the periodic shift of the piece, added after the difference:
        // d = (x_j - x_i) + s L (exactly antisymmetric under exchange); a
        // chunk with no shifted candidate skips the adds (x + 0 = x up to
        // the sign of a zero, which r^2 does not see).  Lanes past the last
        // candidate sit far away, so their test fails without a mask.
        const double sx = (double)(((int32_t)(code << 4)) >> 30) * R.L;
        const double sy = (double)(((int32_t)(code << 2)) >> 30) * R.L;
        const double sz = (double)(((int32_t)code) >> 30) * R.L;
        const double xq = valid ? q.x : kFar, yq = q.y, zq = q.z;
        const bool shifted = __builtin_amdgcn_ballot_w64(valid && code != 0u) != 0;
        const int32_t tj = (int32_t)q.w;  // thr[4 ta + tj] is the pair (ta, tj)
        const double t0 = s_thr[tj], t1 = s_thr[4 + tj], t2 = s_thr[8 + tj], t3 = s_thr[12 + tj];
        const double d01 = t1 - t0;
        uint32_t entry;
        if constexpr (TILE) {
          entry = (uint32_t)((s_l0[w][p] + (v - s_pre[w][p])) & 0x3fff) | ((uint32_t)tj << 14);
        } else {
          entry = (uint32_t)k | (uint32_t)s_ecode[w][p];
        }
        ent[ci * 64 + lane] = entry;
        // chunks that miss the group's own particles skip the self test
        const bool self_chunk = base < gs0 + gn && gs0 < base + 64;
        uint32_t mlo = 0, mhi = 0;  // lane h: hit bits of home gbase + h
        int32_t h = 0;
        // U home particles (wave-uniform, scalar loads): the distances
        // first (independent work), then the ballots; blocks of HPI, then
        // one of 2 and one of 1 for the rest, all with the same code
        auto block = [&](auto self_tag, auto shift_tag, auto u_tag) {
          constexpr bool SELF = decltype(self_tag)::value;
          constexpr bool SHIFT = decltype(shift_tag)::value;
          constexpr int U = decltype(u_tag)::value;
          const int32_t i0 = __builtin_amdgcn_readfirstlane(gbase + h);
          double ra[U], tha[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const double4 pa = pos_tmp[i0 + u];
            double ax = xq - pa.x, ay = yq - pa.y, az = zq - pa.z;
            if constexpr (SHIFT) {
              ax = ax + sx;
              ay = ay + sy;
              az = az + sz;
            }
            ra[u] = (ax * ax + ay * ay) + az * az;
            tha[u] = pick_thr<NT>(pa.w, t0, d01, t1, t2, t3);
          }
          uint64_t m[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bool hit = SELF ? ((k != i0 + u) & (ra[u] < tha[u])) : ra[u] < tha[u];
            m[u] = __builtin_amdgcn_ballot_w64(hit);
          }
          write_lanes<U>(mlo, mhi, m, h);
          h += U;
        };
        auto homes = [&](auto self_tag, auto shift_tag) {
          while (h + HPI <= gn) block(self_tag, shift_tag, std::integral_constant<int, HPI>{});
          if (h + 2 <= gn) block(self_tag, shift_tag, std::integral_constant<int, 2>{});
          if (h < gn) block(self_tag, shift_tag, std::integral_constant<int, 1>{});
        };
        if (shifted) {
          if (self_chunk)
            homes(std::true_type{}, std::true_type{});
          else
            homes(std::false_type{}, std::true_type{});
        } else {
          if (self_chunk)
            homes(std::true_type{}, std::false_type{});
          else
            homes(std::false_type{}, std::false_type{});
        }
        if (lane < kCwGroup) {
          hits[(2 * ci) * kCwGroup + lane] = mlo;
          hits[(2 * ci + 1) * kCwGroup + lane] = mhi;
        }
        passv += (int32_t)(__popc(mlo) + __popc(mhi));  // 0 on lanes >= gn
      }
      wave_lds_sync();
      // ---- write phase ----
      // home h = lane & 31 stores its first lim rows of the pass, from row
      // cntv on: lane h the first S of them, lane h + 32 the rest (S = half
      // the longest), each lane walking the home's hit bits from its first
      // rank on.  Both halves store whole row segments.
      const int32_t room = cap - cntv > 0 ? cap - cntv : 0;
      const int32_t lim = lane < gn ? (passv < room ? passv : room) : 0;
      int32_t mxl = lim;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) mxl = max(mxl, __shfl_xor(mxl, d, 64));
      const int32_t half = (__builtin_amdgcn_readfirstlane(mxl) + 1) >> 1;
      const int32_t hl = lane & (kCwGroup - 1), seg = lane >> 5;
      const int32_t lim_h = __shfl(lim, hl, 64), cnt_h = __shfl(cntv, hl, 64);
      const int32_t rbeg = seg ? half : 0;
      const int32_t nseg = (seg ? lim_h : (lim_h < half ? lim_h : half)) - rbeg;
      int32_t wi = 0;
      uint32_t cur = 0u;
      if (nseg > 0) {
        cur = hits[hl];
        if (seg) {
          // the word holding the home's hit of rank rbeg, then that bit
          int32_t acc = 0, pc = __popc(cur);
          while (acc + pc <= rbeg && wi + 1 < nwords) {
            acc += pc;
            ++wi;
            cur = hits[wi * kCwGroup + hl];
            pc = __popc(cur);
          }
          for (int32_t j = acc; j < rbeg; ++j) cur &= cur - 1u;
        }
      }
      // list slot of home gbase + hl relative to grow (a group of at most 32
      // consecutive particles spans at most two slices)
      const uint32_t hslot =
          (uint32_t)hl +
          (((gbase & (kSlice - 1)) + hl) >= kSlice ? (uint32_t)(cap - 1) * (uint32_t)kSlice : 0u);
      const uint32_t loff = hslot + (uint32_t)(cnt_h + rbeg) * (uint32_t)kSlice;
      // lane: rows [0, nseg) of its segment.  An iteration stores the next
      // row; when the lane's word is used up it first takes the word read
      // ahead, and the word after that is read with no select on its value,
      // so that read stays in flight beside the entry read instead of being
      // waited for (t < nseg leaves a set bit in words wi.., so a refill
      // never passes the last word; the clamp on wi and the spare word only
      // keep every access inside the wave's arrays).  A lane that meets an
      // empty word (rare) spends an iteration on it and stores its later
      // rows one iteration late; every lane is done within half + nwords
      // iterations (at most half rows, at most one word change per word).
      uint32_t nxt = hits[(wi + 1) * kCwGroup + hl];
      const uint32_t* ew = ent + wi * 32;  // entries of the current word
      E* rowp = grow + loff;               // the lane's next row slot
      int32_t r = 0;
      const int32_t tmax = half + nwords;
      for (int32_t t = 0; t < tmax; ++t) {
        if (!__builtin_amdgcn_ballot_w64(r < nseg)) break;
        if (r < nseg) {
          if (cur == 0u) {
            wi = wi + 1 < nwords ? wi + 1 : wi;
            ew = ent + wi * 32;
            // the copy as an instruction of its own, kept above the read:
            // the new word then lands in nxt's own register and nothing
            // waits for it here
            asm volatile("v_mov_b32 %0, %1" : "=v"(cur) : "v"(nxt));
            __builtin_amdgcn_sched_barrier(0);
            nxt = hits[(wi + 1) * kCwGroup + hl];
          }
          if (cur != 0u) {
            const uint32_t b = (uint32_t)__builtin_ctz(cur);
            cur &= cur - 1u;
            *rowp = (E)ew[b];
            rowp += kSlice;
            ++r;
          }
        }
      }
      cntv += passv;
      wave_lds_sync();  // the next pass or group rewrites ent and hits
    }
    if (lane < gn) {
      ncount[gbase + lane] = cntv;
      if (cntv > cap) atomicOr(&st->err, kErrOverflow);
    }
  }
  // the new cell order becomes the live state
  for (int32_t h = lane; h < nh; h += 64) {
    const int32_t i = h0 + h;
    const double4 p4 = pos_tmp[i];
    if (pos16)
      pos16[i] = make_recq(p4.x, p4.y, p4.z, pack_cell(qx, qy, qz, (int32_t)p4.w), R.cside, R.qs);
    pos[i] = p4;
    xref[i] = p4.x;
    xref[stride + i] = p4.y;
    xref[2 * (size_t)stride + i] = p4.z;
    vel[i] = vel_tmp[i];
    vel[stride + i] = vel_tmp[stride + i];
    vel[2 * (size_t)stride + i] = vel_tmp[2 * (size_t)stride + i];
    id[i] = id_tmp[i];
  }
}

}  // namespace

void launch_nlist(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                  const int32_t* rebuild, const PairTab* tab, int32_t thr_form,
                  const int32_t* cell_start, int32_t stride, int32_t cap,
                  const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                  double4* pos, double* vel, int32_t* id, double* xref, uint32_t* nbr,
                  int32_t* ncount, DevState* st, int32_t ncells, const int32_t* cell_rep,
                  int32_t any_single, int32_t any_multi, int4* pos16, int32_t spread) {
  // mixed lists (records present) carry cell offsets instead of images
  const int32_t dcode = pos16 != nullptr;
  if (any_multi) {
    const int32_t nb = (ncells + kCwWaves - 1) / kCwWaves;
    const int32_t g = spread / kCwWaves, grid = g ? spread_grid(nb, g) : nb;
#define KN(NT)                                                                             \
  k_nlist_cells<kCwHomes, false, NT><<<grid, 64 * kCwWaves, 0, s>>>(                       \
          ncells, cell_rep, reps, rebuild, tab, cell_start, stride, cap, pos_tmp, vel_tmp, \
          id_tmp, pos, vel, id, xref, nbr, ncount, st, pos16, nullptr, nullptr, dcode, g)
    if (thr_form == 2) KN(2); else KN(4);
#undef KN
  }
  if (any_single)
    k_nlist<<<ntiles, kTile, 0, s>>>(tiles, reps, rebuild, tab, stride, cap, pos_tmp, vel_tmp,
                                     id_tmp, pos, vel, id, xref, nbr, ncount, st, dcode, pos16);
}

void launch_nlist_tiles(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const RepDesc* reps, const int32_t* rebuild, const PairTab* tab,
                        int32_t thr_form, const int32_t* cell_start, int32_t stride, int32_t cap,
                        const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                        double4* pos, double* vel, int32_t* id, double* xref, uint16_t* nbr16,
                        int32_t* ncount, DevState* st, const int32_t* cell_tile,
                        const RowTile* rtiles, int32_t spread) {
  const int32_t nb = (ncells + kCwWaves - 1) / kCwWaves;
  const int32_t g = spread / kCwWaves, grid = g ? spread_grid(nb, g) : nb;
#define KT(NT)                                                                                   \
  k_nlist_cells<kCwHomes, true, NT><<<grid, 64 * kCwWaves, 0, s>>>(                              \
          ncells, cell_rep, reps, rebuild, tab, cell_start, stride, cap, pos_tmp, vel_tmp, id_tmp, \
          pos, vel, id, xref, nbr16, ncount, st, nullptr, cell_tile, rtiles, 0, g)
  if (thr_form == 2) KT(2); else KT(4);
#undef KT
}

}  // namespace mdk
