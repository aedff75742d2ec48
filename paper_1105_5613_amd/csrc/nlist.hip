// nlist.hip -- cut-off neighbour search over the 27-cell stencil.
//
// The paper finds interacting pairs with a linked-cell grid search over
// neighbouring cubic cells ("Grid-search method", Fig. 1).  Here the same
// search fills a full (both directions) neighbour list with a skin, so the
// force kernel can reuse it for several steps.  The inclusion test must give
// exactly the same set as a plain FP64 evaluation of
//     d = (x_j + s L) - x_i,  r^2 = (dx dx + dy dy) + dz dz  <  (rc_ab + skin)^2
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


// One wave per home cell (nc >= 3).  The candidates of the cell -- the 9
// neighbour rows, each one to three contiguous particle ranges with their
// periodic shift -- are packed 64 to a chunk, one candidate per lane, with
// x_j + s L formed once per chunk.  For every home particle (uniform loop,
// coordinates through scalar loads) each lane tests its candidate; the hits
// are compacted with a ballot and appended to the home particle's row in
// candidate order.  Copying the new order into the live arrays is done here
// as well.
constexpr int kCwGroup = 64;  // home particles per pass: lane h keeps the count of home h
constexpr int kCwHomes = 4;   // home particles tested per iteration
constexpr int kCwBuf = 1024;  // list entries staged in LDS per wave (4 KB)
constexpr double kFar = 1.0e300;  // x of the idle lanes of a chunk: r^2 overflows to +inf

// Append the hits of the lane's candidate for home particle hl of the group
// (wave-uniform) at that particle's running count cnt.  Rows below rows_lds
// go to the wave's LDS buffer ([home][row] layout: a wave-uniform base plus
// the row, one full-rate address operation; rows_lds is odd, so the row
// write-out, whose lanes read one row of consecutive homes, is free of bank
// conflicts) and reach the list later as whole row segments; rows above it
// are stored straight into the home particle's list row hrow (a wave-uniform
// pointer: one scalar base plus a 32-bit lane offset per store).
template <typename E>
__device__ inline int32_t cw_append(uint64_t mask, bool hit, int32_t cnt, int32_t hl,
                                    uint32_t entry, int32_t cap, int32_t rows_lds,
                                    uint32_t* buf, E* __restrict__ hrow) {
  if (mask) {
    const int32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
    const int32_t k = cnt + rk;
    if (hit && k < cap) {
      if (k < rows_lds)
        buf[hl * rows_lds + k] = entry;
      else
        *reinterpret_cast<E*>(reinterpret_cast<char*>(hrow) +
                              (uint32_t)k * (uint32_t)(kSlice * sizeof(E))) = (E)entry;
    }
    cnt += (int32_t)__popcll(mask);
  }
  return cnt;
}

// v[l] = x for the wave-uniform lane l (one v_writelane; the clang in use
// has no builtin for it).  Lanes other than l keep their value.
__device__ inline int32_t write_lane(int32_t v, int32_t x, int32_t l) {
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "{m0}"(l));
  return v;
}

// List row of home particle gbase + h, from the row of gbase: a group of at
// most 64 consecutive particles spans at most two slices.
template <typename E>
__device__ inline E* home_row(E* grow, int32_t gbase, int32_t h, int32_t cap) {
  const uint32_t off = (uint32_t)h + (((gbase & (kSlice - 1)) + h) >= kSlice
                                          ? (uint32_t)(cap - 1) * (uint32_t)kSlice
                                          : 0u);
  return grow + __builtin_amdgcn_readfirstlane(off);
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

// One wave per home cell (nc >= 3): the lanes take the 64 candidates of one
// chunk of the cell's packed 27-cell neighbourhood, and the wave walks the
// home particles (kCwHomes per iteration, positions in scalar registers);
// hits are compacted with a ballot.  The first kCwBuf / (homes) rows of the
// cell's lists are assembled in LDS and written out row by row (one
// contiguous store per row instead of scattered single entries); the LDS
// buffer is kept small because occupancy matters more here than write
// combining.
//
// TILE = false: entries are sorted index | image code (uint32, gather path).
// TILE = true: entries are the partner's LDS slot in the staged neighbourhood
// of the row tile holding the home cell (stage.h) | species << 14 (uint16,
// staged path); the slot of a candidate is its piece's first slot in that
// layout plus its offset inside the piece.
template <int HPI, int BUF, bool TILE, int NT>
__global__ __launch_bounds__(256) void k_nlist_cells(
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
  __shared__ int32_t s_pre[4][28];    // first packed candidate of piece p
  __shared__ int32_t s_k0[4][27];     // first sorted index of piece p
  __shared__ int32_t s_code[4][27];   // image code of piece p (shift -1/0/1 per axis)
  __shared__ int32_t s_l0[4][27];     // TILE: first LDS slot of piece p in the tile layout
  __shared__ int32_t s_rowsz[4][9];   // TILE: slots of tile row q
  extern __shared__ uint32_t s_list[];  // [4][kCwBuf]
  if (!st->any_rebuild) return;  // whole block: one flag load when nothing rebuilds
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t c =
      (spread ? xcd_spread(blockIdx.x, spread) : xcd_block(blockIdx.x, gridDim.x)) * 4 + w;
  if (c >= ncells) return;
  const int32_t r = cell_rep[c];
  if (!rebuild[r]) return;
  const RepDesc R = reps[r];
  if (R.nc == 1) return;  // minimum-image kernel
  const int32_t nc = R.nc;
  const int32_t lc = c - R.coff;
  const int32_t qx = lc % nc, qy = (lc / nc) % nc, qz = lc / (nc * nc);
  const int32_t h0 = cell_start[c], nh = cell_start[c + 1] - h0;
  uint32_t* buf = s_list + w * BUF;

  // pieces: lane q < 9 builds neighbour row q (dz = q/3 - 1, dy = q%3 - 1)
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
    if constexpr (TILE) {
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
    if constexpr (TILE) {
      int32_t ro = 0;
      for (int q = 0; q < 9; ++q) {
        for (int u = 0; u < 3; ++u) s_l0[w][3 * q + u] += ro;
        ro += s_rowsz[w][q];
      }
      if (ro > kMaxStaged) atomicOr(&st->err, kErrSlots);
    }
  }
  __builtin_amdgcn_wave_barrier();
  const int32_t ncand = s_pre[w][27];

  for (int32_t g0 = 0; g0 < nh; g0 += kCwGroup) {
    const int32_t gn = nh - g0 < kCwGroup ? nh - g0 : kCwGroup;
    const int32_t gbase = __builtin_amdgcn_readfirstlane(h0 + g0);  // wave-uniform
    const int32_t rows_lds = (BUF / gn - 1) | 1;  // odd, <= BUF / gn
    E* const grow = nbr + list_base(gbase, cap);
    int32_t cntv = 0;  // lane h: neighbours found so far for home gbase + h
    for (int32_t base = 0; base < ncand; base += 64) {
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
      // the periodic shift of the piece: x_j + s L; lanes past the last
      // candidate sit far away, so their test fails without a mask
      const double sx = (double)(((int32_t)(code << 4)) >> 30) * R.L;
      const double sy = (double)(((int32_t)(code << 2)) >> 30) * R.L;
      const double sz = (double)(((int32_t)code) >> 30) * R.L;
      const double xs = valid ? q.x + sx : kFar, ys = q.y + sy, zs = q.z + sz;
      const int32_t tj = (int32_t)q.w;  // thr[4 ta + tj] is the pair (ta, tj)
      const double t0 = s_thr[tj], t1 = s_thr[4 + tj], t2 = s_thr[8 + tj], t3 = s_thr[12 + tj];
      const double d01 = t1 - t0;
      uint32_t entry;
      if constexpr (TILE) {
        entry = (uint32_t)((s_l0[w][p] + (v - s_pre[w][p])) & 0x3fff) | ((uint32_t)tj << 14);
      } else if (dcode) {
        // d = c_i - c_j - s nc: -dy, -dz of the row; along x from the
        // partner's build-time cell and the piece's shift
        const int32_t row = p / 3, kind = p - 3 * row;
        const int32_t cxj = cell_coord(q.x, R.inv_cell, nc);
        entry = (uint32_t)k | image_code(qx - cxj - (kind - 1) * nc, 1 - row % 3, 1 - row / 3);
      } else {
        entry = (uint32_t)k | code;
      }
      // the cell's own particles -- the only candidates that can be the home
      // particle itself -- are the main piece of the central row; chunks that
      // miss them skip the self test
      const int32_t sv0 = s_pre[w][13] + (h0 - s_k0[w][13]);
      const bool self_chunk = base < sv0 + nh && sv0 < base + 64;
      int32_t h = 0;
      // HPI home particles per iteration (wave-uniform, scalar loads): the
      // distances first (independent work), then test, ballot and append
      // home by home
      auto homes = [&](auto self_tag) {
        constexpr bool SELF = decltype(self_tag)::value;
        for (; h + HPI <= gn; h += HPI) {
          const int32_t i0 = __builtin_amdgcn_readfirstlane(gbase + h);
          double ra[HPI], tha[HPI];
#pragma unroll
          for (int u = 0; u < HPI; ++u) {
            const double4 pa = pos_tmp[i0 + u];
            const double ax = xs - pa.x, ay = ys - pa.y, az = zs - pa.z;
            ra[u] = (ax * ax + ay * ay) + az * az;
            tha[u] = pick_thr<NT>(pa.w, t0, d01, t1, t2, t3);
          }
#pragma unroll
          for (int u = 0; u < HPI; ++u) {
            const bool hit = SELF ? (k != i0 + u && ra[u] < tha[u]) : ra[u] < tha[u];
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            int32_t cu = __builtin_amdgcn_readlane(cntv, h + u);
            cu = cw_append(m, hit, cu, h + u, entry, cap, rows_lds, buf,
                           home_row(grow, gbase, h + u, cap));
            cntv = write_lane(cntv, cu, h + u);
          }
        }
      };
      if (self_chunk)
        homes(std::true_type{});
      else
        homes(std::false_type{});
      for (; h < gn; ++h) {
        const int32_t ia = __builtin_amdgcn_readfirstlane(gbase + h);
        const double4 pa = pos_tmp[ia];
        const double ax = xs - pa.x, ay = ys - pa.y, az = zs - pa.z;
        const double ra = (ax * ax + ay * ay) + az * az;
        const double tha = pick_thr<NT>(pa.w, t0, d01, t1, t2, t3);
        const bool hita = k != ia && ra < tha;
        const uint64_t ma = __builtin_amdgcn_ballot_w64(hita);
        int32_t ca = __builtin_amdgcn_readlane(cntv, h);
        ca = cw_append(ma, hita, ca, h, entry, cap, rows_lds, buf, home_row(grow, gbase, h, cap));
        cntv = write_lane(cntv, ca, h);
      }
    }
    if (lane < gn) {
      ncount[gbase + lane] = cntv;
      if (cntv > cap) atomicOr(&st->err, kErrOverflow);
    }
    if (BUF == 0) continue;
    // write the staged rows: row k of the group is gn consecutive entries
    int32_t mx = lane < gn ? cntv : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
    const int32_t rows = min(min(mx, cap), rows_lds);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t per = 64 / gn;  // rows per store
    const int32_t lr = lane / gn, lh = lane - lr * gn;
    if (lr < per)
      for (int32_t kk = lr; kk < rows; kk += per)
        nbr[list_base(gbase + lh, cap) + (size_t)kk * kSlice] = (E)buf[lh * rows_lds + kk];
    // the next group reuses the buffer
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
    const int32_t nb = (ncells + 3) / 4, grid = spread ? spread_grid(nb, spread) : nb;
#define KN(NT)                                                                             \
  k_nlist_cells<kCwHomes, kCwBuf, false, NT>                                               \
      <<<grid, 256, 4 * kCwBuf * sizeof(uint32_t), s>>>(                                   \
          ncells, cell_rep, reps, rebuild, tab, cell_start, stride, cap, pos_tmp, vel_tmp, \
          id_tmp, pos, vel, id, xref, nbr, ncount, st, pos16, nullptr, nullptr, dcode, spread)
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
  const int32_t nb = (ncells + 3) / 4, grid = spread ? spread_grid(nb, spread) : nb;
#define KT(NT)                                                                                   \
  k_nlist_cells<kCwHomes, kCwBuf, true, NT>                                                      \
      <<<grid, 256, 4 * kCwBuf * sizeof(uint32_t), s>>>(                                         \
          ncells, cell_rep, reps, rebuild, tab, cell_start, stride, cap, pos_tmp, vel_tmp, id_tmp, \
          pos, vel, id, xref, nbr16, ncount, st, nullptr, cell_tile, rtiles, 0, spread)
  if (thr_form == 2) KT(2); else KT(4);
#undef KT
}

}  // namespace mdk
