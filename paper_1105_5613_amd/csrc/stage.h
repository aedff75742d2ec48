// stage.h -- row tiles and their LDS-staged neighbourhoods (device helpers
// shared by the staged force kernel, the staged neighbour-list entries and
// their decode).
//
// A row tile is a run of home cells [a, a + nx) of one x-row (cy, cz) of a
// replica's cell grid.  With cells of side >= cutoff + skin, every partner of
// a home particle lies in the 3 x 3 neighbour rows (dz, dy in {-1, 0, 1}) and,
// along x, in the logical cells a-1 .. a+nx.  Cells are stored in z-major
// order, so each neighbour row contributes up to three contiguous particle
// ranges ("pieces"): the main range and, where the row wraps around the
// periodic box, one cell on either side.  All 27 pieces are staged into LDS
// once per block, with their periodic shift s*L already added, in FP64, i.e.
// exactly the value x_j + s*L that the cut-off test uses; rows follow each
// other in the order (dz, dy) = (-1,-1), (-1,0), ... (1,1) and inside a row
// the left piece, the main range and the right piece.  Logical cells stay
// contiguous in LDS, so the partners of a home particle in cell cx are, per
// neighbour row, in the single slot range [start(cx-1), start(cx+2)).
//
// A staged list entry is the LDS slot (14 bits) | species << 14.  Slots at or
// above the LDS capacity of a launch are fetched from global memory through
// the piece table ("virtual" slots), so an unusually dense tile still works.
#pragma once
#include "md_internal.h"

namespace mdk {

struct RowTile {
  int32_t rep;
  int32_t row;  // cz * nc + cy
  int32_t a;    // first home cell along x
  int32_t nx;   // home cells, 1 .. kMaxRowCells
};

constexpr int kMaxRowCells = 64;
constexpr int kPieces = 27;          // 9 neighbour rows x (left, main, right)
constexpr int32_t kMaxStaged = 16383;  // slots fit 14 bits (force entries carry the species)

struct StageLayout {
  int32_t total;                     // staged slots S
  int32_t home0, home1;              // sorted indices of the home particles
  int32_t home_lds;                  // slot of particle home0
  int32_t cnt[9];                    // slots per neighbour row
  int32_t pc_g[kPieces];             // first sorted index of piece p
  int32_t pc_l[kPieces + 1];         // first slot of piece p (pc_l[27] = total)
  double pc_sx[kPieces], pc_sy[kPieces], pc_sz[kPieces];
  int32_t loff[9][kMaxRowCells + 3]; // first slot of logical cell a-1+c, c = 0..nx+2
};

__device__ inline void wrap_axis(int32_t q, int32_t nc, int32_t& qn, int32_t& s) {
  s = 0;
  if (q < 0) {
    q += nc;
    s = -1;
  } else if (q >= nc) {
    q -= nc;
    s = 1;
  }
  qn = q;
}

// All threads of the block call this; it ends with a barrier.
__device__ inline void build_layout(StageLayout& S, const RowTile& T, const RepDesc& R,
                                    const int32_t* __restrict__ cell_start) {
  const int k = threadIdx.x;
  const int32_t nc = R.nc;
  const int32_t cy = T.row % nc, cz = T.row / nc;
  const int32_t a = T.a, nx = T.nx;
  int32_t rowbase = 0, sy = 0, sz = 0;
  if (k < 9) {
    int32_t rz, ry;
    wrap_axis(cz + k / 3 - 1, nc, rz, sz);
    wrap_axis(cy + k % 3 - 1, nc, ry, sy);
    rowbase = R.coff + (rz * nc + ry) * nc;
    const int32_t lo = a - 1, hi = a + nx;  // logical x range, inclusive
    const int32_t mlo = lo < 0 ? 0 : lo, mhi = hi >= nc ? nc - 1 : hi;
    int32_t c = cell_start[rowbase + mhi + 1] - cell_start[rowbase + mlo];
    if (lo < 0) c += cell_start[rowbase + nc] - cell_start[rowbase + nc - 1];
    if (hi >= nc) c += cell_start[rowbase + 1] - cell_start[rowbase];
    S.cnt[k] = c;
  }
  __syncthreads();
  if (k < 9) {
    int32_t off = 0;
    for (int m = 0; m < k; ++m) off += S.cnt[m];
    const int32_t lo = a - 1, hi = a + nx;
    const int32_t mlo = lo < 0 ? 0 : lo, mhi = hi >= nc ? nc - 1 : hi;
    const double shy = (double)sy * R.L, shz = (double)sz * R.L;
    const int p = 3 * k;
    // left piece: logical cell a-1 < 0 is cell nc-1 of the image at -L
    S.pc_l[p] = off;
    S.pc_sx[p] = -R.L;
    S.pc_g[p] = cell_start[rowbase + nc - 1];
    if (lo < 0) {
      S.loff[k][0] = off;
      off += cell_start[rowbase + nc] - cell_start[rowbase + nc - 1];
    }
    // main piece: cells mlo .. mhi, unshifted along x
    const int32_t g0 = cell_start[rowbase + mlo];
    S.pc_l[p + 1] = off;
    S.pc_sx[p + 1] = 0.0;
    S.pc_g[p + 1] = g0;
    for (int32_t c = mlo; c <= mhi; ++c) S.loff[k][c - lo] = off + (cell_start[rowbase + c] - g0);
    off += cell_start[rowbase + mhi + 1] - g0;
    // right piece: logical cell a+nx >= nc is cell 0 of the image at +L
    S.pc_l[p + 2] = off;
    S.pc_sx[p + 2] = R.L;
    S.pc_g[p + 2] = cell_start[rowbase];
    if (hi >= nc) {
      S.loff[k][nx + 1] = off;
      off += cell_start[rowbase + 1] - cell_start[rowbase];
    }
    S.loff[k][nx + 2] = off;
    for (int q = 0; q < 3; ++q) {
      S.pc_sy[p + q] = shy;
      S.pc_sz[p + q] = shz;
    }
    if (k == 8) {
      S.pc_l[kPieces] = off;
      S.total = off;
    }
    if (k == 4) {
      const int32_t hb = R.coff + T.row * nc;
      S.home0 = cell_start[hb + a];
      S.home1 = cell_start[hb + a + nx];
      S.home_lds = S.loff[4][1];
    }
  }
  __syncthreads();
}

// Piece of slot v: the last p with pc_l[p] <= v (binary lifting; empty
// pieces never match because the next piece starts at the same slot).
__device__ inline int piece_of(const StageLayout& S, int32_t v) {
  int p = 0;
#pragma unroll
  for (int step = 16; step >= 1; step >>= 1)
    if (p + step < kPieces && S.pc_l[p + step] <= v) p += step;
  return p;
}

// Staged coordinates of slot v straight from global memory (virtual slots).
// A slot past the layout (only after a reported overflow) is clamped so the
// read stays inside the tile's pieces.
__device__ inline double4 fetch_slot(const StageLayout& S, const double4* __restrict__ pos,
                                     int32_t v) {
  v = v < S.total ? v : S.total - 1;
  const int p = piece_of(S, v);
  const double4 q = pos[S.pc_g[p] + (v - S.pc_l[p])];
  return make_double4(q.x + S.pc_sx[p], q.y + S.pc_sy[p], q.z + S.pc_sz[p], q.w);
}

// Copy all pieces into LDS (slots below cap) as (x, y) pairs and z values;
// ends with a barrier.
__device__ inline void stage_all(const StageLayout& S, const double4* __restrict__ pos,
                                 int32_t cap, double2* xy, double* zz) {
  const int32_t m = S.total < cap ? S.total : cap;
  for (int32_t v = threadIdx.x; v < m; v += blockDim.x) {
    const int p = piece_of(S, v);
    const double4 r = pos[S.pc_g[p] + (v - S.pc_l[p])];
    xy[v] = make_double2(r.x + S.pc_sx[p], r.y + S.pc_sy[p]);
    zz[v] = r.z + S.pc_sz[p];
  }
  __syncthreads();
}

}  // namespace mdk
