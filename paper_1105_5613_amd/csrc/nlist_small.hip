// nlist_small.hip -- the cut-off neighbour search of a small box: one
// replica of at most kSmallListN particles with at least three cells per
// side, gather path.  It writes the rows of k_nlist_cells bit for bit: the same
// inclusion test (FP64, no FMA contraction, d = (x_j - x_i) + s L and
// r^2 = (dx dx + dy dy) + dz dz against (r_c,ab + skin)^2; "Grid-search
// method"), the same entries and the same row order (the home cell, then
// each forward stencil offset o in (dz, dy, dx) order followed by its mirror
// -o, candidates in sorted index order within a cell).
//
// The search of k_nlist_cells gives each home cell one wave; a box of a few
// thousand particles has a few hundred cells, so the build takes the latency
// of one wave's walk over its cell.  Here a home particle gets 32 lanes and
// lane k walks stencil cell k of its row order: it counts its hits, an
// exclusive scan over the 32 lanes gives each cell its first row, and a
// second walk stores the hits from there.
#include "md_internal.h"

#pragma clang fp contract(off)

namespace mdk {
namespace {

// neighbour cell q + o along one axis with its periodic image s in {-1, 0, 1}
__device__ inline void wrap_axis(int32_t q, int32_t o, int32_t nc, int32_t& qn, int32_t& s) {
  int32_t t = q + o;
  s = t < 0 ? -1 : (t >= nc ? 1 : 0);
  qn = t - s * nc;
}

// two-bit two's-complement shift per axis above the index bits
__device__ inline uint32_t entry_code(int32_t sx, int32_t sy, int32_t sz) {
  return ((uint32_t)(sx & 3) | ((uint32_t)(sy & 3) << 2) | ((uint32_t)(sz & 3) << 4))
         << kIdxBits;
}

__device__ inline int32_t home_coord(double c, double inv_cell, int32_t nc) {
  const int32_t q = (int32_t)(c * inv_cell);
  return q > nc - 1 ? nc - 1 : q;
}

constexpr int kSmallGroup = 32;  // lanes per home particle (27 stencil cells)

__global__ __launch_bounds__(256) void k_nlist_small(
    const RepDesc* __restrict__ reps, const int32_t* __restrict__ rebuild,
    const PairTab* __restrict__ tab, const int32_t* __restrict__ cell_start, int32_t stride,
    int32_t cap, const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref, uint32_t* __restrict__ nbr,
    int32_t* __restrict__ ncount, DevState* st, int4* __restrict__ pos16) {
  __shared__ double s_thr[16];
  if (!st->any_rebuild) return;
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  __syncthreads();
  if (!rebuild[0]) return;
  const RepDesc R = reps[0];
  const int k = threadIdx.x & (kSmallGroup - 1);
  const int32_t i = R.off + (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kSmallGroup);
  if (i >= R.off + R.n) return;  // whole groups
  const double4 p = pos_tmp[i];
  const int32_t ti = (int32_t)p.w;
  const int32_t nc = R.nc;
  // the cell the particle was binned into (the same wrapped coordinates)
  const int32_t qx = home_coord(p.x, R.inv_cell, nc), qy = home_coord(p.y, R.inv_cell, nc),
                qz = home_coord(p.z, R.inv_cell, nc);
  // lane k: stencil offset q (= (oz + 1) 9 + (oy + 1) 3 + (ox + 1)) at place k
  // of the row order 13, 14, 12, 15, 11, ..., 26, 0
  int32_t j0 = 0, j1 = 0;
  double shx = 0.0, shy = 0.0, shz = 0.0;
  uint32_t code = 0u;
  if (k < 27) {
    const int32_t q = k == 0 ? 13 : ((k & 1) ? 13 + (k + 1) / 2 : 13 - k / 2);
    const int32_t ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
    int32_t nx, sx, ny, sy, nz, sz;
    wrap_axis(qx, ox, nc, nx, sx);
    wrap_axis(qy, oy, nc, ny, sy);
    wrap_axis(qz, oz, nc, nz, sz);
    const int32_t cn = R.coff + (nz * nc + ny) * nc + nx;
    j0 = cell_start[cn];
    j1 = cell_start[cn + 1];
    shx = (double)sx * R.L;
    shy = (double)sy * R.L;
    shz = (double)sz * R.L;
    // FP64 lists: the partner's image s; mixed lists (records present): the
    // cell offset d = c_i - c_j - s nc = -o of the pair
    code = pos16 ? entry_code(-ox, -oy, -oz) : entry_code(sx, sy, sz);
  }
  const double* thr = &s_thr[ti * 4];
  auto hit = [&](int32_t j) {
    const double4 qj = pos_tmp[j];
    const double ex = (qj.x - p.x) + shx, ey = (qj.y - p.y) + shy, ez = (qj.z - p.z) + shz;
    const double r2 = (ex * ex + ey * ey) + ez * ez;
    return j != i && r2 < thr[(int32_t)qj.w];
  };
  int32_t cnt = 0;
  for (int32_t j = j0; j < j1; ++j) cnt += hit(j) ? 1 : 0;
  // first row of this lane's cell: exclusive scan over the home's 32 lanes
  int32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < kSmallGroup; d <<= 1) {
    const int32_t y = __shfl_up(incl, d, kSmallGroup);
    if (k >= d) incl += y;
  }
  const int32_t total = __shfl(incl, kSmallGroup - 1, kSmallGroup);
  int32_t row = incl - cnt;
  if (cnt > 0 && row < cap) {
    uint32_t* out = nbr + list_base(i, cap);
    for (int32_t j = j0; j < j1 && row < cap; ++j) {
      if (hit(j)) {
        out[(size_t)row * kSlice] = (uint32_t)j | code;
        ++row;
      }
    }
  }
  if (k != 0) return;
  ncount[i] = total;
  if (total > cap) atomicOr(&st->err, kErrOverflow);
  // the new cell order becomes the live state
  if (pos16) pos16[i] = make_recq(p.x, p.y, p.z, pack_cell(qx, qy, qz, ti), R.cside, R.qs);
  pos[i] = p;
  xref[i] = p.x;
  xref[stride + i] = p.y;
  xref[2 * (size_t)stride + i] = p.z;
  vel[i] = vel_tmp[i];
  vel[stride + i] = vel_tmp[stride + i];
  vel[2 * (size_t)stride + i] = vel_tmp[2 * (size_t)stride + i];
  id[i] = id_tmp[i];
}

}  // namespace

void launch_nlist_small(hipStream_t s, int32_t ntot, const RepDesc* reps,
                        const int32_t* rebuild, const PairTab* tab, const int32_t* cell_start,
                        int32_t stride, int32_t cap, const double4* pos_tmp,
                        const double* vel_tmp, const int32_t* id_tmp, double4* pos, double* vel,
                        int32_t* id, double* xref, uint32_t* nbr, int32_t* ncount, DevState* st,
                        int4* pos16) {
  const int32_t per_block = 256 / kSmallGroup;
  const int32_t grid = (ntot + per_block - 1) / per_block;
  k_nlist_small<<<grid, 256, 0, s>>>(reps, rebuild, tab, cell_start, stride, cap, pos_tmp,
                                     vel_tmp, id_tmp, pos, vel, id, xref, nbr, ncount, st, pos16);
}

}  // namespace mdk
