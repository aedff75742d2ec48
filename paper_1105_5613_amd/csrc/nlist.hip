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
// List entry: sorted index j (26 bits) | periodic image code (6 bits): two
// bits per axis holding s in {-1, 0, 1} in two's complement, so an entry
// without a periodic shift is the plain index.
#include "md_internal.h"

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

__global__ __launch_bounds__(kTile) void k_nlist(
    const Tile* __restrict__ tiles, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ rebuild, const PairTab* __restrict__ tab, int32_t ntypes,
    const int32_t* __restrict__ cell_start, int32_t stride, int32_t cap,
    const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref, uint32_t* __restrict__ nbr,
    int32_t* __restrict__ ncount, DevState* st) {
  __shared__ double s_thr[16];
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  __syncthreads();
  const Tile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
  if (!rebuild[t.rep]) return;
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  const RepDesc R = reps[t.rep];
  const double4 p = pos_tmp[i];
  const int32_t ti = (int32_t)p.w;
  const double* thr = &s_thr[ti * 4];
  int32_t cnt = 0;
  uint32_t* out = nbr + i;
  if (R.nc == 1) {
    // one cell: the minimum image  d - L nearbyint(d / L)
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
        if (cnt < cap)
          out[(size_t)cnt * stride] =
              (uint32_t)j | image_code(-(int32_t)kx, -(int32_t)ky, -(int32_t)kz);
        ++cnt;
      }
    }
  } else {
    const int32_t nc = R.nc;
    const int32_t qx = cell_coord(p.x, R.inv_cell, nc);
    const int32_t qy = cell_coord(p.y, R.inv_cell, nc);
    const int32_t qz = cell_coord(p.z, R.inv_cell, nc);
    for (int32_t oz = -1; oz <= 1; ++oz) {
      int32_t nz, sz;
      stencil_axis(qz, oz, nc, nz, sz);
      const double shz = (double)sz * R.L;
      for (int32_t oy = -1; oy <= 1; ++oy) {
        int32_t ny, sy;
        stencil_axis(qy, oy, nc, ny, sy);
        const double shy = (double)sy * R.L;
        for (int32_t ox = -1; ox <= 1; ++ox) {
          int32_t nx, sx;
          stencil_axis(qx, ox, nc, nx, sx);
          const double shx = (double)sx * R.L;
          const uint32_t code = image_code(sx, sy, sz);
          const int32_t cn = R.coff + (nz * nc + ny) * nc + nx;
          const int32_t k1 = cell_start[cn + 1];
          for (int32_t k = cell_start[cn]; k < k1; ++k) {
            if (k == i) continue;
            const double4 q = pos_tmp[k];
            double ex = (q.x + shx) - p.x;
            double ey = (q.y + shy) - p.y;
            double ez = (q.z + shz) - p.z;
            double r2 = (ex * ex + ey * ey) + ez * ez;
            if (r2 < thr[(int32_t)q.w]) {
              if (cnt < cap) out[(size_t)cnt * stride] = (uint32_t)k | code;
              ++cnt;
            }
          }
        }
      }
    }
  }
  ncount[i] = cnt;
  if (cnt > cap) atomicOr(&st->err, kErrOverflow);
  // the new cell order becomes the live state; the list is built on it
  pos[i] = p;
  xref[i] = p.x;
  xref[stride + i] = p.y;
  xref[2 * (size_t)stride + i] = p.z;
  vel[i] = vel_tmp[i];
  vel[stride + i] = vel_tmp[stride + i];
  vel[2 * (size_t)stride + i] = vel_tmp[2 * (size_t)stride + i];
  id[i] = id_tmp[i];
  (void)ntypes;
}

}  // namespace

void launch_nlist(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                  const int32_t* rebuild, const PairTab* tab, int32_t ntypes,
                  const int32_t* cell_start, int32_t stride, int32_t cap,
                  const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                  double4* pos, double* vel, int32_t* id, double* xref, uint32_t* nbr,
                  int32_t* ncount, DevState* st) {
  k_nlist<<<ntiles, kTile, 0, s>>>(tiles, reps, rebuild, tab, ntypes, cell_start, stride, cap,
                                   pos_tmp, vel_tmp, id_tmp, pos, vel, id, xref, nbr, ncount,
                                   st);
}

}  // namespace mdk
