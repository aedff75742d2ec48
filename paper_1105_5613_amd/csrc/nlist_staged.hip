// nlist_staged.hip -- cut-off neighbour search of the staged path: one block
// per row tile, candidates read from the tile's LDS-staged neighbourhood,
// staged one z-slab of rows (pass) at a time (see stage.h).  The test is the exact FP64 evaluation
//     d = (x_j + s L) - x_i,  r^2 = (dx dx + dy dy) + dz dz  <  (rc_ab + skin)^2
// (the staged value already is x_j + s L), so this file is compiled without
// FMA contraction.  Entries are 16 bit: LDS slot (14 bits) | species << 14.
// Also holds the decode of staged entries back to sorted particle indices,
// used by the neighbour-list parity hook.
#include "stage.h"

#pragma clang fp contract(off)

namespace mdk {
namespace {

__device__ inline int32_t cell_coord(double c, double inv_cell, int32_t nc) {
  int32_t q = (int32_t)(c * inv_cell);
  return q > nc - 1 ? nc - 1 : q;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_nlist_staged(
    const RowTile* __restrict__ rtiles, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ rebuild, const PairTab* __restrict__ tab,
    const int32_t* __restrict__ cell_start, int32_t stride, int32_t cap, int32_t lcap,
    const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref, uint16_t* __restrict__ nbr,
    int32_t* __restrict__ ncount, uint32_t* __restrict__ nsplit, DevState* st) {
  __shared__ StageLayout S;
  __shared__ double s_thr[16];
  extern __shared__ double dyn[];
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  const RowTile T = rtiles[tb];
  if (!rebuild[T.rep]) return;
  const RepDesc R = reps[T.rep];
  if (threadIdx.x < 16) s_thr[threadIdx.x] = tab->thr[threadIdx.x];
  build_layout(S, T, R, cell_start);
  if (pass_size(S, 0) > kMaxStaged || pass_size(S, 1) > kMaxStaged ||
      pass_size(S, 2) > kMaxStaged) {
    if (threadIdx.x == 0) atomicOr(&st->err, kErrOverflow);
    return;
  }
  double* xs = dyn;
  double* ys = xs + lcap;
  double* zs = ys + lcap;
  uint8_t* ts = (uint8_t*)(zs + lcap);
  const int32_t nh = S.home1 - S.home0;
  // home particles in groups of BT (one per thread); the passes restage per group
  for (int32_t g0 = 0; g0 < nh; g0 += BT) {
    const int32_t li = g0 + (int32_t)threadIdx.x;
    const bool mine = li < nh;
    const int32_t i = S.home0 + (mine ? li : 0);
    const double4 pi = pos_tmp[i];
    const int32_t ti = (int32_t)pi.w;
    const int32_t hv = S.home_lds + li;  // full slot of the home particle
    int32_t cl = cell_coord(pi.x, R.inv_cell, R.nc) - T.a;
    cl = cl < 0 ? 0 : (cl >= T.nx ? T.nx - 1 : cl);
    const double* thr = &s_thr[ti * 4];
    int32_t cnt = 0, n0 = 0, n1 = 0;
    uint16_t* out = nbr + i;
    for (int pass = 0; pass < 3; ++pass) {
      const int32_t base = pass_base(S, pass);
      stage<true>(S, pass, pos_tmp, lcap, xs, ys, zs, ts);
      if (mine) {
        for (int k = 3 * pass; k < 3 * pass + 3; ++k) {
          int32_t v = S.loff[k][cl] - base;  // slots relative to the pass
          const int32_t v1 = S.loff[k][cl + 3] - base;
          const int32_t vl = v1 < lcap ? v1 : lcap;
          const int32_t hl = hv - base;  // the home particle's own slot (pass 1 only)
          // LDS-resident slots, four per iteration for instruction-level parallelism
          for (; v + 4 <= vl; v += 4) {
            double qx[4], qy[4], qz[4];
            int32_t tj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              qx[u] = xs[v + u];
              qy[u] = ys[v + u];
              qz[u] = zs[v + u];
              tj[u] = ts[v + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const double ex = qx[u] - pi.x, ey = qy[u] - pi.y, ez = qz[u] - pi.z;
              const double r2 = (ex * ex + ey * ey) + ez * ez;
              if (v + u != hl && r2 < thr[tj[u]]) {
                if (cnt < cap) out[(size_t)cnt * stride] = (uint16_t)((v + u) | (tj[u] << 14));
                ++cnt;
              }
            }
          }
          for (; v < v1; ++v) {
            if (v == hl) continue;
            double qx, qy, qz;
            int32_t tj;
            if (v < lcap) {
              qx = xs[v];
              qy = ys[v];
              qz = zs[v];
              tj = ts[v];
            } else {
              const double4 q = fetch_slot(S, pos_tmp, v + base);
              qx = q.x;
              qy = q.y;
              qz = q.z;
              tj = (int32_t)q.w;
            }
            const double ex = qx - pi.x, ey = qy - pi.y, ez = qz - pi.z;
            const double r2 = (ex * ex + ey * ey) + ez * ez;
            if (r2 < thr[tj]) {
              if (cnt < cap) out[(size_t)cnt * stride] = (uint16_t)(v | (tj << 14));
              ++cnt;
            }
          }
        }
      }
      if (pass == 0) n0 = cnt;
      if (pass == 1) n1 = cnt - n0;
      __syncthreads();  // the next pass overwrites the staged rows
    }
    if (mine) {
      ncount[i] = cnt;
      nsplit[i] = (uint32_t)n0 | ((uint32_t)n1 << 16);
      if (cnt > cap || n0 > 0xffff || n1 > 0xffff) atomicOr(&st->err, kErrOverflow);
      // the new cell order becomes the live state
      pos[i] = pi;
      xref[i] = pi.x;
      xref[stride + i] = pi.y;
      xref[2 * (size_t)stride + i] = pi.z;
      vel[i] = vel_tmp[i];
      vel[stride + i] = vel_tmp[stride + i];
      vel[2 * (size_t)stride + i] = vel_tmp[2 * (size_t)stride + i];
      id[i] = id_tmp[i];
    }
  }
}

// Staged entries -> sorted particle indices (parity hook only).
__global__ __launch_bounds__(256) void k_decode_staged(
    const RowTile* __restrict__ rtiles, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ cell_start, int32_t stride, int32_t rows,
    const uint16_t* __restrict__ nbr, const int32_t* __restrict__ ncount,
    const uint32_t* __restrict__ nsplit, uint32_t* __restrict__ out) {
  __shared__ StageLayout S;
  const RowTile T = rtiles[blockIdx.x];
  const RepDesc R = reps[T.rep];
  build_layout(S, T, R, cell_start);
  const int32_t nh = S.home1 - S.home0;
  for (int32_t li = threadIdx.x; li < nh; li += blockDim.x) {
    const int32_t i = S.home0 + li;
    int32_t n = ncount[i];
    n = n < rows ? n : rows;
    const int32_t n0 = (int32_t)(nsplit[i] & 0xffffu), n1 = (int32_t)(nsplit[i] >> 16);
    for (int32_t k = 0; k < n; ++k) {
      const int pass = k < n0 ? 0 : (k < n0 + n1 ? 1 : 2);
      const int32_t v = (nbr[(size_t)k * stride + i] & 0x3fff) + pass_base(S, pass);
      const int p = piece_of(S, v);
      out[(size_t)k * stride + i] = (uint32_t)(S.pc_g[p] + (v - S.pc_l[p]));
    }
  }
}

}  // namespace

size_t nlist_staged_lds_bytes(int32_t lcap) { return (size_t)lcap * 25 + 8; }

void launch_nlist_staged(hipStream_t s, int32_t bt, int32_t nrt, const RowTile* rtiles,
                         const RepDesc* reps, const int32_t* rebuild, const PairTab* tab,
                         const int32_t* cell_start, int32_t stride, int32_t cap, int32_t lcap,
                         const double4* pos_tmp, const double* vel_tmp, const int32_t* id_tmp,
                         double4* pos, double* vel, int32_t* id, double* xref, uint16_t* nbr,
                         int32_t* ncount, uint32_t* nsplit, DevState* st) {
  const size_t lds = nlist_staged_lds_bytes(lcap);
  if (bt == 128)
    k_nlist_staged<128><<<nrt, 128, lds, s>>>(rtiles, reps, rebuild, tab, cell_start, stride, cap,
                                              lcap, pos_tmp, vel_tmp, id_tmp, pos, vel, id, xref,
                                              nbr, ncount, nsplit, st);
  else
    k_nlist_staged<256><<<nrt, 256, lds, s>>>(rtiles, reps, rebuild, tab, cell_start, stride, cap,
                                              lcap, pos_tmp, vel_tmp, id_tmp, pos, vel, id, xref,
                                              nbr, ncount, nsplit, st);
}

void launch_decode_staged(hipStream_t s, int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                          const int32_t* cell_start, int32_t stride, int32_t rows,
                          const uint16_t* nbr, const int32_t* ncount, const uint32_t* nsplit,
                          uint32_t* out) {
  k_decode_staged<<<nrt, 256, 0, s>>>(rtiles, reps, cell_start, stride, rows, nbr, ncount, nsplit,
                                      out);
}

}  // namespace mdk
