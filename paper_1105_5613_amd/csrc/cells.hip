// cells.hip -- state upload/download, periodic wrap + cell binning, and the
// stable counting sort of particles by (cell, original id).
//
// The cell grid follows the paper's cubic cells of side >= cutoff holding
// any number of particles (Fig. 1; "Grid-search method").  The doubly linked
// per-cell particle lists of the paper become, on the GPU, a counting sort:
// an atomic histogram per cell, an exclusive scan into cell_start, a scatter
// to the cell segments, and a per-cell rank sort by original id that makes
// the order deterministic, followed by a gather of the particle records into
// the new order.
#include "md_internal.h"

namespace mdk {
namespace {

__device__ inline void latch(DevState* st, int32_t bits) { atomicOr(&st->err, bits); }

__global__ void k_set_state(int32_t ntot, int32_t stride, const double* __restrict__ x,
                            const double* __restrict__ v, const int32_t* __restrict__ type,
                            int32_t ntypes, double4* __restrict__ pos, double* __restrict__ vel,
                            int32_t* __restrict__ id, int32_t* __restrict__ img, DevState* st) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  int32_t t = type[i];
  double x0 = x[3 * (size_t)i], x1 = x[3 * (size_t)i + 1], x2 = x[3 * (size_t)i + 2];
  double v0 = v[3 * (size_t)i], v1 = v[3 * (size_t)i + 1], v2 = v[3 * (size_t)i + 2];
  if (t < 0 || t >= ntypes) {
    latch(st, kErrType);
    t = 0;
  }
  if (!isfinite(x0 + x1 + x2 + v0 + v1 + v2)) latch(st, kErrNonFinite);
  pos[i] = make_double4(x0, x1, x2, (double)t);
  vel[i] = v0;
  vel[stride + i] = v1;
  vel[2 * (size_t)stride + i] = v2;
  id[i] = i;
  img[3 * (size_t)i] = 0;
  img[3 * (size_t)i + 1] = 0;
  img[3 * (size_t)i + 2] = 0;
}

__global__ void k_get_state(int32_t ntot, int32_t stride, const double4* __restrict__ pos,
                            const double* __restrict__ vel, const int32_t* __restrict__ id,
                            double* __restrict__ x, double* __restrict__ v) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  size_t o = 3 * (size_t)id[i];
  if (x) {
    double4 p = pos[i];
    x[o] = p.x;
    x[o + 1] = p.y;
    x[o + 2] = p.z;
  }
  if (v) {
    v[o] = vel[i];
    v[o + 1] = vel[stride + i];
    v[o + 2] = vel[2 * (size_t)stride + i];
  }
}

template <typename FT>
__global__ void k_get_forces(int32_t ntot, int32_t stride, const FT* __restrict__ frc,
                             const int32_t* __restrict__ id, FT* __restrict__ F) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  size_t o = 3 * (size_t)id[i];
  F[o] = frc[i];
  F[o + 1] = frc[stride + i];
  F[o + 2] = frc[2 * (size_t)stride + i];
}

__global__ void k_mark_rebuild(int32_t nrep, int32_t* rebuild, DevState* st) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrep) rebuild[r] = 1;
  if (r == 0) st->any_rebuild = 1;
}

// Capacity growth: row k of particle i moves from list_base(i, cap_old) +
// k * kSlice to list_base(i, cap_new) + k * kSlice; rows past the old
// capacity (truncated) are rebuilt afterwards.
template <typename E>
__global__ void k_relayout_list(int32_t ntot, const int32_t* __restrict__ ncount, int32_t cap_old,
                                int32_t cap_new, const E* __restrict__ src, E* __restrict__ dst) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const int32_t m = min(ncount[i], cap_old);
  const E* a = src + list_base(i, cap_old);
  E* b = dst + list_base(i, cap_new);
  for (int32_t k = 0; k < m; ++k) b[(size_t)k * kSlice] = a[(size_t)k * kSlice];
}

__global__ void k_zero_counts(int32_t ncells, const int32_t* __restrict__ cell_rep,
                              const int32_t* __restrict__ rebuild, const DevState* st,
                              int32_t* __restrict__ counts) {
  if (!st->any_rebuild) return;
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncells && rebuild[cell_rep[c]]) counts[c] = 0;
}

// One periodic wrap (enough between list builds, where every particle moved
// less than skin/2); x == L after rounding maps to 0 in the next image.
__device__ inline int32_t wrap1(double& c, double L, int32_t& bad) {
  int32_t d = 0;
  if (c < 0.0) {
    c += L;
    d = -1;
  } else if (c >= L) {
    c -= L;
    d = 1;
  }
  if (c == L) {
    c = 0.0;
    d += 1;
  }
  if (!(c >= 0.0 && c < L)) {
    bad = 1;
    c = 0.0;
  }
  return d;
}

__device__ inline int32_t cell_coord(double c, double inv_cell, int32_t nc) {
  int32_t q = (int32_t)(c * inv_cell);
  return q > nc - 1 ? nc - 1 : q;
}

// Wrap particle i of replica R, whose position p was just read from pos[i],
// into the box (p, pos[i] and the image counter updated; a coordinate that
// one wrap does not bring into [0, L) latches kErrStray) and return its
// cell, numbered from the first cell of all replicas.
__device__ inline int32_t bin_particle(int32_t i, double4& p, const RepDesc& R,
                                       double4* __restrict__ pos, const int32_t* __restrict__ id,
                                       int32_t* __restrict__ img, DevState* st) {
  const double4 p0 = p;
  int32_t bad = 0;
  int32_t dx = wrap1(p.x, R.L, bad);
  int32_t dy = wrap1(p.y, R.L, bad);
  int32_t dz = wrap1(p.z, R.L, bad);
  if (bad) latch(st, kErrStray);
  if (dx | dy | dz) {
    size_t o = 3 * (size_t)id[i];
    img[o] += dx;
    img[o + 1] += dy;
    img[o + 2] += dz;
  }
  // most particles stay in the box: write back only a changed position
  // (a tiny negative coordinate can wrap to L and then to 0 with no net
  // image change)
  if (bad || p.x != p0.x || p.y != p0.y || p.z != p0.z) pos[i] = p;
  int32_t qx = cell_coord(p.x, R.inv_cell, R.nc);
  int32_t qy = cell_coord(p.y, R.inv_cell, R.nc);
  int32_t qz = cell_coord(p.z, R.inv_cell, R.nc);
  return R.coff + (qz * R.nc + qy) * R.nc + qx;
}

// Wrap + bin.  Particles arrive in the cell order of the previous build, so
// the lanes of a wave form a few runs of equal cell: one atomic per run
// reserves the run's slots (the in-cell order is fixed later by the rank
// sort, so slot order does not matter).
__global__ __launch_bounds__(kTile) void k_bin(const Tile* __restrict__ tiles,
                                               const RepDesc* __restrict__ reps,
                                               const int32_t* __restrict__ rebuild,
                                               double4* __restrict__ pos,
                                               const int32_t* __restrict__ id,
                                               int32_t* __restrict__ img,
                                               int32_t* __restrict__ counts,
                                               int32_t* __restrict__ cell_of,
                                               int32_t* __restrict__ slot, DevState* st,
                                               int32_t ntiles, int32_t spread) {
  if (!st->any_rebuild) return;  // one flag load when nothing rebuilds
  const int32_t lt = spread ? xcd_spread(blockIdx.x, spread) : xcd_block(blockIdx.x, gridDim.x);
  if (lt >= ntiles) return;
  const Tile t = tiles[lt];
  if (!rebuild[t.rep]) return;
  const int lane = threadIdx.x & 63;
  const int32_t i = t.start + threadIdx.x;
  const int32_t wave0 = t.start + (int32_t)(threadIdx.x & ~63u);
  if (wave0 >= t.end) return;  // whole wave past the tile
  const bool active = i < t.end;
  const RepDesc R = reps[t.rep];
  int32_t c = -1;
  if (active) {
    double4 p = pos[i];
    c = bin_particle(i, p, R, pos, id, img, st);
    cell_of[i] = c;
  }
  // runs of equal cell among consecutive active lanes
  const int32_t cp = __shfl_up(c, 1, 64);
  const bool lead = active && (lane == 0 || cp != c);
  const uint64_t leaders = __ballot(lead);
  const uint64_t act = __ballot(active);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int my_lead = 63 - __builtin_clzll((leaders & upto) | 1ull);
  const uint64_t after = my_lead == 63 ? 0ull : (leaders >> (my_lead + 1));
  const int n_act = __popcll(act);
  const int next = after ? my_lead + 1 + __builtin_ctzll(after) : n_act;
  int32_t base = 0;
  if (lead) base = atomicAdd(&counts[c], next - my_lead);
  base = __shfl(base, my_lead, 64);
  if (active) slot[i] = base + (lane - my_lead);
}

// ---- exclusive scan of the cell counts ------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) base += wsum[k];
    tot += wsum[k];
  }
  *total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t* __restrict__ in,
                                                              int32_t* __restrict__ out,
                                                              int32_t* __restrict__ bsum,
                                                              int32_t n, const DevState* st) {
  if (!st->any_rebuild) return;
  const int32_t base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int32_t loc[kScanPer];
  int32_t s = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    int32_t v = (base + e < n) ? in[base + e] : 0;
    loc[e] = s;
    s += v;
  }
  int32_t tot;
  int32_t pre = block_exclusive_scan(s, &tot);
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (base + e < n) out[base + e] = pre + loc[e];
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ bsum, int32_t nb,
                                                   const DevState* st) {
  if (!st->any_rebuild) return;
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int32_t c0 = 0; c0 < nb; c0 += 1024) {
    int32_t k = c0 + threadIdx.x;
    int32_t v = k < nb ? bsum[k] : 0;
    int32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
      int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t base = carry_s, tot = 0;
    for (int q = 0; q < 16; ++q) {
      if (q < w) base += wsum[q];
      tot += wsum[q];
    }
    if (k < nb) bsum[k] = base + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry_s;
}

// Small grids: the whole exclusive scan in one block, chunk by chunk with a
// running carry (one launch instead of three).
// Eight consecutive counts of one thread (zeros past n), as two 16-byte
// loads when the group lies inside the array.
__device__ inline void load8(const int32_t* __restrict__ in, int32_t base, int32_t n,
                             int32_t v[8]) {
  if (base + 8 <= n) {
    const int4 a = *reinterpret_cast<const int4*>(in + base);
    const int4 b = *reinterpret_cast<const int4*>(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = base + e < n ? in[base + e] : 0;
  }
}

// Exclusive scan of up to 65,536 counts in one block: 8,192 per pass, each
// thread 8 consecutive values; the next pass's values are loaded before the
// current pass's block scan so the passes do not each wait a full memory
// round trip.  Requires `in` 16-byte aligned (device allocations are).
__global__ __launch_bounds__(1024) void k_scan_single(const int32_t* __restrict__ in,
                                                      int32_t* __restrict__ out, int32_t n,
                                                      const DevState* st) {
  if (!st->any_rebuild) return;
  __shared__ int32_t wsum[16];
  constexpr int kPer = 8, kPass = 1024 * kPer;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t carry = 0;
  int32_t cur[kPer], nxt[kPer] = {};
  load8(in, threadIdx.x * kPer, n, cur);
  for (int32_t c0 = 0; c0 < n; c0 += kPass) {
    const int32_t base = c0 + threadIdx.x * kPer;
    if (c0 + kPass < n) load8(in, base + kPass, n, nxt);
    int32_t loc[kPer];
    int32_t s = 0;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      loc[e] = s;
      s += cur[e];
    }
    int32_t x = s;
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t pre = carry, tot = 0;
    for (int q = 0; q < 16; ++q) {
      if (q < w) pre += wsum[q];
      tot += wsum[q];
    }
    pre += x - s;
    if (base + kPer <= n) {
      *reinterpret_cast<int4*>(out + base) =
          make_int4(pre + loc[0], pre + loc[1], pre + loc[2], pre + loc[3]);
      *reinterpret_cast<int4*>(out + base + 4) =
          make_int4(pre + loc[4], pre + loc[5], pre + loc[6], pre + loc[7]);
    } else {
#pragma unroll
      for (int e = 0; e < kPer; ++e)
        if (base + e < n) out[base + e] = pre + loc[e];
    }
    carry += tot;
    __syncthreads();  // wsum is rewritten by the next pass
#pragma unroll
    for (int e = 0; e < kPer; ++e) cur[e] = nxt[e];
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ bsum,
                           int32_t n, int32_t nb, const DevState* st) {
  if (!st->any_rebuild) return;
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / kScanBlock];
  else if (i == n) out[n] = bsum[nb];
}

__global__ __launch_bounds__(kTile) void k_scatter(const Tile* __restrict__ tiles,
                                                   const int32_t* __restrict__ rebuild,
                                                   const int32_t* __restrict__ cell_of,
                                                   const int32_t* __restrict__ slot,
                                                   const int32_t* __restrict__ cell_start,
                                                   int32_t* __restrict__ tmp_src,
                                                   const DevState* __restrict__ st,
                                                   int32_t ntiles, int32_t spread) {
  if (!st->any_rebuild) return;
  const int32_t lt = spread ? xcd_spread(blockIdx.x, spread) : xcd_block(blockIdx.x, gridDim.x);
  if (lt >= ntiles) return;
  const Tile t = tiles[lt];
  if (!rebuild[t.rep]) return;
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  tmp_src[cell_start[cell_of[i]] + slot[i]] = i;
}

// One wave per cell: rank the cell's particles by original id (ids are
// unique) and gather their records to cell_start + rank.
__global__ __launch_bounds__(256) void k_cell_gather(
    int32_t ncells, const int32_t* __restrict__ cell_rep, const int32_t* __restrict__ rebuild,
    const int32_t* __restrict__ cell_start, const int32_t* __restrict__ tmp_src, int32_t stride,
    const int32_t* __restrict__ id, const double4* __restrict__ pos,
    const double* __restrict__ vel, int32_t* __restrict__ id_tmp, double4* __restrict__ pos_tmp,
    double* __restrict__ vel_tmp, const DevState* __restrict__ st) {
  if (!st->any_rebuild) return;
  const int32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= ncells) return;
  if (!rebuild[cell_rep[c]]) return;
  const int32_t s = cell_start[c], n = cell_start[c + 1] - s;
  if (n <= 64) {
    int32_t src = 0, myid = 0x7fffffff;
    if (lane < n) {
      src = tmp_src[s + lane];
      myid = id[src];
    }
    int32_t rank = 0;
    for (int m = 0; m < n; ++m) {
      int32_t o = __shfl(myid, m, 64);
      rank += (o < myid) ? 1 : 0;
    }
    if (lane < n) {
      int32_t d = s + rank;
      id_tmp[d] = myid;
      pos_tmp[d] = pos[src];
      vel_tmp[d] = vel[src];
      vel_tmp[stride + d] = vel[stride + src];
      vel_tmp[2 * (size_t)stride + d] = vel[2 * (size_t)stride + src];
    }
  } else {
    // crowded cell: quadratic rank straight from memory
    for (int32_t k = lane; k < n; k += 64) {
      int32_t src = tmp_src[s + k];
      int32_t myid = id[src];
      int32_t rank = 0;
      for (int32_t m = 0; m < n; ++m) rank += (id[tmp_src[s + m]] < myid) ? 1 : 0;
      int32_t d = s + rank;
      id_tmp[d] = myid;
      pos_tmp[d] = pos[src];
      vel_tmp[d] = vel[src];
      vel_tmp[stride + d] = vel[stride + src];
      vel_tmp[2 * (size_t)stride + d] = vel[2 * (size_t)stride + src];
    }
  }
}

// The whole chain for a context of one replica with at most kSmallN
// particles and kSmallCells cells, in one block: wrap + bin (histogram in
// LDS), the exclusive scan, then the ids of every cell in slot order in LDS
// and each particle's rank among its cell's ids counted there, with a block
// barrier between the phases.  It leaves the arrays of the launches above
// (cell_start and the records in the new order) bit for bit: the slots
// within a cell come out of the atomics in another order, which the rank by
// id removes.  At this size a launch costs far more than its work, so a
// step that does not rebuild pays one gated launch instead of four.  Thread
// t takes particles t, t + 1024, ... (at most kSmallN / kSmallThreads) in
// every phase, keeps their cells, slots and ids in registers, and reads the
// records of all of them with one round trip per phase.
__global__ __launch_bounds__(kSmallThreads) void k_chain_small(
    const RepDesc* __restrict__ reps, const int32_t* __restrict__ rebuild,
    double4* __restrict__ pos, const int32_t* __restrict__ id, int32_t* __restrict__ img,
    int32_t* __restrict__ cell_start, int32_t stride, const double* __restrict__ vel,
    int32_t* __restrict__ id_tmp, double4* __restrict__ pos_tmp, double* __restrict__ vel_tmp,
    DevState* st) {
  constexpr int kPer = kSmallN / kSmallThreads;
  __shared__ int32_t s_start[kSmallCells + 1];  // counts, then first particle of each cell
  __shared__ int32_t s_id[kSmallN];             // ids by cell, then slot
  __shared__ int32_t s_wsum[kSmallThreads / 64];
  if (!st->any_rebuild) return;
  if (!rebuild[0]) return;
  const RepDesc R = reps[0];
  const int32_t ncl = R.nc * R.nc * R.nc;
  const int32_t end = R.off + R.n;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int32_t c = t; c <= ncl; c += kSmallThreads) s_start[c] = 0;
  int32_t idv[kPer], cl[kPer], sl[kPer];
  {
    double4 pv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t i = R.off + t + u * kSmallThreads;
      if (i < end) {
        pv[u] = pos[i];
        idv[u] = id[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t i = R.off + t + u * kSmallThreads;
      cl[u] = 0;
      sl[u] = 0;
      if (i < end) {
        // writes the wrapped position back to pos[i] when it changed
        cl[u] = bin_particle(i, pv[u], R, pos, id, img, st) - R.coff;
        sl[u] = atomicAdd(&s_start[cl[u]], 1);
      }
    }
  }
  __syncthreads();
  // exclusive scan: thread t holds cells [4t, 4t + 4)
  int32_t v[4], loc[4], sum = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int32_t c = 4 * t + e;
    v[e] = c < ncl ? s_start[c] : 0;
    loc[e] = sum;
    sum += v[e];
  }
  int32_t x = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_wsum[w] = x;
  __syncthreads();  // also: every count is read before the starts overwrite them
  int32_t pre = R.off + x - sum, tot = R.off;
#pragma unroll
  for (int q = 0; q < kSmallThreads / 64; ++q) {
    if (q < w) pre += s_wsum[q];
    tot += s_wsum[q];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int32_t c = 4 * t + e;
    if (c < ncl) s_start[c] = pre + loc[e];
  }
  if (t == 0) s_start[ncl] = tot;
  __syncthreads();
  for (int32_t c = t; c <= ncl; c += kSmallThreads) cell_start[R.coff + c] = s_start[c];
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (R.off + t + u * kSmallThreads < end) s_id[s_start[cl[u]] - R.off + sl[u]] = idv[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int32_t i = R.off + t + u * kSmallThreads;
    if (i < end) {
      const int32_t lo = s_start[cl[u]] - R.off, hi = s_start[cl[u] + 1] - R.off;
      int32_t rank = 0;
      for (int32_t m = lo; m < hi; ++m) rank += s_id[m] < idv[u] ? 1 : 0;  // ids are unique
      const int32_t d = R.off + lo + rank;
      id_tmp[d] = idv[u];
      pos_tmp[d] = pos[i];  // this thread's own write-back, if any
      vel_tmp[d] = vel[i];
      vel_tmp[stride + d] = vel[stride + i];
      vel_tmp[2 * (size_t)stride + d] = vel[2 * (size_t)stride + i];
    }
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_set_state(hipStream_t s, int32_t ntot, int32_t stride, const double* x,
                      const double* v, const int32_t* type, int32_t ntypes, double4* pos,
                      double* vel, int32_t* id, int32_t* img, DevState* st) {
  k_set_state<<<nblk(ntot, 256), 256, 0, s>>>(ntot, stride, x, v, type, ntypes, pos, vel, id,
                                              img, st);
}

void launch_get_state(hipStream_t s, int32_t ntot, int32_t stride, const double4* pos,
                      const double* vel, const int32_t* id, double* x, double* v) {
  k_get_state<<<nblk(ntot, 256), 256, 0, s>>>(ntot, stride, pos, vel, id, x, v);
}

void launch_get_forces(hipStream_t s, int32_t ntot, int32_t stride, const void* frc,
                       int32_t mixed, const int32_t* id, void* F) {
  if (mixed)
    k_get_forces<float><<<nblk(ntot, 256), 256, 0, s>>>(ntot, stride, (const float*)frc, id,
                                                       (float*)F);
  else
    k_get_forces<double><<<nblk(ntot, 256), 256, 0, s>>>(ntot, stride, (const double*)frc, id,
                                                        (double*)F);
}

void launch_relayout_list(hipStream_t s, int32_t ntot, const int32_t* ncount, int32_t cap_old,
                          int32_t cap_new, int32_t elem, const void* src, void* dst) {
  if (elem == 2)
    k_relayout_list<uint16_t><<<nblk(ntot, 256), 256, 0, s>>>(
        ntot, ncount, cap_old, cap_new, (const uint16_t*)src, (uint16_t*)dst);
  else
    k_relayout_list<uint32_t><<<nblk(ntot, 256), 256, 0, s>>>(
        ntot, ncount, cap_old, cap_new, (const uint32_t*)src, (uint32_t*)dst);
}

void launch_mark_rebuild(hipStream_t s, int32_t nrep, int32_t* rebuild, DevState* st) {
  k_mark_rebuild<<<nblk(nrep, 256), 256, 0, s>>>(nrep, rebuild, st);
}

void launch_zero_counts(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const int32_t* rebuild, const DevState* st, int32_t* counts) {
  k_zero_counts<<<nblk(ncells, 256), 256, 0, s>>>(ncells, cell_rep, rebuild, st, counts);
}

void launch_bin(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                const int32_t* rebuild, double4* pos, const int32_t* id, int32_t* img,
                int32_t* counts, int32_t* cell_of, int32_t* slot, DevState* st, int32_t spread) {
  const int32_t grid = spread ? spread_grid(ntiles, spread) : ntiles;
  k_bin<<<grid, kTile, 0, s>>>(tiles, reps, rebuild, pos, id, img, counts, cell_of, slot, st,
                               ntiles, spread);
}

size_t scan_bsum_elems(int32_t ncells) { return (size_t)nblk(ncells, kScanBlock) + 1; }

void launch_scan(hipStream_t s, int32_t ncells, const int32_t* counts, int32_t* cell_start,
                 int32_t* bsum, const DevState* st) {
  if (ncells <= 65536) {
    k_scan_single<<<1, 1024, 0, s>>>(counts, cell_start, ncells, st);
    return;
  }
  int32_t nb = (int32_t)nblk(ncells, kScanBlock);
  k_scan_blocks<<<nb, kScanThreads, 0, s>>>(counts, cell_start, bsum, ncells, st);
  k_scan_top<<<1, 1024, 0, s>>>(bsum, nb, st);
  k_scan_add<<<nblk(ncells + 1, 256), 256, 0, s>>>(cell_start, bsum, ncells, nb, st);
}

void launch_scatter(hipStream_t s, int32_t ntiles, const Tile* tiles, const int32_t* rebuild,
                    const int32_t* cell_of, const int32_t* slot, const int32_t* cell_start,
                    int32_t* tmp_src, const DevState* st, int32_t spread) {
  const int32_t grid = spread ? spread_grid(ntiles, spread) : ntiles;
  k_scatter<<<grid, kTile, 0, s>>>(tiles, rebuild, cell_of, slot, cell_start, tmp_src, st,
                                   ntiles, spread);
}

void launch_chain_small(hipStream_t s, const RepDesc* reps, const int32_t* rebuild,
                        double4* pos, const int32_t* id, int32_t* img, int32_t* cell_start,
                        int32_t stride, const double* vel, int32_t* id_tmp, double4* pos_tmp,
                        double* vel_tmp, DevState* st) {
  k_chain_small<<<1, kSmallThreads, 0, s>>>(reps, rebuild, pos, id, img, cell_start, stride,
                                            vel, id_tmp, pos_tmp, vel_tmp, st);
}

void launch_cell_gather(hipStream_t s, int32_t ncells, const int32_t* cell_rep,
                        const int32_t* rebuild, const int32_t* cell_start,
                        const int32_t* tmp_src, int32_t stride, const int32_t* id,
                        const double4* pos, const double* vel, int32_t* id_tmp,
                        double4* pos_tmp, double* vel_tmp, const DevState* st) {
  k_cell_gather<<<nblk(ncells, 4), 256, 0, s>>>(ncells, cell_rep, rebuild, cell_start, tmp_src,
                                                stride, id, pos, vel, id_tmp, pos_tmp, vel_tmp,
                                                st);
}

}  // namespace mdk
