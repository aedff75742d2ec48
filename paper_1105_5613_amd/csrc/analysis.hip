// analysis.hip -- observables of the glass study: mean-squared displacement
// of the unwrapped positions, and the radial distribution function
//   g(r) = 2V/N^2 < sum_{i<j} delta(r - r_ij) >
// of the glass-transition section, as a histogram of all pair distances
// below rmax under the minimum image (exact FP64 distances; every unordered
// pair once).  Compiled without FMA contraction so the distances (and hence
// the bins) round exactly like a plain FP64 evaluation.
#include "md_internal.h"

#pragma clang fp contract(off)

namespace mdk {
namespace {

// Unwrapped positions u = x + img L of every particle into u0 (original id order).
__global__ __launch_bounds__(kTile) void k_msd_ref(const Tile* __restrict__ tiles,
                                                   const RepDesc* __restrict__ reps,
                                                   const double4* __restrict__ pos,
                                                   const int32_t* __restrict__ id,
                                                   const int32_t* __restrict__ img,
                                                   double* __restrict__ u0) {
  const Tile t = tiles[blockIdx.x];
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  const double L = reps[t.rep].L;
  const double4 p = pos[i];
  const size_t o = 3 * (size_t)id[i];
  u0[o] = p.x + (double)img[o] * L;
  u0[o + 1] = p.y + (double)img[o + 1] * L;
  u0[o + 2] = p.z + (double)img[o + 2] * L;
}

// Per-tile sums of |u - u0|^2.
__global__ __launch_bounds__(kTile) void k_msd(const Tile* __restrict__ tiles,
                                               const RepDesc* __restrict__ reps,
                                               const double4* __restrict__ pos,
                                               const int32_t* __restrict__ id,
                                               const int32_t* __restrict__ img,
                                               const double* __restrict__ u0,
                                               double* __restrict__ part) {
  __shared__ double red[kTile / 64];
  const Tile t = tiles[blockIdx.x];
  const int32_t i = t.start + threadIdx.x;
  double s = 0.0;
  if (i < t.end) {
    const double L = reps[t.rep].L;
    const double4 p = pos[i];
    const size_t o = 3 * (size_t)id[i];
    const double dx = p.x + (double)img[o] * L - u0[o];
    const double dy = p.y + (double)img[o + 1] * L - u0[o + 1];
    const double dz = p.z + (double)img[o + 2] * L - u0[o + 2];
    s = (dx * dx + dy * dy) + dz * dz;
  }
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0];
    for (int k = 1; k < kTile / 64; ++k) a += red[k];
    part[blockIdx.x] = a;
  }
}

// One block per replica: mean of the tile sums in a fixed order.
__global__ __launch_bounds__(256) void k_msd_reduce(const RepDesc* __restrict__ reps,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double red[256];
  const RepDesc R = reps[blockIdx.x];
  double s = 0.0;
  for (int32_t b = R.tile0 + threadIdx.x; b < R.tile1; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] / (double)R.n;
}

// Pair-distance histogram of particles [off, off + n): block b takes i in a
// tile of 256, loops over j tiles staged in LDS, counts j > i with r < rmax.
constexpr int kRdfTile = 256;
__global__ __launch_bounds__(kRdfTile) void k_rdf(const double4* __restrict__ pos, int32_t off,
                                                  int32_t n, double L, double rmax, double dr,
                                                  int32_t nbins,
                                                  unsigned long long* __restrict__ hist) {
  extern __shared__ unsigned int s_h[];
  __shared__ double jx[kRdfTile], jy[kRdfTile], jz[kRdfTile];
  for (int b = threadIdx.x; b < nbins; b += kRdfTile) s_h[b] = 0u;
  const int32_t i = blockIdx.x * kRdfTile + threadIdx.x;
  const bool act = i < n;
  const double4 pi = pos[off + (act ? i : 0)];
  for (int32_t j0 = blockIdx.x * kRdfTile; j0 < n; j0 += kRdfTile) {
    __syncthreads();
    const int32_t jl = j0 + threadIdx.x;
    if (jl < n) {
      const double4 q = pos[off + jl];
      jx[threadIdx.x] = q.x;
      jy[threadIdx.x] = q.y;
      jz[threadIdx.x] = q.z;
    }
    __syncthreads();
    const int32_t m = n - j0 < kRdfTile ? n - j0 : kRdfTile;
    if (act) {
      for (int32_t k = 0; k < m; ++k) {
        if (j0 + k <= i) continue;
        double dx = pi.x - jx[k], dy = pi.y - jy[k], dz = pi.z - jz[k];
        const double kx = rint(dx / L), ky = rint(dy / L), kz = rint(dz / L);
        const double tx = L * kx, ty = L * ky, tz = L * kz;
        dx = dx - tx;
        dy = dy - ty;
        dz = dz - tz;
        const double r = sqrt((dx * dx + dy * dy) + dz * dz);
        if (r < rmax) {
          int32_t b = (int32_t)(r / dr);
          b = b >= nbins ? nbins - 1 : b;
          atomicAdd(&s_h[b], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kRdfTile)
    if (s_h[b]) atomicAdd(&hist[b], (unsigned long long)s_h[b]);
}

// Pair-distance histogram over the cells of replica [c0, c0 + nc^3): one
// wave per home cell; the lanes take packed candidates of the 27 neighbour
// cells (distinct for nc >= 3), the wave walks the home particles, and each
// unordered pair is counted once (sorted partner index above the home's).
// Distances use the same minimum-image arithmetic as k_rdf; every pair
// closer than the cell side minus the skin is in the stencil while the
// skin rule holds.
__global__ __launch_bounds__(256) void k_rdf_cells(int32_t c0, int32_t nc,
                                                   const int32_t* __restrict__ cell_start,
                                                   const double4* __restrict__ pos, double L,
                                                   double rmax, double dr, int32_t nbins,
                                                   unsigned long long* __restrict__ hist) {
  extern __shared__ unsigned int s_h[];
  __shared__ int32_t s_pre[4][28], s_k0[4][27];
  for (int b = threadIdx.x; b < nbins; b += 256) s_h[b] = 0u;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t lc = (int32_t)blockIdx.x * 4 + w;
  if (lc < nc * nc * nc) {
    const int32_t qx = lc % nc, qy = (lc / nc) % nc, qz = lc / (nc * nc);
    const int32_t h0 = cell_start[c0 + lc], nh = cell_start[c0 + lc + 1] - h0;
    if (lane < 27) {
      const int32_t nx = (qx + lane % 3 - 1 + nc) % nc, ny = (qy + (lane / 3) % 3 - 1 + nc) % nc,
                    nz = (qz + lane / 9 - 1 + nc) % nc;
      const int32_t cn = c0 + (nz * nc + ny) * nc + nx;
      s_k0[w][lane] = cell_start[cn];
      s_pre[w][lane] = cell_start[cn + 1] - cell_start[cn];
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
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t ncand = s_pre[w][27];
    for (int32_t base = 0; base < ncand; base += 64) {
      const int32_t v = base + lane;
      const bool valid = v < ncand;
      int p = 0;
#pragma unroll
      for (int step = 16; step >= 1; step >>= 1)
        if (p + step <= 26 && s_pre[w][p + step] <= v) p += step;
      const int32_t k = valid ? s_k0[w][p] + (v - s_pre[w][p]) : h0;
      const double4 q = pos[k];
      for (int32_t h = 0; h < nh; ++h) {
        const int32_t i = __builtin_amdgcn_readfirstlane(h0 + h);
        const double4 pa = pos[i];
        if (valid && k > i) {
          double dx = pa.x - q.x, dy = pa.y - q.y, dz = pa.z - q.z;
          const double kx = rint(dx / L), ky = rint(dy / L), kz = rint(dz / L);
          const double tx = L * kx, ty = L * ky, tz = L * kz;
          dx = dx - tx;
          dy = dy - ty;
          dz = dz - tz;
          const double r = sqrt((dx * dx + dy * dy) + dz * dz);
          if (r < rmax) {
            int32_t b = (int32_t)(r / dr);
            b = b >= nbins ? nbins - 1 : b;
            atomicAdd(&s_h[b], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 256)
    if (s_h[b]) atomicAdd(&hist[b], (unsigned long long)s_h[b]);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ a, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

}  // namespace

void launch_zero_u64(hipStream_t s, unsigned long long* a, int32_t n) {
  k_zero_u64<<<(n + 255) / 256, 256, 0, s>>>(a, n);
}

void launch_rdf_cells(hipStream_t s, int32_t c0, int32_t nc, const int32_t* cell_start,
                      const double4* pos, double L, double rmax, int32_t nbins,
                      unsigned long long* hist) {
  const double dr = rmax / nbins;
  const int32_t ncell = nc * nc * nc;
  k_rdf_cells<<<(ncell + 3) / 4, 256, sizeof(unsigned int) * nbins, s>>>(
      c0, nc, cell_start, pos, L, rmax, dr, nbins, hist);
}

void launch_msd_ref(hipStream_t s, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                    const double4* pos, const int32_t* id, const int32_t* img, double* u0) {
  k_msd_ref<<<ntiles, kTile, 0, s>>>(tiles, reps, pos, id, img, u0);
}

void launch_msd(hipStream_t s, int32_t ntiles, int32_t nrep, const Tile* tiles,
                const RepDesc* reps, const double4* pos, const int32_t* id, const int32_t* img,
                const double* u0, double* part, double* out) {
  k_msd<<<ntiles, kTile, 0, s>>>(tiles, reps, pos, id, img, u0, part);
  k_msd_reduce<<<nrep, 256, 0, s>>>(reps, part, out);
}

void launch_rdf(hipStream_t s, const double4* pos, int32_t off, int32_t n, double L, double rmax,
                int32_t nbins, unsigned long long* hist) {
  const double dr = rmax / nbins;
  k_rdf<<<(n + kRdfTile - 1) / kRdfTile, kRdfTile, sizeof(unsigned int) * nbins, s>>>(
      pos, off, n, L, rmax, dr, nbins, hist);
}

}  // namespace mdk
