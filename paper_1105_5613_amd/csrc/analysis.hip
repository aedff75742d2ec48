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

}  // namespace

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
