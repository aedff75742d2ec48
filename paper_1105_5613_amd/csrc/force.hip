// force.hip -- the pair-force hot spot: truncated shifted-force pair
// potential (Eq. (1)/(2) with the shifted-force form Eq. (3)) summed over the
// full neighbour list, with per-particle potential energy and virial halves
// reduced to per-tile FP64 partials.
//
// FP64 form: everything in double; 1/r from an FP32 reciprocal-square-root
// seed refined by two Newton-Raphson steps y <- y (3 - r^2 y^2) / 2, the
// scheme the paper uses on BlueGene/P ("BlueGene specific optimizations").
// Mixed form: neighbours are gathered as 16-byte records holding their
// offsets from the build-time cell centre in 32-bit fixed point (make_recq);
// the list entry carries the cell offset d of the pair, so the displacement
// is (off_i - off_j) + d * side, formed in FP64 from the exact integer
// difference and a table of d * side by the entry's code (error ~1e-9 from
// the fixed-point positions), with r^2 and the cut-off test in FP64; one
// gather per entry instead of two; the pair arithmetic from r^2 on and the
// per-particle force sum are FP32; per-particle energy/virial are widened to
// FP64 for the reductions.
//
// One thread per particle (tpp = 1) walks its ELL row; threads per particle
// tpp in {2, 4, 8} split the row into interleaved slots and combine their
// partial sums with cross-lane shuffles.  The walk is software-pipelined: the
// list entries of the next chunk of U slots are loaded while the U gathered
// neighbour positions of the current chunk are processed, so each lane keeps
// U gathers and U index loads in flight instead of one dependent pair.
#include "md_internal.h"

namespace mdk {
namespace {

__device__ inline double rsqrt_nr(double r2) {
  double y = (double)__builtin_amdgcn_rsqf((float)r2);
  const double h = 0.5 * r2;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

template <typename T>
struct PairLds {
  T rc2[16], sig2[16], c12[16], c6[16], f12[16], f6[16], vc[16], fs[16], rc[16];
};

template <typename T>
__device__ inline void load_pair(PairLds<T>& s, const PairTab* __restrict__ tab) {
  const int k = threadIdx.x;
  if (k < 16) {
    s.rc2[k] = (T)tab->rc2[k];
    s.sig2[k] = (T)tab->sig2[k];
    s.c12[k] = (T)tab->c12[k];
    s.c6[k] = (T)tab->c6[k];
    s.f12[k] = (T)tab->f12[k];
    s.f6[k] = (T)tab->f6[k];
    s.vc[k] = (T)tab->vc[k];
    s.fs[k] = (T)tab->fs[k];
    s.rc[k] = (T)tab->rc[k];
  }
}

// Mixed form: one 64-byte LDS record per species pair, so the cut-off test
// and the pair constants take one address computation (ab << 6).
struct alignas(16) PairRec {
  float sig2, f12, f6, fs;  // force
  double rc2;               // the FP64 cut-off test
  double pad;
  float c12, c6, vc, rc;    // energy
  float pad2[4];
};
static_assert(sizeof(PairRec) == 64, "PairRec is addressed as ab << 6");

__device__ inline int32_t decode_shift(uint32_t e, int lsb) {
  // two-bit two's-complement field at bit lsb of e
  return ((int32_t)(e << (30 - lsb))) >> 30;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Deterministic block sum of three values; result valid in thread 0.
__device__ inline void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][kTile / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = red[0][0];
    b = red[1][0];
    c = red[2][0];
    for (int k = 1; k < kTile / 64; ++k) {
      a += red[0][k];
      b += red[1][k];
      c += red[2][k];
    }
  }
}

// List entry k of a row.  NTL (a list larger than the last-level cache
// could hold): non-temporal loads, so the entries streamed once per launch
// do not evict the neighbour records from the L2.  A list that fits stays
// cached from one launch to the next and is read normally.
template <bool NTL>
__device__ inline uint32_t list_entry(const uint32_t* p) {
  if constexpr (NTL)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Block reduction of (sum, sum, sum, max); results valid in thread 0.
__device__ inline void block_sum3_max(double& a, double& b, double& c, double& m) {
  __shared__ double red[4][kTile / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
    red[3][w] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = red[0][0];
    b = red[1][0];
    c = red[2][0];
    m = red[3][0];
    for (int k = 1; k < kTile / 64; ++k) {
      a += red[0][k];
      b += red[1][k];
      c += red[2][k];
      m = fmax(m, red[3][k]);
    }
  }
}

// MODE 0: forces only.  MODE 1: forces and the step's second half kick.
// MODE 2 (NVE, one replica): as MODE 1, then the next step's first half kick
// and drift with the same arithmetic as k_kick_drift; the drifted positions
// go to pos_out / pos16_out (the other buffer of a pair: the neighbour
// records of this launch are read from pos / pos16), the forces are not
// stored (the next kick has used them), the largest squared displacement
// from xref per logical block goes to the fourth partial, and the cell
// histogram of the next rebuild is cleared (nzero cells).
// EN = false (in-step launches on steps whose observables are not read):
// the per-pair energy and virial terms are skipped and their partials are 0.
template <bool MIXED, int MODE, int TPP, int U, bool EN, bool NTL>
__global__ __launch_bounds__(kTile) void k_force(
    const Tile* __restrict__ tiles, const RepDesc* __restrict__ reps,
    const PairTab* __restrict__ tab, const double4* __restrict__ pos,
    const int4* __restrict__ pos16, double* __restrict__ vel, void* __restrict__ frc_,
    const uint32_t* __restrict__ nbr, const int32_t* __restrict__ ncount, int32_t stride,
    int32_t cap, double dt, double* __restrict__ part, DevState* st, FuseOut fo) {
  using T = typename std::conditional<MIXED, float, double>::type;
  __shared__ PairLds<T> P;
  __shared__ double s_mass[4], s_im[4];
  __shared__ double4 s_doff[64];  // mixed: d * cell side for each entry code
  __shared__ PairRec s_pr[16];    // mixed: the pair constants, one record per pair
  if (halted(st)) {
    // a list build queued before this launch overflowed (see kHalt): the
    // step is not taken; the later queued rebuild chains are switched off,
    // and a fused launch hands the positions unchanged to the buffer the
    // host swaps in
    if (blockIdx.x == 0 && threadIdx.x == 0) st->any_rebuild = 0;
    if constexpr (MODE == 2) {
      const int32_t hb = xcd_block(blockIdx.x, gridDim.x);
      const Tile th = tiles[hb / TPP];
      const int32_t ih = th.start + (hb % TPP) * (kTile / TPP) + threadIdx.x / TPP;
      if (ih < th.end && threadIdx.x % TPP == 0) {
        fo.pos_out[ih] = pos[ih];
        if constexpr (MIXED) fo.pos16_out[ih] = pos16[ih];
      }
    }
    return;
  }
  load_pair<T>(P, tab);
  if (threadIdx.x < 4) {
    s_mass[threadIdx.x] = tab->mass[threadIdx.x];
    s_im[threadIdx.x] = tab->inv_mass[threadIdx.x];
  }
  if constexpr (MODE == 2) {
    const int32_t gz = blockIdx.x * kTile + threadIdx.x;
    if (gz < fo.nzero) fo.counts[gz] = 0;
  }

  // with TPP lanes per particle a block covers kTile / TPP particles; a tile
  // of kTile particles takes TPP consecutive (logical) blocks
  const int32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int32_t tile_id = lb / TPP;
  const int32_t sub = lb % TPP;
  const Tile t = tiles[tile_id];
  const RepDesc& Rp = reps[t.rep];
  if (MIXED && threadIdx.x < 64) {
    const double sd = Rp.cside;
    const uint32_t c = threadIdx.x << kIdxBits;
    s_doff[threadIdx.x] = make_double4((double)decode_shift(c, 26) * sd,
                                       (double)decode_shift(c, 28) * sd,
                                       (double)decode_shift(c, 30) * sd, 0.0);
    if (threadIdx.x < 16) {
      const int k = threadIdx.x;
      PairRec r;
      r.sig2 = (float)tab->sig2[k];
      r.f12 = (float)tab->f12[k];
      r.f6 = (float)tab->f6[k];
      r.fs = (float)tab->fs[k];
      r.rc2 = tab->rc2[k];
      r.pad = 0.0;
      r.c12 = (float)tab->c12[k];
      r.c6 = (float)tab->c6[k];
      r.vc = (float)tab->vc[k];
      r.rc = (float)tab->rc[k];
      r.pad2[0] = r.pad2[1] = r.pad2[2] = r.pad2[3] = 0.0f;
      s_pr[k] = r;
    }
  }
  __syncthreads();
  const double L = Rp.L;
  const int32_t lane_p = threadIdx.x % TPP;
  const int32_t i = t.start + sub * (kTile / TPP) + threadIdx.x / TPP;
  const bool active = i < t.end;

  double pe = 0.0, w = 0.0, ke = 0.0;
  T fx = 0, fy = 0, fz = 0;
  T pe_i = 0, w_i = 0;
  int32_t ti = 0;
  uint32_t wbits = 0;  // mixed: the home record's species and cell code
  if (active) {
    int32_t n = ncount[i];
    n = n < cap ? n : cap;
    const uint32_t* row = nbr + list_base(i, cap);
    // entries are fetched one chunk of U ahead; slots past n point at the
    // particle itself and are masked out
    const uint32_t self = (uint32_t)i;
    uint32_t e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t k = lane_p + u * TPP;
      e[u] = k < n ? list_entry<NTL>(row + (size_t)k * kSlice) : self;
    }
    if constexpr (MIXED) {
      // 16-byte fixed-point cell-relative records (see make_recq)
      const int4 pi = pos16[i];
      const double qinv = Rp.qinv;
      wbits = (uint32_t)pi.w;
      ti = (int32_t)(wbits >> 30);
      for (int32_t k0 = lane_p; k0 < n; k0 += U * TPP) {
        int4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = pos16[e[u] & kIdxMask];
        uint32_t en[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t k = k0 + (U + u) * TPP;
          en[u] = k < n ? list_entry<NTL>(row + (size_t)k * kSlice) : self;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // (off_i - off_j) + d * side, d = c_i - c_j - s nc from the entry:
          // the integer difference is exact, the rest FP64
          const double4 dd = s_doff[e[u] >> kIdxBits];
          const double ex = __builtin_fma((double)(pi.x - q[u].x), qinv, dd.x),
                       ey = __builtin_fma((double)(pi.y - q[u].y), qinv, dd.y),
                       ez = __builtin_fma((double)(pi.z - q[u].z), qinv, dd.z);
          const int32_t ab = ti * 4 + (int32_t)((uint32_t)q[u].w >> 30);
          const double r2d = ex * ex + ey * ey + ez * ez;
          // slots past the row hold the particle itself (r^2 = 0): one
          // non-short-circuit condition, so the species word is read with
          // the rest of the record
          const PairRec& pr = s_pr[ab];
          if ((r2d > 0.0) & (r2d < pr.rc2)) {
            const float r2 = (float)r2d;
            const float ddx = (float)ex, ddy = (float)ey, ddz = (float)ez;
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float r2inv = rinv * rinv;
            const float sr2 = pr.sig2 * r2inv;
            const float sr6 = sr2 * sr2 * sr2;
            const float sr12 = sr6 * sr6;
            const float fr = (pr.f12 * sr12 + pr.f6 * sr6) * r2inv + pr.fs * rinv;
            fx += fr * ddx;
            fy += fr * ddy;
            fz += fr * ddz;
            if constexpr (EN) {
              pe_i += pr.c12 * sr12 + pr.c6 * sr6 - pr.vc - (r2 * rinv - pr.rc) * pr.fs;
              w_i += fr * r2;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = en[u];
      }
    } else {
      const double4 p = pos[i];
      ti = (int32_t)p.w;
      for (int32_t k0 = lane_p; k0 < n; k0 += U * TPP) {
        double4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = pos[e[u] & kIdxMask];
        uint32_t en[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t k = k0 + (U + u) * TPP;
          en[u] = k < n ? list_entry<NTL>(row + (size_t)k * kSlice) : self;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          double dx = p.x - q[u].x, dy = p.y - q[u].y, dz = p.z - q[u].z;
          // x_i - (x_j + s L); wave-uniform test: only waves with a periodic
          // partner pay for the shift (s = 0 leaves d unchanged)
          if (__ballot(e[u] >> kIdxBits)) {
            dx -= (double)decode_shift(e[u], 26) * L;
            dy -= (double)decode_shift(e[u], 28) * L;
            dz -= (double)decode_shift(e[u], 30) * L;
          }
          const int32_t ab = ti * 4 + (int32_t)q[u].w;
          const double r2 = dx * dx + dy * dy + dz * dz;
          if ((r2 > 0.0) & (r2 < P.rc2[ab])) {  // slots past the row: self, r^2 = 0
            const double rinv = rsqrt_nr(r2);
            const double r2inv = rinv * rinv;
            const double sr2 = P.sig2[ab] * r2inv;
            const double sr6 = sr2 * sr2 * sr2;
            const double sr12 = sr6 * sr6;
            const double fr = (P.f12[ab] * sr12 + P.f6[ab] * sr6) * r2inv + P.fs[ab] * rinv;
            fx += fr * dx;
            fy += fr * dy;
            fz += fr * dz;
            if constexpr (EN) {
              pe_i += P.c12[ab] * sr12 + P.c6[ab] * sr6 - P.vc[ab] -
                      (r2 * rinv - P.rc[ab]) * P.fs[ab];
              w_i += fr * r2;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = en[u];
      }
    }
  }
  if constexpr (TPP > 1) {
#pragma unroll
    for (int d = 1; d < TPP; d <<= 1) {
      fx += __shfl_xor(fx, d, 64);
      fy += __shfl_xor(fy, d, 64);
      fz += __shfl_xor(fz, d, 64);
      pe_i += __shfl_xor(pe_i, d, 64);
      w_i += __shfl_xor(w_i, d, 64);
    }
  }
  double d2 = 0.0;
  if (active && lane_p == 0) {
    if (!isfinite((double)(fx + fy + fz))) atomicOr(&st->err, kErrNonFinite);
    if constexpr (MODE != 2) {
      T* frc = (T*)frc_;
      frc[i] = fx;
      frc[stride + i] = fy;
      frc[2 * (size_t)stride + i] = fz;
    }
    pe = 0.5 * (double)pe_i;
    w = 0.5 * (double)w_i;
    const double m = s_mass[ti];
    double v0 = vel[i], v1 = vel[stride + i], v2 = vel[2 * (size_t)stride + i];
    if (MODE >= 1) {
      const double hm = 0.5 * dt / m;
      v0 += hm * (double)fx;
      v1 += hm * (double)fy;
      v2 += hm * (double)fz;
    }
    ke = 0.5 * m * (v0 * v0 + v1 * v1 + v2 * v2);
    if constexpr (MODE == 2) {
      // the next step's first half kick and drift
      double4 p = pos[i];
      const double hk = 0.5 * dt * s_im[(int32_t)p.w];
      v0 += hk * (double)fx;
      v1 += hk * (double)fy;
      v2 += hk * (double)fz;
      p.x += dt * v0;
      p.y += dt * v1;
      p.z += dt * v2;
      fo.pos_out[i] = p;
      if constexpr (MIXED) fo.pos16_out[i] = make_recq(p.x, p.y, p.z, wbits, Rp.cside, Rp.qs);
      const double e0 = p.x - fo.xref[i], e1 = p.y - fo.xref[stride + i],
                   e2 = p.z - fo.xref[2 * (size_t)stride + i];
      d2 = e0 * e0 + e1 * e1 + e2 * e2;
    }
    if (MODE >= 1) {
      vel[i] = v0;
      vel[stride + i] = v1;
      vel[2 * (size_t)stride + i] = v2;
    }
  }
  if constexpr (MODE == 2)
    block_sum3_max(pe, w, ke, d2);
  else
    block_sum3(pe, w, ke);
  if (threadIdx.x == 0) {
    double* o = part + 4 * (size_t)lb;
    o[0] = pe;
    o[1] = w;
    o[2] = ke;
    if (MODE == 2) o[3] = d2;
  }
}

template <bool MIXED, int MODE, bool EN, bool NTL>
void launch_t(hipStream_t s, int32_t tpp, int32_t unroll, int32_t ntiles, const Tile* tiles,
              const RepDesc* reps, const PairTab* tab, const double4* pos, const int4* pos16,
              double* vel, void* frc, const uint32_t* nbr, const int32_t* ncount, int32_t stride,
              int32_t cap, double dt, double* part, DevState* st, const FuseOut& fo) {
#define KF(TPP, U)                                                                       \
  k_force<MIXED, MODE, TPP, U, EN, NTL><<<ntiles * TPP, kTile, 0, s>>>(tiles, reps, tab, pos, pos16, \
                                                              vel, frc, nbr, ncount, stride, \
                                                              cap, dt, part, st, fo)
  const int key = tpp * 16 + unroll;
  switch (key) {
    case 1 * 16 + 1: KF(1, 1); break;
    case 1 * 16 + 2: KF(1, 2); break;
    case 1 * 16 + 8: KF(1, 8); break;
    case 2 * 16 + 1: KF(2, 1); break;
    case 2 * 16 + 2: KF(2, 2); break;
    case 2 * 16 + 4: KF(2, 4); break;
    case 4 * 16 + 1: KF(4, 1); break;
    case 4 * 16 + 2: KF(4, 2); break;
    case 8 * 16 + 1: KF(8, 1); break;
    default: KF(1, 4); break;
  }
#undef KF
}

}  // namespace

// Partials: one FP64 triple (pe, w, ke) per logical block; with tpp lanes
// per particle, tile t owns logical blocks [t*tpp, (t+1)*tpp).
void launch_force(hipStream_t s, int32_t mixed, int32_t mode, int32_t energy,
                  int32_t stream_list, int32_t tpp,
                  int32_t unroll, int32_t ntiles, const Tile* tiles, const RepDesc* reps,
                  const PairTab* tab, const double4* pos, const int4* pos16, double* vel,
                  void* frc, const uint32_t* nbr, const int32_t* ncount, int32_t stride,
                  int32_t cap, double dt, double* part, DevState* st, const FuseOut& fo) {
#define LT1(M, MO, EN, NTL)                                                                  \
  launch_t<M, MO, EN, NTL>(s, tpp, unroll, ntiles, tiles, reps, tab, pos, pos16, vel, frc, nbr, \
                           ncount, stride, cap, dt, part, st, fo)
#define LT(M, MO, EN) \
  if (stream_list) LT1(M, MO, EN, true); else LT1(M, MO, EN, false)
  // mode 0 (a plain force evaluation) always forms the energies
  if (mixed) {
    if (mode == 0) { LT(true, 0, true); }
    else if (mode == 2) { if (energy) { LT(true, 2, true); } else { LT(true, 2, false); } }
    else if (energy) { LT(true, 1, true); }
    else { LT(true, 1, false); }
  } else {
    if (mode == 0) { LT(false, 0, true); }
    else if (mode == 2) { if (energy) { LT(false, 2, true); } else { LT(false, 2, false); } }
    else if (energy) { LT(false, 1, true); }
    else { LT(false, 1, false); }
  }
#undef LT
#undef LT1
}

}  // namespace mdk
