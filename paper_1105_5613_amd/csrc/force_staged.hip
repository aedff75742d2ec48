// force_staged.hip -- the pair-force hot spot on the staged path: one block
// per row tile (stage.h) copies the tile's whole 27-piece neighbourhood
// (positions with their periodic shift applied, FP64) into LDS with
// coalesced loads, then every home particle walks its 16-bit slot list
// against LDS instead of gathering its partners from global memory.  TPP
// lanes per particle take interleaved list slots and combine their sums with
// cross-lane shuffles; the list walk is software-pipelined by U slots.
//
// Pair arithmetic as in force.hip: shifted-force Eq. (3) on Eq. (1)/(2);
// FP64 with an FP32-seeded two-step Newton-Raphson 1/r, or FP32 pair math
// from the FP64 displacement (mixed); per-particle energy and virial halves
// reduced per block in FP64.  Also holds the decode of staged entries back to
// sorted particle indices (neighbour-list parity hook).
#include "stage.h"

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

template <int BT>
__device__ inline void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][BT / 64];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
    c += __shfl_xor(c, d, 64);
  }
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
    for (int k = 1; k < BT / 64; ++k) {
      a += red[0][k];
      b += red[1][k];
      c += red[2][k];
    }
  }
}

// home particles handled per group: kStageHomes x TPP threads per block
constexpr int kStageHomes = 128;

template <bool MIXED, int MODE, int TPP, int U>
__global__ __launch_bounds__(kStageHomes* TPP) void k_force_staged(
    const RowTile* __restrict__ rtiles, const RepDesc* __restrict__ reps,
    const PairTab* __restrict__ tab, const int32_t* __restrict__ cell_start,
    const double4* __restrict__ pos, double* __restrict__ vel, void* __restrict__ frc_,
    const uint16_t* __restrict__ nbr, const int32_t* __restrict__ ncount, int32_t stride,
    int32_t cap, int32_t lcap, double dt, double* __restrict__ part, DevState* st) {
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr int BT = kStageHomes * TPP;
  __shared__ StageLayout S;
  __shared__ PairLds<T> P;
  __shared__ double s_mass[4], s_rc2[16];
  extern __shared__ double dyn[];
  if (halted(st)) {  // an overflowed list build halts the queued steps (kHalt)
    if (blockIdx.x == 0 && threadIdx.x == 0) st->any_rebuild = 0;
    return;
  }
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  const RowTile Tl = rtiles[tb];
  const RepDesc R = reps[Tl.rep];
  if (threadIdx.x < 16) {
    const int k = threadIdx.x;
    P.rc2[k] = (T)tab->rc2[k];
    P.sig2[k] = (T)tab->sig2[k];
    P.c12[k] = (T)tab->c12[k];
    P.c6[k] = (T)tab->c6[k];
    P.f12[k] = (T)tab->f12[k];
    P.f6[k] = (T)tab->f6[k];
    P.vc[k] = (T)tab->vc[k];
    P.fs[k] = (T)tab->fs[k];
    P.rc[k] = (T)tab->rc[k];
    s_rc2[k] = tab->rc2[k];
  }
  if (threadIdx.x < 4) s_mass[threadIdx.x] = tab->mass[threadIdx.x];
  build_layout(S, Tl, R, cell_start);
  double2* xy = (double2*)dyn;
  double* zz = (double*)(xy + lcap);
  stage_all(S, pos, lcap, xy, zz);

  double pe = 0.0, w = 0.0, ke = 0.0;
  const int32_t nh = S.home1 - S.home0;
  const int32_t lane_p = (int32_t)threadIdx.x % TPP;
  for (int32_t g0 = 0; g0 < nh; g0 += kStageHomes) {
    const int32_t li = g0 + (int32_t)threadIdx.x / TPP;
    const bool mine = li < nh;
    const int32_t i = S.home0 + (mine ? li : 0);
    const double4 p = pos[i];
    const int32_t ti = (int32_t)p.w;
    int32_t n = mine ? ncount[i] : 0;
    n = n < cap ? n : cap;
    const uint16_t* row = nbr + list_base(i, cap);
    T fx = 0, fy = 0, fz = 0, pe_i = 0, w_i = 0;
    // list slots of the next chunk are loaded ahead; slots past n repeat
    // slot 0 and are masked out
    uint32_t e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t k = lane_p + u * TPP;
      e[u] = k < n ? (uint32_t)row[(size_t)k * kSlice] : 0u;
    }
    for (int32_t k0 = lane_p; k0 < n; k0 += U * TPP) {
      uint32_t en[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + (U + u) * TPP;
        en[u] = k < n ? (uint32_t)row[(size_t)k * kSlice] : 0u;
      }
      double qx[U], qy[U], qz[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t v = (int32_t)(e[u] & 0x3fffu);
        if (v < lcap) {
          const double2 a = xy[v];
          qx[u] = a.x;
          qy[u] = a.y;
          qz[u] = zz[v];
        } else {
          const double4 q = fetch_slot(S, pos, v);
          qx[u] = q.x;
          qy[u] = q.y;
          qz[u] = q.z;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t ab = ti * 4 + (int32_t)(e[u] >> 14);
        // displacement, r^2 and the cut-off test in FP64 (the mixed form
        // rounds them to FP32 for the pair arithmetic)
        const double ex = p.x - qx[u], ey = p.y - qy[u], ez = p.z - qz[u];
        const double r2d = ex * ex + ey * ey + ez * ez;
        if (k0 + u * TPP < n && r2d < s_rc2[ab]) {
          const T dx = (T)ex, dy = (T)ey, dz = (T)ez;
          const T r2 = (T)r2d;
          T rinv;
          if constexpr (MIXED)
            rinv = __builtin_amdgcn_rsqf(r2);
          else
            rinv = rsqrt_nr(r2);
          const T r2inv = rinv * rinv;
          const T sr2 = P.sig2[ab] * r2inv;
          const T sr6 = sr2 * sr2 * sr2;
          const T sr12 = sr6 * sr6;
          const T fr = (P.f12[ab] * sr12 + P.f6[ab] * sr6) * r2inv + P.fs[ab] * rinv;
          fx += fr * dx;
          fy += fr * dy;
          fz += fr * dz;
          pe_i += P.c12[ab] * sr12 + P.c6[ab] * sr6 - P.vc[ab] -
                  (r2 * rinv - P.rc[ab]) * P.fs[ab];
          w_i += fr * r2;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) e[u] = en[u];
    }
    // combine the TPP partial sums (fixed order: deterministic)
#pragma unroll
    for (int d = 1; d < TPP; d <<= 1) {
      fx += __shfl_xor(fx, d, 64);
      fy += __shfl_xor(fy, d, 64);
      fz += __shfl_xor(fz, d, 64);
    }
    pe += 0.5 * (double)pe_i;
    w += 0.5 * (double)w_i;
    if (mine && lane_p == 0) {
      if (!isfinite((double)(fx + fy + fz))) atomicOr(&st->err, kErrNonFinite);
      T* frc = (T*)frc_;
      frc[i] = fx;
      frc[stride + i] = fy;
      frc[2 * (size_t)stride + i] = fz;
      const double m = s_mass[ti];
      double v0 = vel[i], v1 = vel[stride + i], v2 = vel[2 * (size_t)stride + i];
      if (MODE == 1) {
        const double hm = 0.5 * dt / m;
        v0 += hm * (double)fx;
        v1 += hm * (double)fy;
        v2 += hm * (double)fz;
        vel[i] = v0;
        vel[stride + i] = v1;
        vel[2 * (size_t)stride + i] = v2;
      }
      ke += 0.5 * m * (v0 * v0 + v1 * v1 + v2 * v2);
    }
  }
  block_sum3<BT>(pe, w, ke);
  if (threadIdx.x == 0) {
    double* o = part + 4 * (size_t)tb;
    o[0] = pe;
    o[1] = w;
    o[2] = ke;
  }
}

// Staged entries -> sorted particle indices (parity hook only).
__global__ __launch_bounds__(256) void k_decode_staged(
    const RowTile* __restrict__ rtiles, const RepDesc* __restrict__ reps,
    const int32_t* __restrict__ cell_start, int32_t cap, const uint16_t* __restrict__ nbr,
    const int32_t* __restrict__ ncount, uint32_t* __restrict__ out) {
  __shared__ StageLayout S;
  const RowTile T = rtiles[blockIdx.x];
  const RepDesc R = reps[T.rep];
  build_layout(S, T, R, cell_start);
  const int32_t nh = S.home1 - S.home0;
  for (int32_t li = threadIdx.x; li < nh; li += blockDim.x) {
    const int32_t i = S.home0 + li;
    int32_t n = ncount[i];
    n = n < cap ? n : cap;
    const size_t b = list_base(i, cap);
    for (int32_t k = 0; k < n; ++k) {
      int32_t v = nbr[b + (size_t)k * kSlice] & 0x3fff;
      v = v < S.total ? v : S.total - 1;  // only after a reported overflow
      const int p = piece_of(S, v);
      out[b + (size_t)k * kSlice] = (uint32_t)(S.pc_g[p] + (v - S.pc_l[p]));
    }
  }
}

}  // namespace

size_t force_staged_lds_bytes(int32_t lcap) { return (size_t)lcap * 24; }

int32_t staged_homes_per_group() { return kStageHomes; }

void launch_force_staged(hipStream_t s, int32_t mixed, int32_t mode, int32_t tpp, int32_t unroll,
                         int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                         const PairTab* tab, const int32_t* cell_start, const double4* pos,
                         double* vel, void* frc, const uint16_t* nbr, const int32_t* ncount,
                         int32_t stride, int32_t cap, int32_t lcap, double dt, double* part,
                         DevState* st) {
  const size_t lds = force_staged_lds_bytes(lcap);
#define KS(M, MO, TP, UU)                                                                    \
  k_force_staged<M, MO, TP, UU><<<nrt, kStageHomes * TP, lds, s>>>(                          \
      rtiles, reps, tab, cell_start, pos, vel, frc, nbr, ncount, stride, cap, lcap, dt, part, \
      st)
#define BYTU(M, MO)                                   \
  do {                                                \
    if (tpp == 1) {                                   \
      if (unroll == 8) KS(M, MO, 1, 8);               \
      else KS(M, MO, 1, 4);                           \
    } else if (tpp == 4) {                            \
      KS(M, MO, 4, 2);                                \
    } else {                                          \
      if (unroll == 2) KS(M, MO, 2, 2);               \
      else if (unroll == 8) KS(M, MO, 2, 8);          \
      else KS(M, MO, 2, 4);                           \
    }                                                 \
  } while (0)
  if (mixed) {
    if (mode) BYTU(true, 1); else BYTU(true, 0);
  } else {
    if (mode) BYTU(false, 1); else BYTU(false, 0);
  }
#undef BYTU
#undef KS
}

void launch_decode_staged(hipStream_t s, int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                          const int32_t* cell_start, int32_t cap, const uint16_t* nbr,
                          const int32_t* ncount, uint32_t* out) {
  k_decode_staged<<<nrt, 256, 0, s>>>(rtiles, reps, cell_start, cap, nbr, ncount, out);
}

}  // namespace mdk
