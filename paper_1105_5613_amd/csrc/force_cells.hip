// force_cells.hip -- the paper's list-free linked-cell force evaluation
// ("Grid-search method", Fig. 1): no neighbour list; every force launch
// finds the interacting pairs from the cell grid itself.
//
// One block per row tile (stage.h gives the tile's 27 pieces: global
// particle ranges and periodic shifts).  A lane holds one home particle.  The
// lanes of a wave share one x-row of cells, so for every neighbour row they
// walk the union of their three-cell candidate ranges together: each step
// reads one candidate that all lanes need, through the scalar cache (a
// wave-uniform address), and tests the FP64 cutoff r^2 < rc_ab^2.
// Candidates outside a lane's own three cells are farther than rc (cells are
// at least rc + skin wide and nothing moved more than skin / 2 since binning)
// and fail the test.  Hits (particle index and piece) go to a small per-lane
// buffer in LDS; when any lane's buffer fills, and after the last row, the
// wave evaluates the buffered pairs densely (shifted-force Eq. (3) on
// Eq. (1)/(2), the arithmetic of force.hip).  Cells are rebuilt by the same
// skin rule as the lists of the other paths.
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
  T sig2[16], c12[16], c6[16], f12[16], f6[16], vc[16], fs[16], rc[16];
  double rc2[16];  // the cutoff test is FP64 in both precisions
};

constexpr int kCellHomes = 128;  // home particles per block (one lane each)
constexpr int kHitBuf = 16;      // buffered hits per lane before a flush
constexpr int kCand = 8;         // candidates tested per step of the search
constexpr double kFar = 1.0e300; // x of the idle lanes: every r^2 is +inf

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

template <typename T>
struct Acc {
  T fx = 0, fy = 0, fz = 0, pe = 0, w = 0;
};

// Pair (i, slot v) with i's position p and species ti; the displacement is
// recomputed from the staged slot.
template <typename T>
__device__ inline void pair_force(const PairLds<T>& P, const double4& p, int32_t ti, double qx,
                                  double qy, double qz, int32_t tj, Acc<T>& a) {
  const int32_t ab = ti * 4 + tj;
  // displacement and r^2 in FP64 (the mixed form rounds them to FP32 after)
  const double ex = p.x - qx, ey = p.y - qy, ez = p.z - qz;
  const T dx = (T)ex, dy = (T)ey, dz = (T)ez;
  const T r2 = (T)(ex * ex + ey * ey + ez * ez);
  T rinv;
  if constexpr (std::is_same<T, float>::value)
    rinv = __builtin_amdgcn_rsqf(r2);
  else
    rinv = rsqrt_nr(r2);
  const T r2inv = rinv * rinv;
  const T sr2 = P.sig2[ab] * r2inv;
  const T sr6 = sr2 * sr2 * sr2;
  const T sr12 = sr6 * sr6;
  const T fr = (P.f12[ab] * sr12 + P.f6[ab] * sr6) * r2inv + P.fs[ab] * rinv;
  a.fx += fr * dx;
  a.fy += fr * dy;
  a.fz += fr * dz;
  a.pe += P.c12[ab] * sr12 + P.c6[ab] * sr6 - P.vc[ab] - (r2 * rinv - P.rc[ab]) * P.fs[ab];
  a.w += fr * r2;
}

// Register budget for 6 waves per SIMD (80 VGPRs; 88-117 otherwise, 4-5
// waves): the candidate loop is latency-bound, 1.36 -> 1.31 ms at 1M FP64.
// NT = 2: the cutoff of (home species a, candidate species value s_b) is
// rc2[0][a] + (rc2[1][a] - rc2[0][a]) s_b as one FMA (exact: the launch checks
// the table, see fma_pair_form; the table is symmetric); NT = 4: a select.
template <bool MIXED, int MODE, int NT>
__global__ __launch_bounds__(kCellHomes) __attribute__((amdgpu_waves_per_eu(6))) void k_force_cells(
    const RowTile* __restrict__ rtiles, const RepDesc* __restrict__ reps,
    const PairTab* __restrict__ tab, const int32_t* __restrict__ cell_start,
    const double4* __restrict__ pos, double* __restrict__ vel, void* __restrict__ frc_,
    int32_t stride, double dt, double* __restrict__ part, DevState* st) {
  using T = typename std::conditional<MIXED, float, double>::type;
  __shared__ StageLayout S;
  __shared__ PairLds<T> P;
  __shared__ double s_mass[4];
  // hit = offset of the particle in its piece | piece << 27 (offsets are
  // below the piece's length, so any particle count fits)
  __shared__ uint32_t s_hit[kHitBuf][kCellHomes];
  if (halted(st)) {  // an overflowed list build halts the queued steps (kHalt)
    if (blockIdx.x == 0 && threadIdx.x == 0) st->any_rebuild = 0;
    return;
  }
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  const RowTile Tl = rtiles[tb];
  const RepDesc R = reps[Tl.rep];
  if (threadIdx.x < 16) {
    const int k = threadIdx.x;
    P.rc2[k] = tab->rc2[k];
    P.sig2[k] = (T)tab->sig2[k];
    P.c12[k] = (T)tab->c12[k];
    P.c6[k] = (T)tab->c6[k];
    P.f12[k] = (T)tab->f12[k];
    P.f6[k] = (T)tab->f6[k];
    P.vc[k] = (T)tab->vc[k];
    P.fs[k] = (T)tab->fs[k];
    P.rc[k] = (T)tab->rc[k];
  }
  if (threadIdx.x < 4) s_mass[threadIdx.x] = tab->mass[threadIdx.x];
  build_layout(S, Tl, R, cell_start);

  double pe = 0.0, w = 0.0, ke = 0.0;
  const int32_t nh = S.home1 - S.home0;
  for (int32_t g0 = 0; g0 < nh; g0 += kCellHomes) {
    const int32_t li = g0 + (int32_t)threadIdx.x;
    const bool mine = li < nh;
    const int32_t i = S.home0 + (mine ? li : 0);
    const int32_t hs = S.home_lds + (mine ? li : 0);  // the home particle's layout slot
    const double4 p = pos[i];
    const int32_t ti = (int32_t)p.w;
    // logical cell of the home particle in the tile (row 4 holds the homes)
    int32_t cl = 1;
    while (cl < Tl.nx && S.loff[4][cl + 1] <= hs) ++cl;
    // the wave's range of home cells
    int32_t clo = mine ? cl : 0x7fffffff, chi = mine ? cl : -1;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      clo = min(clo, __shfl_xor(clo, d, 64));
      chi = max(chi, __shfl_xor(chi, d, 64));
    }
    Acc<T> a;
    int32_t cnt = 0;
    const double rc2_0 = P.rc2[ti * 4], rc2_1 = P.rc2[ti * 4 + 1], rc2_2 = P.rc2[ti * 4 + 2],
                 rc2_3 = P.rc2[ti * 4 + 3];
    const double drc2 = P.rc2[4 + ti] - P.rc2[ti];
    const double px = mine ? p.x : kFar;
    // candidate c (index j, piece pc) against the lane's home particle;
    // only the home cell's own piece can hold the particle itself
    auto test = [&](auto self_tag, const double4& c, int32_t j, int32_t pc, double hx, double hy,
                    double hz) {
      constexpr bool SELF = decltype(self_tag)::value;
      const double ex = hx - c.x, ey = hy - c.y, ez = hz - c.z;
      const double r2 = ex * ex + ey * ey + ez * ez;
      double rc2;
      if constexpr (NT == 2) {
        rc2 = __builtin_fma(drc2, c.w, rc2_0);
      } else {
        const int32_t tj = (int32_t)c.w;
        rc2 = tj == 0 ? rc2_0 : (tj == 1 ? rc2_1 : (tj == 2 ? rc2_2 : rc2_3));
      }
      const bool hit = SELF ? (j != i && r2 < rc2) : r2 < rc2;
      if (hit) s_hit[cnt++][threadIdx.x] = (uint32_t)(j - S.pc_g[pc]) | ((uint32_t)pc << 27);
    };
    auto flush = [&]() {
      int32_t mx = cnt;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
      for (int32_t k = 0; k < mx; ++k) {
        if (k < cnt) {
          const uint32_t e = s_hit[k][threadIdx.x];
          const int32_t pc = (int32_t)(e >> 27);
          const double4 q = pos[S.pc_g[pc] + (int32_t)(e & 0x07ffffffu)];
          pair_force<T>(P, p, ti, q.x + S.pc_sx[pc], q.y + S.pc_sy[pc], q.z + S.pc_sz[pc],
                        (int32_t)q.w, a);
        }
      }
      cnt = 0;
    };
    if (chi >= 0) {  // the wave holds home particles
      for (int q = 0; q < 9; ++q) {
        const int32_t u0 = S.loff[q][clo - 1], u1 = S.loff[q][chi + 2];
        // the union range crosses at most the row's three pieces
        for (int pc = 3 * q; pc < 3 * q + 3; ++pc) {
          const int32_t a0 = max(u0, S.pc_l[pc]), a1 = min(u1, S.pc_l[pc + 1]);
          if (a0 >= a1) continue;
          // home position minus the piece's shift: d = x_i - (x_j + s L)
          const double hx = px - S.pc_sx[pc], hy = p.y - S.pc_sy[pc], hz = p.z - S.pc_sz[pc];
          const int32_t g = __builtin_amdgcn_readfirstlane(S.pc_g[pc] + (a0 - S.pc_l[pc]));
          const int32_t m = a1 - a0;
          auto scan = [&](auto self_tag) {
            // kCand candidates per step: their scalar loads are issued together
            int32_t t = 0;
            for (; t + kCand <= m; t += kCand) {
              if (__ballot(cnt > kHitBuf - kCand)) flush();
              double4 cd[kCand];
#pragma unroll
              for (int u = 0; u < kCand; ++u) cd[u] = pos[g + t + u];  // wave-uniform
#pragma unroll
              for (int u = 0; u < kCand; ++u) test(self_tag, cd[u], g + t + u, pc, hx, hy, hz);
            }
            for (; t < m; ++t) {
              if (__ballot(cnt == kHitBuf)) flush();
              test(self_tag, pos[g + t], g + t, pc, hx, hy, hz);
            }
          };
          if (pc == 13)  // row 4 (the home row), main piece
            scan(std::true_type{});
          else
            scan(std::false_type{});
        }
      }
      flush();
    }
    pe += 0.5 * (double)a.pe;
    w += 0.5 * (double)a.w;
    if (mine) {
      if (!isfinite((double)(a.fx + a.fy + a.fz))) atomicOr(&st->err, kErrNonFinite);
      T* frc = (T*)frc_;
      frc[i] = a.fx;
      frc[stride + i] = a.fy;
      frc[2 * (size_t)stride + i] = a.fz;
      const double ms = s_mass[ti];
      double v0 = vel[i], v1 = vel[stride + i], v2 = vel[2 * (size_t)stride + i];
      if (MODE == 1) {
        const double hm = 0.5 * dt / ms;
        v0 += hm * (double)a.fx;
        v1 += hm * (double)a.fy;
        v2 += hm * (double)a.fz;
        vel[i] = v0;
        vel[stride + i] = v1;
        vel[2 * (size_t)stride + i] = v2;
      }
      ke += 0.5 * ms * (v0 * v0 + v1 * v1 + v2 * v2);
    }
  }
  block_sum3<kCellHomes>(pe, w, ke);
  if (threadIdx.x == 0) {
    double* o = part + 4 * (size_t)tb;
    o[0] = pe;
    o[1] = w;
    o[2] = ke;
  }
}

// After a rebuild: the sorted order becomes the live state and the
// reference positions of the skin rule are reset (the list-building kernels
// do this on the other paths).
__global__ __launch_bounds__(kTile) void k_commit_order(
    const Tile* __restrict__ tiles, const int32_t* __restrict__ rebuild, int32_t stride,
    const double4* __restrict__ pos_tmp, const double* __restrict__ vel_tmp,
    const int32_t* __restrict__ id_tmp, double4* __restrict__ pos, double* __restrict__ vel,
    int32_t* __restrict__ id, double* __restrict__ xref, const DevState* __restrict__ st) {
  if (!st->any_rebuild) return;
  const Tile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
  if (!rebuild[t.rep]) return;
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  const double4 p = pos_tmp[i];
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

int32_t cells_homes_per_block() { return kCellHomes; }

void launch_force_cells(hipStream_t s, int32_t mixed, int32_t mode, int32_t rc2_form,
                        int32_t nrt, const RowTile* rtiles, const RepDesc* reps,
                        const PairTab* tab, const int32_t* cell_start, const double4* pos,
                        double* vel, void* frc, int32_t stride, double dt, double* part,
                        DevState* st) {
#define KC(M, MO, NT)                                                                 \
  k_force_cells<M, MO, NT><<<nrt, kCellHomes, 0, s>>>(rtiles, reps, tab, cell_start, pos, \
                                                      vel, frc, stride, dt, part, st)
#define KN(M, MO) \
  if (rc2_form == 2) KC(M, MO, 2); else KC(M, MO, 4)
  if (mixed) {
    if (mode) { KN(true, 1); } else { KN(true, 0); }
  } else {
    if (mode) { KN(false, 1); } else { KN(false, 0); }
  }
#undef KN
#undef KC
}

void launch_commit_order(hipStream_t s, int32_t ntiles, const Tile* tiles,
                         const int32_t* rebuild, int32_t stride, const double4* pos_tmp,
                         const double* vel_tmp, const int32_t* id_tmp, double4* pos,
                         double* vel, int32_t* id, double* xref, const DevState* st) {
  k_commit_order<<<ntiles, kTile, 0, s>>>(tiles, rebuild, stride, pos_tmp, vel_tmp, id_tmp, pos,
                                          vel, id, xref, st);
}

}  // namespace mdk
