// integrate.hip -- velocity-Verlet kick/drift with the skin check, and the
// per-replica reductions, observables and isokinetic thermostat.
//
// Velocity Verlet ("Parallel force calculation"): v += dt/2 F/m; x += dt v;
// forces; v += dt/2 F/m.  The second half kick runs inside the force kernel;
// this file holds the first half kick and the drift, fused with the
// displacement test |x - x_ref|^2 > (skin/2)^2 that schedules list rebuilds
// and with the pending thermostat factor of the previous step.  (In NVE
// steps of a one-replica context the force kernel's mode 2 applies the next
// step's first half kick and drift itself, with the same arithmetic.)
//
// Canonical runs (fixed T, "BBMD scaling results"; the glass-section T ramp)
// rescale v by lambda = sqrt(T_target / T_inst) after the second half kick,
// with T_inst = 2 KE / (3 n - 3).  lambda is computed by the reduction and
// applied at the start of the next kick (or by apply_lambda at the end of a
// call), which is the same arithmetic as rescaling right away.
#include "md_internal.h"

namespace mdk {
namespace {

template <typename FT, bool THERMO>
__global__ __launch_bounds__(kTile) void k_kick_drift(
    const Tile* __restrict__ tiles, const RepDesc* __restrict__ reps,
    const PairTab* __restrict__ tab, double4* __restrict__ pos, int4* __restrict__ pos16,
    double* __restrict__ vel, const FT* __restrict__ frc, const double* __restrict__ xref,
    int32_t stride, double dt,
    const double* __restrict__ lam, int32_t* __restrict__ rebuild,
    double* __restrict__ dmax, DevState* st, int32_t* __restrict__ counts, int32_t nzero) {
  __shared__ double s_im[4];
  __shared__ double s_red[kTile / 64];
  if (halted(st)) return;  // an overflowed list build halts the queued steps
  if (threadIdx.x < 4) s_im[threadIdx.x] = tab->inv_mass[threadIdx.x];
  __syncthreads();
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  // one replica: the cell histogram is only read inside a rebuild, so it is
  // cleared here every step instead of by a separate gated launch
  const int32_t gz = blockIdx.x * kTile + threadIdx.x;
  if (gz < nzero) counts[gz] = 0;
  const Tile t = tiles[tb];
  const int32_t i = t.start + threadIdx.x;
  double d2 = 0.0;
  if (i < t.end) {
    double4 p = pos[i];
    const double hm = 0.5 * dt * s_im[(int32_t)p.w];
    double v0 = vel[i], v1 = vel[stride + i], v2 = vel[2 * (size_t)stride + i];
    if (THERMO) {
      const double l = lam[t.rep];
      v0 *= l;
      v1 *= l;
      v2 *= l;
    }
    v0 += hm * (double)frc[i];
    v1 += hm * (double)frc[stride + i];
    v2 += hm * (double)frc[2 * (size_t)stride + i];
    p.x += dt * v0;
    p.y += dt * v1;
    p.z += dt * v2;
    pos[i] = p;
    if (pos16) {
      const RepDesc& R = reps[t.rep];
      pos16[i] = make_recq(p.x, p.y, p.z, (uint32_t)pos16[i].w, R.cside, R.qs);
    }
    vel[i] = v0;
    vel[stride + i] = v1;
    vel[2 * (size_t)stride + i] = v2;
    const double e0 = p.x - xref[i], e1 = p.y - xref[stride + i],
                 e2 = p.z - xref[2 * (size_t)stride + i];
    d2 = e0 * e0 + e1 * e1 + e2 * e2;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) d2 = fmax(d2, __shfl_xor(d2, d, 64));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = s_red[0];
    for (int k = 1; k < kTile / 64; ++k) m = fmax(m, s_red[k]);
    const RepDesc& R = reps[t.rep];
    if (m > R.half_skin2) {
      rebuild[t.rep] = 1;
      st->any_rebuild = 1;
    }
    dmax[tb] = m;  // the per-replica maximum is taken by the reduction
  }
}

__device__ inline void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

// One block per replica: compensated sums of the per-block partials in a
// fixed order (deterministic), then observables and the thermostat factor.
constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void k_reduce(const RepDesc* __restrict__ reps,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ dmax,
                                                        const double* __restrict__ part2,
                                                        int32_t step, int32_t energy,
                                                        DriftArgs drift, ThermoArgs ta,
                                                        int64_t* __restrict__ kcall,
                                                        double* __restrict__ lam,
                                                        int32_t* __restrict__ rebuild,
                                                        md_obs* __restrict__ obs, DevState* st) {
  __shared__ double red[5][kRedThreads / 64];
  if (halted(st)) return;  // the step was not taken (kHalt)
  const int32_t r = blockIdx.x;
  const RepDesc R = reps[r];
  // thread 0's per-replica inputs, fetched before the sums so that their
  // latency overlaps them (only this block reads or writes index r)
  md_obs o;
  int64_t kc = 0;
  int32_t rb = 0;
  double tt0 = 0.0, tt1 = 0.0, pend = 0.0;
  if (threadIdx.x == 0) {
    o = obs[r];
    if (step) {
      kc = kcall[r];
      rb = rebuild[r];
      if (ta.thermo) {
        tt0 = ta.T0[r];
        tt1 = ta.T1[r];
      }
      if (drift.src) pend = drift.pend[r];
    }
  }
  double s[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
  double m = 0.0;   // largest squared displacement of this step's drift
  double mn = 0.0;  // ... of the next step's drift (fused force launch)
  if (part2) {
    for (int32_t b = R.cb0 + threadIdx.x; b < R.cb1; b += kRedThreads) {
      for (int k = 0; k < 3; ++k) neumaier(s[k], c[k], part2[kPart2 * (size_t)b + k]);
      m = fmax(m, part2[kPart2 * (size_t)b + 3]);
      mn = fmax(mn, part2[kPart2 * (size_t)b + 4]);
    }
  } else {
#pragma unroll 4
    for (int32_t b = R.fb0 + threadIdx.x; b < R.fb1; b += kRedThreads) {
      const double4 q = *reinterpret_cast<const double4*>(part + 4 * (size_t)b);
      neumaier(s[0], c[0], q.x);
      neumaier(s[1], c[1], q.y);
      neumaier(s[2], c[2], q.z);
      if (drift.next) mn = fmax(mn, q.w);
    }
    if (step && drift.src == 0)
      for (int32_t b = R.tile0 + threadIdx.x; b < R.tile1; b += kRedThreads)
        m = fmax(m, dmax[b]);
  }
  // each wave's totals by a butterfly over its lanes, then the wave totals
  // in wave order by thread 0: a fixed order, one barrier
  double v[5] = {s[0] + c[0], s[1] + c[1], s[2] + c[2], m, mn};
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += __shfl_xor(v[k], d, 64);
    v[3] = fmax(v[3], __shfl_xor(v[3], d, 64));
    v[4] = fmax(v[4], __shfl_xor(v[4], d, 64));
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = red[k][0];
  for (int q = 1; q < kRedThreads / 64; ++q) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += red[k][q];
    v[3] = fmax(v[3], red[3][q]);
    v[4] = fmax(v[4], red[4][q]);
  }
  const double pe = v[0], w = v[1];
  double ke = v[2];
  if (energy) {
    o.pe = pe;
    o.virial = w;
  }
  o.T_target = 0.0;
  if (step) o.max_disp = sqrt(drift.src ? pend : v[3]);
  if (step) {
    const int64_t k = kc + 1;
    kcall[r] = k;
    if (ta.thermo) {
      const double t0 = tt0, t1 = tt1;
      double tt = t0;
      if (ta.ramp > 0) {
        double f = (double)k / (double)ta.ramp;
        f = f > 1.0 ? 1.0 : f;
        tt = t0 + (t1 - t0) * f;
      }
      const double ti = 2.0 * ke / R.dof;
      const double l = sqrt(tt / ti);
      lam[r] = l;
      ke = ke * l * l;
      o.T_target = tt;
    }
    o.step += 1;
    if (rb) o.n_rebuild += 1;
    if (drift.next) {
      // the next step's positions are drifted already: its rebuild decision
      const double mx = v[4];
      const int32_t nb = mx > R.half_skin2 ? 1 : 0;
      drift.pend[r] = mx;
      rebuild[r] = nb;
      st->any_rebuild = nb;
    } else {
      rebuild[r] = 0;
      if (r == 0) st->any_rebuild = 0;
    }
  }
  o.ke = ke;
  o.T = 2.0 * ke / R.dof;
  if (energy) {
    o.P = (2.0 * ke + w) / (3.0 * R.volume);
    o.E = ke + pe;
  }
  obs[r] = o;
  if (step && ta.log_every > 0) {
    const int64_t k = kc + 1;
    if (k % ta.log_every == 0) {
      const int64_t idx = k / ta.log_every - 1;
      if (idx >= 0 && idx < ta.nlog) ta.log[idx * gridDim.x + r] = o;
    }
  }
}

// First level of the two-level reduction: one block per chunk, fixed order.
constexpr int kChunkThreads = 256;
__global__ __launch_bounds__(kChunkThreads) void k_reduce_chunks(const RedChunk* __restrict__ ch,
                                                                 const double* __restrict__ part,
                                                                 const double* __restrict__ dmax,
                                                                 int32_t step, int32_t next,
                                                                 double* __restrict__ part2,
                                                                 const DevState* st) {
  __shared__ double red[5][kChunkThreads];
  if (halted(st)) return;
  const RedChunk C = ch[blockIdx.x];
  double s[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
  double mn = 0.0;
  for (int32_t b = C.b0 + threadIdx.x; b < C.b1; b += kChunkThreads) {
    for (int k = 0; k < 3; ++k) neumaier(s[k], c[k], part[4 * (size_t)b + k]);
    if (next) mn = fmax(mn, part[4 * (size_t)b + 3]);
  }
  double m = 0.0;
  if (step)
    for (int32_t t = C.t0 + threadIdx.x; t < C.t1; t += kChunkThreads) m = fmax(m, dmax[t]);
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k] + c[k];
  red[3][threadIdx.x] = m;
  red[4][threadIdx.x] = mn;
  __syncthreads();
  for (int h = kChunkThreads / 2; h >= 1; h >>= 1) {
    if (threadIdx.x < h) {
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + h]);
      red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) part2[kPart2 * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_after_build(int32_t nrep, int32_t* rebuild, md_obs* obs, DevState* st) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrep && rebuild[r]) {
    obs[r].n_rebuild += 1;
    obs[r].max_disp = 0.0;
    rebuild[r] = 0;
  }
  if (r == 0) st->any_rebuild = 0;
}

__global__ void k_begin_call(int32_t nrep, int64_t* kcall, double* lam) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrep) {
    kcall[r] = 0;
    lam[r] = 1.0;
  }
}

__global__ __launch_bounds__(kTile) void k_apply_lambda(const Tile* __restrict__ tiles,
                                                        int32_t stride, double* __restrict__ vel,
                                                        const double* __restrict__ lam,
                                                        const DevState* st) {
  if (halted(st)) return;  // the factor is applied when the host finishes the call
  const Tile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
  const int32_t i = t.start + threadIdx.x;
  if (i >= t.end) return;
  const double l = lam[t.rep];
  vel[i] *= l;
  vel[stride + i] *= l;
  vel[2 * (size_t)stride + i] *= l;
}

__global__ void k_reset_lambda(int32_t nrep, double* lam, const DevState* st) {
  if (halted(st)) return;
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrep) lam[r] = 1.0;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_kick_drift(hipStream_t s, int32_t mixed, int32_t thermo, int32_t ntiles,
                       const Tile* tiles, const RepDesc* reps, const PairTab* tab, double4* pos,
                       int4* pos16, double* vel, const void* frc, const double* xref,
                       int32_t stride, double dt, const double* lam, int32_t* rebuild,
                       double* dmax, DevState* st, int32_t* counts, int32_t nzero) {
#define KD(FT, TH)                                                                         \
  k_kick_drift<FT, TH><<<ntiles, kTile, 0, s>>>(tiles, reps, tab, pos, pos16, vel,         \
                                                (const FT*)frc, xref, stride, dt, lam,     \
                                                rebuild, dmax, st, counts, nzero)
  if (mixed) {
    if (thermo) KD(float, true); else KD(float, false);
  } else {
    if (thermo) KD(double, true); else KD(double, false);
  }
#undef KD
}

void launch_reduce(hipStream_t s, int32_t nrep, const RepDesc* reps, const double* part,
                   const double* dmax, const double* part2, int32_t step, int32_t energy,
                   DriftArgs drift, ThermoArgs ta, int64_t* kcall, double* lam, int32_t* rebuild,
                   md_obs* obs, DevState* st) {
  k_reduce<<<nrep, kRedThreads, 0, s>>>(reps, part, dmax, part2, step, energy, drift, ta, kcall,
                                        lam, rebuild, obs, st);
}

void launch_reduce_chunks(hipStream_t s, int32_t nchunks, const RedChunk* ch, const double* part,
                          const double* dmax, int32_t step, int32_t next, double* part2,
                          const DevState* st) {
  k_reduce_chunks<<<nchunks, kChunkThreads, 0, s>>>(ch, part, dmax, step, next, part2, st);
}

void launch_after_build(hipStream_t s, int32_t nrep, int32_t* rebuild, md_obs* obs,
                        DevState* st) {
  k_after_build<<<nblk(nrep, 256), 256, 0, s>>>(nrep, rebuild, obs, st);
}

void launch_begin_call(hipStream_t s, int32_t nrep, int64_t* kcall, double* lam) {
  k_begin_call<<<nblk(nrep, 256), 256, 0, s>>>(nrep, kcall, lam);
}

void launch_apply_lambda(hipStream_t s, int32_t ntiles, const Tile* tiles, int32_t stride,
                         double* vel, double* lam, int32_t nrep, const DevState* st) {
  k_apply_lambda<<<ntiles, kTile, 0, s>>>(tiles, stride, vel, lam, st);
  k_reset_lambda<<<nblk(nrep, 256), 256, 0, s>>>(nrep, lam, st);
}

}  // namespace mdk
