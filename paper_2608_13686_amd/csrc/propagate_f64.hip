// FP64 trajectory kernel: one trajectory per lane, one 64-lane pack of
// trajectories of one problem (sorted by birth step) per wavefront.
//
// Per step, for every live lane: HK prefactor from the monodromy matrix,
// coherent-state recombination amplitude, wave-reduced Re a added to the
// dipole accumulator, then one classical RK4 step of (q, p, S) and of the
// six monodromy columns.  (q, p, S), the HK matrix (kept doubled, 2R) and
// the prefactor live in VGPRs for the whole pulse; the monodromy matrix
// lives in LDS.
#include "device_common.h"

namespace sfhk {
namespace {

// Monodromy matrix storage: element-major, lane-minor in LDS, one 18 KB
// slice per wavefront (workgroup = one wavefront), so that every ds access
// of a wavefront touches 64 consecutive doubles.
constexpr int kMonoElems = 36;  // row-major 6x6, rows (q, p), columns (q0, p0)

// One 64-lane pack: every live lane runs its trajectory from its birth step
// to t_N.  U consecutive steps are unrolled per loop trip.  VK: the screening
// exponential's constants are kept in VGPRs (the per-pack kernel has the
// registers; the persistent one would spill).  Track: keep the running
// monodromy maximum and the count of steps that evaluate the recombination
// sum, and write the records asked for in rec.
template <int U, bool VK, bool Track>
__device__ __forceinline__ void run_pack(const Desc* __restrict__ descs,
                                         const double* __restrict__ field, const EnsPtrs& e,
                                         const int32_t* __restrict__ dep_from,
                                         double* __restrict__ accum, const Records& rec,
                                         const Pack& pk, int lane, double (*mono)[kWave]) {
  const Desc& d = descs[pk.prob];
  const int N = d.N;
  const bool valid = pk.valid;
  const uint32_t slot = pk.slot;

  const int k0 = valid ? e.k0[slot] : N + 1;
  // amplitudes are deposited from step kdep on (the re-run of a trajectory
  // that the mixed-precision kernel handed over deposits only its remainder)
  const int kdep = (dep_from != nullptr && valid) ? dep_from[slot] : 0;
  double q[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  double p[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double w = e.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  // phase constant of the amplitude: p0.q0 plus the birth phase
  const double p0q0 = p[0] * q[0] + p[1] * q[1] + p[2] * q[2] + e.dph[slot];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < kMonoElems; ++i) mono[i][lane] = (i % 7 == 0) ? 1.0 : 0.0;
  // twice the HK matrix, R2 = 2R = Mqq + Mpp - i g Mqp + (i/g) Mpq, of the
  // current M
  double Rr[3][3], Ri[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Rr[a][b] = a == b ? 2.0 : 0.0;
      Ri[a][b] = 0.0;
    }
  double Cre = 1.0, Cim = 0.0;
  double flips = 0.0;

  const double h = d.dt;
  const double* __restrict__ fe = field + d.field_off;
  double* __restrict__ acc = accum + d.acc_off;
  const int kmin = __builtin_amdgcn_readfirstlane(k0);
  double acc_reg = 0.0;

  int kend = N + 1;  // first step without contribution (prefactor cap)
  ExpK ekv;
  if constexpr (VK) ekv = make_expk();
  const ExpK* ek = VK ? &ekv : nullptr;
  double mmax = 1.0, n_near = 0.0;  // Track only
  int snap_k = Track && rec.snap ? first_snap_step(kmin, rec.snap_every) : -1;
  const int snap_end = Track && rec.snap ? rec.n_snap * rec.snap_every : 0;

  for (int kc = kmin; kc <= N; kc += U) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = kc + u;
    if (k > N) break;
    bool live = k >= k0 && k < kend;
    double re_a = 0.0;
    const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
    Geom<double> Gk;  // geometry at q_k: amplitude and first RK4 stage
    geometry(d, hRn, q, Gk);
    if (live) {
      prefactor_step(Rr, Ri, Cre, Cim, flips);
      if (d.c_max2 > 0.0 && Cre * Cre + Cim * Cim > d.c_max2) {
        kend = k;
        live = false;
      } else if (k >= kdep) {
        bool near;
        re_a = amplitude_re(d, n, p, Gk, Cre, Cim, S, d.t_first + (double)k * h, t0, p0q0, w,
                            near);
        if constexpr (Track) n_near += near ? 1.0 : 0.0;
      }
    }
    if constexpr (Track) {
      if (k == snap_k && k < snap_end) {  // wave-uniform
        if (valid && k >= k0 && k <= kend)
          write_record(rec.snap + (uint64_t)(k / rec.snap_every) * SFHK_FS_COUNT * rec.capacity +
                           slot, rec.capacity, q, p, mono, lane, S, Cre, Cim, flips, mmax, n_near);
        snap_k += rec.snap_every;
      }
    }
    deposit(re_a, k, N, lane, acc_reg, acc);
    if (k >= N || !live) continue;

    // --- classical RK4 step t_k -> t_{k+1}
    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
    double K1[6], K2[6], K3[6], K4[6];
    double V, g[3];
    double sq[3], sp3[3], sS;  // RK4 weighted sums of the q, p and S slopes
    double yq[3], yp[3];

    potential(d, Gk, V, g, K1, ek);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Ek};
      const double kS = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - V - q[2] * Ek;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] = p[a];
        sp3[a] = kp[a];
        yq[a] = q[a] + 0.5 * h * p[a];
        yp[a] = p[a] + 0.5 * h * kp[a];
      }
      sS = kS;
    }
    potential(d, hRn, yq, V, g, K2, ek);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Eh};
      const double kS = 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh;
      const double kq[3] = {yp[0], yp[1], yp[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += 2.0 * kq[a];
        sp3[a] += 2.0 * kp[a];
        yq[a] = q[a] + 0.5 * h * kq[a];
        yp[a] = p[a] + 0.5 * h * kp[a];
      }
      sS += 2.0 * kS;
    }
    potential(d, hRn, yq, V, g, K3, ek);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Eh};
      const double kS = 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh;
      const double kq[3] = {yp[0], yp[1], yp[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += 2.0 * kq[a];
        sp3[a] += 2.0 * kp[a];
        yq[a] = q[a] + h * kq[a];
        yp[a] = p[a] + h * kp[a];
      }
      sS += 2.0 * kS;
    }
    potential(d, hRn, yq, V, g, K4, ek);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - E1};
      const double kS = 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * E1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += yp[a];
        sp3[a] += kp[a];
        q[a] = q[a] + d.rk.h6 * sq[a];
        p[a] = p[a] + d.rk.h6 * sp3[a];
      }
      sS += kS;
      S = S + d.rk.h6 * sS;
    }
    // monodromy: M <- P M with the RK4 step matrix of the stage Hessians
    // K1..K4 of this step (the exact Jacobian of the discrete RK4 map);
    // columns c and c + 3 give column c of R.
    StepMatrix<double> P;
    rk4_step_matrix(K1, K2, K3, K4, d.rk, P);
    monodromy_step<kWave, Track>(P, mono, lane, d.gamma, d.inv_gamma, Rr, Ri, &mmax);
  }
  }

  if constexpr (Track) {
    if (rec.final_state != nullptr && valid)
      write_record(rec.final_state + slot, rec.capacity, q, p, mono, lane, S, Cre, Cim, flips,
                   mmax, n_near);
  }
}

template <int U, bool Track>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2, 2)))
propagate_f64_kernel(const Desc* __restrict__ descs, int n_prob, const double* __restrict__ field,
                     EnsPtrs e, const int32_t* __restrict__ dep_from, double* __restrict__ accum,
                     Records rec) {
  __shared__ double mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  Pack pk;
  if (!find_pack(e, n_prob, blockIdx.x, lane, pk)) return;
  run_pack<U, true, Track>(descs, field, e, dep_from, accum, rec, pk, lane, mono);
}

// Persistent form: a fixed grid of wavefronts pulls pack indices from
// queue[] through an atomic counter until the queue is exhausted.
template <int U>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2, 2)))
propagate_f64_persistent(const Desc* __restrict__ descs, int n_prob,
                         const double* __restrict__ field, EnsPtrs e,
                         const int32_t* __restrict__ dep_from, double* __restrict__ accum,
                         const uint32_t* __restrict__ queue, uint32_t* __restrict__ counter) {
  __shared__ double mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  const uint32_t total = e.pack_start[n_prob];
  for (;;) {
    uint32_t idx = 0;
    if (lane == 0) idx = atomicAdd(counter, 1u);
    idx = __builtin_amdgcn_readfirstlane(idx);
    if (idx >= total) break;
    Pack pk;
    find_pack(e, n_prob, queue[idx], lane, pk);
    run_pack<U, false, false>(descs, field, e, dep_from, accum, Records{}, pk, lane, mono);
  }
}

}  // namespace

hipError_t launch_propagate_f64(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                                const int32_t* dep_from, uint32_t max_packs, double* accum,
                                const Records& rec, hipStream_t s, const LaunchCfg& cfg) {
  if (max_packs == 0) return hipSuccess;
  auto persistent = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(cfg.grid), dim3(kWave), 0, s, descs, n_prob, field, e,
                       dep_from, accum, cfg.queue, cfg.counter);
  };
  auto per_pack = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(max_packs), dim3(kWave), 0, s, descs, n_prob, field, e,
                       dep_from, accum, rec);
  };
  if (rec.any()) {
    per_pack(propagate_f64_kernel<1, true>);
  } else if (cfg.persistent) {
    if (cfg.unroll == 4) persistent(propagate_f64_persistent<4>);
    else if (cfg.unroll == 2) persistent(propagate_f64_persistent<2>);
    else persistent(propagate_f64_persistent<1>);
  } else {
    if (cfg.unroll == 4) per_pack(propagate_f64_kernel<4, false>);
    else if (cfg.unroll == 2) per_pack(propagate_f64_kernel<2, false>);
    else per_pack(propagate_f64_kernel<1, false>);
  }
  return hipGetLastError();
}

}  // namespace sfhk
