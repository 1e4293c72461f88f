// Mixed-precision trajectory kernel: positions, momenta, the potential, its
// Hessian, the 6x6 monodromy matrix and det R are computed in FP32; the
// action S is accumulated in FP64 (from FP32 stage Lagrangians), and the
// square root of det R with its branch, the recombination element, the
// amplitude and the dipole sum are FP64.
// One trajectory per lane, one 64-lane pack per wavefront; the monodromy
// matrix lives in LDS (element-major, lane-minor, 9 KB per wavefront), the
// rest of the state in VGPRs, so that three wavefronts fit on each SIMD.
#include "device_common.h"

namespace sfhk {
namespace {

constexpr int kMonoElems = 36;  // row-major 6x6, rows (q, p), columns (q0, p0)

// M <- M + (P - I) M for the FP32 monodromy in LDS, one column at a time
// (the next column loaded before the current one is computed); returns the
// largest |entry| of the new matrix.
__device__ __forceinline__ float monodromy_step_f32(const StepMatrix<float>& P,
                                                    float (*mono)[kWave], int lane) {
  float x[3] = {mono[0][lane], mono[6][lane], mono[12][lane]};
  float v[3] = {mono[18][lane], mono[24][lane], mono[30][lane]};
  float mmax = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    __builtin_amdgcn_sched_barrier(0);
    float xl[3] = {0.0f, 0.0f, 0.0f}, vl[3] = {0.0f, 0.0f, 0.0f};
    if (c < 5) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        xl[r] = mono[6 * r + c + 1][lane];
        vl[r] = mono[18 + 6 * r + c + 1][lane];
      }
    }
    float xn[3], vn[3];
    apply_step_increment(P, x, v, xn, vn);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      mono[6 * r + c][lane] = xn[r];
      mono[18 + 6 * r + c][lane] = vn[r];
      mmax = fmaxf(mmax, fmaxf(fabsf(xn[r]), fabsf(vn[r])));
      x[r] = xl[r];
      v[r] = vl[r];
    }
  }
  return mmax;
}

// Track: keep the running monodromy maximum and the count of steps that
// evaluate the recombination sum, and write the records asked for in rec
// (those of trajectories handed to the FP64 re-run are rewritten by it).
template <int U, bool Track>
__device__ __forceinline__ void run_pack_mixed(const Desc* __restrict__ descs,
                                               const double* __restrict__ field,
                                               const EnsPtrs& e, int32_t* __restrict__ redo,
                                               double* __restrict__ accum, const Records& rec,
                                               const Pack& pk, int lane,
                                               float (*mono)[kWave]) {
  const Desc& d = descs[pk.prob];
  const int N = d.N;
  const bool valid = pk.valid;
  const uint32_t slot = pk.slot;

  // initial conditions (FP64 as sampled; FP32 copies for the stepping)
  const int k0 = valid ? e.k0[slot] : N + 1;
  const double q0d[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  const double p0d[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double w = e.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  const double p0q0 = p0d[0] * q0d[0] + p0d[1] * q0d[1] + p0d[2] * q0d[2] + e.dph[slot];
  float q[3] = {(float)q0d[0], (float)q0d[1], (float)q0d[2]};
  float p[3] = {(float)p0d[0], (float)p0d[1], (float)p0d[2]};
  const float hRn[3] = {(float)(d.half_R * n[0]), (float)(d.half_R * n[1]),
                        (float)(d.half_R * n[2])};
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < kMonoElems; ++i) mono[i][lane] = (i % 7 == 0) ? 1.0f : 0.0f;
  double Cre = 1.0, Cim = 0.0, flips = 0.0;

  const double hd = d.dt;
  const float h = d.frk.h, hh = d.frk.hh, h6 = d.frk.h6;
  const double* __restrict__ fe = field + d.field_off;
  double* __restrict__ acc = accum + d.acc_off;
  const int kmin = __builtin_amdgcn_readfirstlane(k0);
  double acc_reg = 0.0;
  int kend = N + 1;  // first step not run here (handed to the FP64 re-run)
  float mmax_all = 1.0f;
  double n_near = 0.0;  // Track only
  int snap_k = Track && rec.snap ? first_snap_step(kmin, rec.snap_every) : -1;
  const int snap_end = Track && rec.snap ? rec.n_snap * rec.snap_every : 0;

  for (int kc = kmin; kc <= N; kc += U) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = kc + u;
    if (k > N) break;
    bool live = k >= k0 && k < kend;
    double re_a = 0.0;
    if (live) {
      // HK matrix and its determinant from the FP32 monodromy matrix, in FP32;
      // the square root, its branch and the amplitude in FP64
      const float ig = (float)d.inv_gamma, gm = (float)d.gamma;
      float Rr[3][3], Ri[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          // R2 = 2R: Mqq[a][b] + Mpp[a][b], (1/g) Mpq[a][b] - g Mqp[a][b]
          Rr[a][b] = mono[6 * a + b][lane] + mono[18 + 6 * a + 3 + b][lane];
          Ri[a][b] = ig * mono[18 + 6 * a + b][lane] - gm * mono[6 * a + 3 + b][lane];
        }
      float Dr, Di;
      det3c(Rr, Ri, Dr, Di);
      // det R = det R2 / 8 (exact)
      sqrt_continued(0.125 * (double)Dr, 0.125 * (double)Di, Cre, Cim, flips);
      if (d.c_max2 > 0.0 && Cre * Cre + Cim * Cim > kMixedCapHandover2 * d.c_max2) {
        // near the prefactor cap: the FP64 re-run deposits from this step on
        // and stops the trajectory where the FP64 prefactor reaches the cap
        kend = k;
        redo[slot] = k;
        live = false;
      } else {
        const double pd_[3] = {(double)p[0], (double)p[1], (double)p[2]};
        const double qd_[3] = {(double)q[0], (double)q[1], (double)q[2]};
        const double hRnd[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
        Geom<double> Gd;
        geometry(d, hRnd, qd_, Gd);
        bool near;
        re_a = amplitude_re(d, n, pd_, Gd, Cre, Cim, S, d.t_first + (double)k * hd, t0, p0q0,
                            w, near);
        if constexpr (Track) n_near += near ? 1.0 : 0.0;
      }
    }
    if constexpr (Track) {
      if (k == snap_k && k < snap_end) {  // wave-uniform
        if (valid && k >= k0 && k < kend)
          write_record(rec.snap + (uint64_t)(k / rec.snap_every) * SFHK_FS_COUNT * rec.capacity +
                           slot, rec.capacity, q, p, mono, lane, S, Cre, Cim, flips,
                       (double)mmax_all, n_near);
        snap_k += rec.snap_every;
      }
    }
    deposit(re_a, k, N, lane, acc_reg, acc);
    if (k >= N || !live) continue;

    // --- classical RK4 step t_k -> t_{k+1}; (q, p, M) in FP32, S in FP64
    const float Ek = (float)fe[2 * k], Eh = (float)fe[2 * k + 1], E1 = (float)fe[2 * k + 2];
    float K1[6], K2[6], K3[6], K4[6];
    float V, g[3];
    float sq[3], sp3[3], yq[3], yp[3];
    float sS;  // weighted sum of the stage Lagrangians p^2/2 - V - q_z E

    potential(d, hRn, q, V, g, K1);
    {
      const float kp[3] = {-g[0], -g[1], -g[2] - Ek};
      sS = 0.5f * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - V - q[2] * Ek;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] = p[a];
        sp3[a] = kp[a];
        yq[a] = q[a] + hh * p[a];
        yp[a] = p[a] + hh * kp[a];
      }
    }
    potential(d, hRn, yq, V, g, K2);
    {
      const float kp[3] = {-g[0], -g[1], -g[2] - Eh};
      sS += 2.0f * (0.5f * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh);
      const float kq[3] = {yp[0], yp[1], yp[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += 2.0f * kq[a];
        sp3[a] += 2.0f * kp[a];
        yq[a] = q[a] + hh * kq[a];
        yp[a] = p[a] + hh * kp[a];
      }
    }
    potential(d, hRn, yq, V, g, K3);
    {
      const float kp[3] = {-g[0], -g[1], -g[2] - Eh};
      sS += 2.0f * (0.5f * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh);
      const float kq[3] = {yp[0], yp[1], yp[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += 2.0f * kq[a];
        sp3[a] += 2.0f * kp[a];
        yq[a] = q[a] + h * kq[a];
        yp[a] = p[a] + h * kp[a];
      }
    }
    potential(d, hRn, yq, V, g, K4);
    {
      const float kp[3] = {-g[0], -g[1], -g[2] - E1};
      sS += 0.5f * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * E1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += yp[a];
        sp3[a] += kp[a];
        q[a] = q[a] + h6 * sq[a];
        p[a] = p[a] + h6 * sp3[a];
      }
      S = S + d.rk.h6 * (double)sS;
    }
    // monodromy: M <- M + (P - I) M with the RK4 step matrix of K1..K4,
    // its identity part left out so that FP32 keeps the O(h^2 K) terms
    StepMatrix<float> P;
    rk4_step_matrix<float, true>(K1, K2, K3, K4, d.frk, P);
    const float mmax = monodromy_step_f32(P, mono, lane);
    if constexpr (Track) mmax_all = fmaxf(mmax_all, mmax);
    // FP32 rounding is amplified by the monodromy matrix: past the bound the
    // trajectory is finished by the FP64 kernel from step k + 1 on
    if (mmax > kMixedFlagNorm) {
      kend = k + 1;
      redo[slot] = kend;
    }
  }
  }

  // trajectories handed to the FP64 re-run get their final state from it
  if constexpr (Track) {
    if (rec.final_state != nullptr && valid && kend > N)
      write_record(rec.final_state + slot, rec.capacity, q, p, mono, lane, S, Cre, Cim, flips,
                   (double)mmax_all, n_near);
  }
}

template <int U, bool Track>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3, 3)))
propagate_mixed_kernel(const Desc* __restrict__ descs, int n_prob,
                       const double* __restrict__ field, EnsPtrs e, int32_t* __restrict__ redo,
                       double* __restrict__ accum, Records rec) {
  __shared__ float mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  Pack pk;
  if (!find_pack(e, n_prob, blockIdx.x, lane, pk)) return;
  run_pack_mixed<U, Track>(descs, field, e, redo, accum, rec, pk, lane, mono);
}

template <int U>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3, 3)))
propagate_mixed_persistent(const Desc* __restrict__ descs, int n_prob,
                           const double* __restrict__ field, EnsPtrs e,
                           int32_t* __restrict__ redo, double* __restrict__ accum,
                           const uint32_t* __restrict__ queue, uint32_t* __restrict__ counter) {
  __shared__ float mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  const uint32_t total = e.pack_start[n_prob];
  for (;;) {
    uint32_t idx = 0;
    if (lane == 0) idx = atomicAdd(counter, 1u);
    idx = __builtin_amdgcn_readfirstlane(idx);
    if (idx >= total) break;
    Pack pk;
    find_pack(e, n_prob, queue[idx], lane, pk);
    run_pack_mixed<U, false>(descs, field, e, redo, accum, Records{}, pk, lane, mono);
  }
}

}  // namespace

hipError_t launch_propagate_mixed(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                                  int32_t* redo, uint32_t max_packs, double* accum,
                                  const Records& rec, hipStream_t s, const LaunchCfg& cfg) {
  if (max_packs == 0) return hipSuccess;
  auto persistent = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(cfg.grid), dim3(kWave), 0, s, descs, n_prob, field, e, redo,
                       accum, cfg.queue, cfg.counter);
  };
  auto per_pack = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(max_packs), dim3(kWave), 0, s, descs, n_prob, field, e, redo,
                       accum, rec);
  };
  if (rec.any()) {
    per_pack(propagate_mixed_kernel<1, true>);
  } else if (cfg.persistent) {
    if (cfg.unroll == 4) persistent(propagate_mixed_persistent<4>);
    else if (cfg.unroll == 2) persistent(propagate_mixed_persistent<2>);
    else persistent(propagate_mixed_persistent<1>);
  } else {
    if (cfg.unroll == 4) per_pack(propagate_mixed_kernel<4, false>);
    else if (cfg.unroll == 2) per_pack(propagate_mixed_kernel<2, false>);
    else per_pack(propagate_mixed_kernel<1, false>);
  }
  return hipGetLastError();
}

}  // namespace sfhk
