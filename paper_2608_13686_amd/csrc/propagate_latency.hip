// FP64 trajectory kernels for launches far below device fill (latency form):
// one trajectory per group of 8 lanes, 8 trajectories per wavefront; without
// records the orbit runs on a second wavefront a step ahead (pipelined form
// below).
//
// Lane c of a group holds column c of the 6x6 monodromy matrix (c < 6; lanes
// 6 and 7 hold a zero column, which the linear update keeps at zero) and
// advances it by classical RK4 with the stage Hessians of the trajectory,
// stage by stage beside the (q, p, S) stages.  Every lane of the group steps
// (q, p, S) and evaluates the potential itself, so no lane waits for another
// within a step.  Column c of the doubled HK matrix 2R needs columns c and
// c + 3 of M: lane c (< 3) reads column c + 3 from lane c + 3, and lane 0
// gathers the other two columns of 2R from lanes 1 and 2 (DPP row shifts
// inside the group's row of 16 lanes); lane 0 then takes det R, continues
// the root C, evaluates the recombination amplitude and deposits.
//
// The per-step work on the critical path is the potential and the (q, p, S)
// stages plus one column's RK4 (84 operations instead of the 6x6 step
// matrix's ~370), so a step of a trajectory takes about two thirds of the
// time of the one-trajectory-per-lane kernel, at eight times the lanes per
// trajectory: the form for a few hundred packs on 1,024 SIMDs (the FP64
// re-run of trajectories the mixed kernel hands over, small workloads).
#include "device_common.h"

namespace sfhk {
namespace {

constexpr int kGroup = 8;                    // lanes per trajectory
constexpr int kPerWave = kWave / kGroup;     // trajectories per wavefront

// x of lane (lane + N) in the same row of 16 lanes (DPP row shift; lanes
// whose source is outside the row read 0).  The callers only use lanes
// whose source lies in their own 8-lane group, which never crosses a row.
template <int N>
__device__ __forceinline__ double from_lane_plus(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x100 + N, 0xf,
                                                            0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32),
                                                            0x100 + N, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// maximum over the 8 lanes of the group (3 butterfly levels)
__device__ __forceinline__ double group_max(double x) {
  x = fmax(x, __shfl_xor(x, 1, kWave));
  x = fmax(x, __shfl_xor(x, 2, kWave));
  return fmax(x, __shfl_xor(x, 4, kWave));
}

// -K x for the symmetric Hessian K (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void neg_hess_times(const double K[6], const double x[3],
                                               double out[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    out[r] = -(K[sym_idx(r, 0)] * x[0] + K[sym_idx(r, 1)] * x[1] + K[sym_idx(r, 2)] * x[2]);
}

// One group's record (SFHK_FS_* layout): lane c < 6 writes column c of M,
// lane 0 the rest.  mmax is the group's running maximum (all lanes).
__device__ __forceinline__ void write_group_record(double* __restrict__ f, uint64_t st, int c,
                                                   const double q[3], const double p[3],
                                                   const double x[3], const double v[3],
                                                   double S, double Cre, double Cim,
                                                   double flips, double mmax, double n_near) {
  if (c < 6) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      f[(SFHK_FS_M + 6 * r + c) * st] = x[r];
      f[(SFHK_FS_M + 18 + 6 * r + c) * st] = v[r];
    }
  }
  if (c == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[(SFHK_FS_Q + a) * st] = q[a];
      f[(SFHK_FS_P + a) * st] = p[a];
    }
    f[SFHK_FS_S * st] = S;
    f[SFHK_FS_CRE * st] = Cre;
    f[SFHK_FS_CIM * st] = Cim;
    f[SFHK_FS_FLIPS * st] = flips;
    f[SFHK_FS_MMAX * st] = mmax;
    f[SFHK_FS_NEAR * st] = n_near;
  }
}

// The trajectories of one unit (8 consecutive positions of a 64-lane pack):
// group g of the wavefront takes position unit_pos + g of its problem.
template <bool Track>
__device__ __forceinline__ void run_unit(const Desc* __restrict__ descs,
                                         const double* __restrict__ field, const EnsPtrs& e,
                                         const int32_t* __restrict__ dep_from,
                                         double* __restrict__ accum, const Records& rec,
                                         int prob, uint32_t unit_pos, int lane) {
  const Desc& d = descs[prob];
  const int N = d.N;
  const int c = lane & (kGroup - 1);
  const uint32_t pos = unit_pos + (uint32_t)(lane / kGroup);
  const bool valid = pos < e.live_count[prob];
  const uint32_t slot = valid ? e.order[e.live_start[prob] + pos] : 0u;

  const int k0 = valid ? e.k0[slot] : N + 1;
  const int kdep = (dep_from != nullptr && valid) ? dep_from[slot] : 0;
  double q[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  double p[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double w = e.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  const double p0q0 = p[0] * q[0] + p[1] * q[1] + p[2] * q[2] + e.dph[slot];
  double S = 0.0;
  // this lane's monodromy column: d(q, p)/dz_c, M(t0) = identity
  double x[3], v[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    x[r] = (c == r) ? 1.0 : 0.0;
    v[r] = (c == r + 3) ? 1.0 : 0.0;
  }
  double Cre = 1.0, Cim = 0.0, flips = 0.0;
  const double h = d.rk.h, hh = d.rk.hh, h6 = d.rk.h6;
  const double* __restrict__ fe = field + d.field_off;
  double* __restrict__ acc = accum + d.acc_off;
  // the wavefront's first trajectory is born first (sorted by birth step)
  const int kmin = __builtin_amdgcn_readfirstlane(k0);
  double acc_reg = 0.0;
  int kend = N + 1;  // first step without contribution (prefactor cap)
  double mmax = 1.0, n_near = 0.0;  // Track only: this lane's column, then the group's
  int snap_k = Track && rec.snap ? first_snap_step(kmin, rec.snap_every) : -1;
  const int snap_end = Track && rec.snap ? rec.n_snap * rec.snap_every : 0;
  const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
  const double gamma = d.gamma, inv_gamma = d.inv_gamma;
  // the screening exponential's constants in VGPRs: a lone wavefront would
  // otherwise wait on a scalar move and its hazard before every Horner step
  const ExpK ekv = make_expk();

  for (int k = kmin; k <= N; ++k) {
    bool live = k >= k0 && k < kend;
    // column c of 2R = Mqq + Mpp - i g Mqp + (i/g) Mpq from columns c, c + 3
    double x3[3], v3[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      x3[r] = from_lane_plus<3>(x[r]);
      v3[r] = from_lane_plus<3>(v[r]);
    }
    double rr[3], ri[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      rr[r] = x[r] + v3[r];
      ri[r] = fma(inv_gamma, v[r], -gamma * x3[r]);
    }
    double Rr[3][3], Ri[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      Rr[r][0] = rr[r];
      Ri[r][0] = ri[r];
      Rr[r][1] = from_lane_plus<1>(rr[r]);
      Ri[r][1] = from_lane_plus<1>(ri[r]);
      Rr[r][2] = from_lane_plus<2>(rr[r]);
      Ri[r][2] = from_lane_plus<2>(ri[r]);
    }
    double re_a = 0.0;
    Geom<double> Gk;  // geometry at q_k: amplitude and first RK4 stage
    geometry(d, hRn, q, Gk);
    if (live && c == 0) {
      prefactor_step(Rr, Ri, Cre, Cim, flips);
      if (d.c_max2 > 0.0 && Cre * Cre + Cim * Cim > d.c_max2) {
        kend = k;
      } else if (k >= kdep) {
        bool near;
        re_a = amplitude_re(d, n, p, Gk, Cre, Cim, S, d.t_first + (double)k * h, t0, p0q0, w,
                            near);
        if constexpr (Track) n_near += near ? 1.0 : 0.0;
      }
    }
    if (d.c_max2 > 0.0) {  // the cap decision of lane 0 holds for its whole group
      kend = __shfl(kend, lane & ~(kGroup - 1), kWave);
      live = k >= k0 && k < kend;
    }
    if constexpr (Track) {
      if (k == snap_k && k < snap_end) {  // wave-uniform
        const double gm = group_max(mmax);
        if (valid && k >= k0 && k <= kend)
          write_group_record(rec.snap + (uint64_t)(k / rec.snap_every) * SFHK_FS_COUNT *
                                            rec.capacity + slot,
                             rec.capacity, c, q, p, x, v, S, Cre, Cim, flips, gm, n_near);
        snap_k += rec.snap_every;
      }
    }
    deposit(re_a, k, N, lane, acc_reg, acc);
    if (k >= N || !live) continue;

    // --- classical RK4 step t_k -> t_{k+1} of (q, p, S) and of this column
    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
    double K[6], V, g[3];
    double sq[3], sp3[3], sS, yq[3], yp[3];
    double sx[3], sv[3], xs[3], vs[3], kv[3];

    potential(d, Gk, V, g, K, &ekv);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Ek};
      sS = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - V - q[2] * Ek;
      neg_hess_times(K, x, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] = p[a];
        sp3[a] = kp[a];
        yq[a] = q[a] + hh * p[a];
        yp[a] = p[a] + hh * kp[a];
        sx[a] = v[a];
        sv[a] = kv[a];
        xs[a] = x[a] + hh * v[a];
        vs[a] = v[a] + hh * kv[a];
      }
    }
    potential(d, hRn, yq, V, g, K, &ekv);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Eh};
      sS += 2.0 * (0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh);
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double kq = yp[a], kx = vs[a];
        sq[a] += 2.0 * kq;
        sp3[a] += 2.0 * kp[a];
        yq[a] = q[a] + hh * kq;
        yp[a] = p[a] + hh * kp[a];
        sx[a] += 2.0 * kx;
        sv[a] += 2.0 * kv[a];
        xs[a] = x[a] + hh * kx;
        vs[a] = v[a] + hh * kv[a];
      }
    }
    potential(d, hRn, yq, V, g, K, &ekv);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - Eh};
      sS += 2.0 * (0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * Eh);
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double kq = yp[a], kx = vs[a];
        sq[a] += 2.0 * kq;
        sp3[a] += 2.0 * kp[a];
        yq[a] = q[a] + h * kq;
        yp[a] = p[a] + h * kp[a];
        sx[a] += 2.0 * kx;
        sv[a] += 2.0 * kv[a];
        xs[a] = x[a] + h * kx;
        vs[a] = v[a] + h * kv[a];
      }
    }
    potential(d, hRn, yq, V, g, K, &ekv);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - E1};
      sS += 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * E1;
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += yp[a];
        sp3[a] += kp[a];
        q[a] = q[a] + h6 * sq[a];
        p[a] = p[a] + h6 * sp3[a];
        sx[a] += vs[a];
        sv[a] += kv[a];
        x[a] = x[a] + h6 * sx[a];
        v[a] = v[a] + h6 * sv[a];
      }
      S = S + h6 * sS;
    }
    if constexpr (Track) {
#pragma unroll
      for (int r = 0; r < 3; ++r) mmax = fmax(mmax, fmax(fabs(x[r]), fabs(v[r])));
    }
  }

  if constexpr (Track) {
    const double gm = group_max(mmax);
    if (rec.final_state != nullptr && valid)
      write_group_record(rec.final_state + slot, rec.capacity, c, q, p, x, v, S, Cre, Cim, flips,
                         gm, n_near);
  }
}

// Unit sub of a pack of 64 trajectories, units of U trajectories: positions
// U sub .. U sub + U - 1 of the pack.
template <int U = kPerWave>
__device__ __forceinline__ bool find_unit(const EnsPtrs& e, int n_prob, uint32_t pack,
                                          uint32_t sub, int& prob, uint32_t& unit_pos) {
  if (pack >= e.pack_start[n_prob]) return false;
  int lo = 0, hi = n_prob;  // pack_start[lo] <= pack < pack_start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (e.pack_start[mid] <= pack) lo = mid; else hi = mid;
  }
  prob = lo;
  unit_pos = (pack - e.pack_start[lo]) * kWave + sub * U;
  return unit_pos < e.live_count[lo];
}

// ------------------------------------------------------------ pipelined
// The same latency form on 1 + M wavefronts per unit of 8 M trajectories
// (M = 1 or 2), so that the two halves of a step run on different SIMDs at
// once: wavefront 0 (the orbit wavefront, lanes 2g and 2g + 1 for trajectory
// g) integrates (q, p, S) and evaluates the four stage Hessians, two stages
// per lane; wavefronts 1 .. M (the monodromy wavefronts, 8 trajectories of 8
// lanes each as above) take the prefactor, amplitude and deposit at step k
// and advance their columns with the Hessians of step k.  The orbit
// wavefront runs one step ahead: in iteration i it writes step i's state and
// Hessians into ring slot i mod 2 of LDS while the monodromy wavefronts read
// step i - 1's from the other slot; one workgroup barrier per iteration
// hands the slots over.  A
// monodromy wavefront spreads det R over lanes 0-2 (one cofactor term each),
// the recombination amplitude's shells over the 8 lanes of the group, and
// keeps each step's amplitudes in LDS, summing them across trajectories once
// every 64 steps.  The orbit and the columns take the one-wavefront form's
// operations on the same operands in the same order; det R's, the
// amplitude's and the dipole's sums are ordered differently
// (rounding-level differences).  The orbit of a trajectory stopped by the
// prefactor cap is integrated on but not used; records (which hold the
// stopping step's state) use the one-wavefront form.
// A unit of M monodromy wavefronts holds 8 M trajectories; its orbit
// wavefront uses 16 M of its lanes.  M = 2 halves the orbit wavefronts of a
// crowded launch (many units per SIMD: the issue slots they take are the
// step time); one unit alone steps faster with M = 1.
template <int M> constexpr int pipe_traj() { return M * kPerWave; }
template <int M> constexpr int pipe_units_per_pack() { return kWave / pipe_traj<M>(); }
template <int M> constexpr int pipe_threads() { return (1 + M) * kWave; }

// 32-bit DPP move of both halves of a double (control code Ctl)
template <int Ctl>
__device__ __forceinline__ double dpp64(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, Ctl, 0xf, 0xf,
                                                            true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), Ctl, 0xf,
                                                            0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 8 lanes of a group, on every lane of it: lanes i ^ 1 and
// i ^ 2 through quad permutations, then the two quads through the half-row
// mirror (lane i <-> 7 - i).  Every lane adds the same operands in the same
// order up to commutation, so all hold the same value.
__device__ __forceinline__ double group_sum(double x) {
  x += dpp64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  return x + dpp64<0x141>(x);  // row_half_mirror
}

// Lane 0's value of x on every lane of its group of 8: the quad broadcast,
// then the half-row mirror written into the upper quad only (bank mask).
__device__ __forceinline__ int group_bcast0(int x) {
  const int y = __builtin_amdgcn_update_dpp(0, x, 0x00, 0xf, 0xf, false);  // quad_perm [0,0,0,0]
  return __builtin_amdgcn_update_dpp(y, y, 0x141, 0xf, 0xA, false);        // row_half_mirror
}

// The recombination amplitude of amplitude_re with the shells spread over
// the 8 lanes of the trajectory's group (lane c takes shells c, c + 8, ...),
// the phase factor evaluated on every lane beside them, and the shells'
// sums gathered by group_sum: the same terms as amplitude_re, summed in a
// different order.  The gate takes the nearest centre's squared distance
// dd_min and the binary exponent of 1 + |C|^2 (ex, lane 0's, on every lane
// of the group); the geometry at q is built only past the gate.  The value
// is lane 0's (the other lanes' C is not the trajectory's).
__device__ __forceinline__ double amplitude_re_group(const Desc& d, const PotK<double>& pk,
                                                     double g_inv4k_min, const double hRn[3],
                                                     const double n[3], const double q[3],
                                                     const double p[3], double dd_min, int ex,
                                                     double Cre, double Cim, double S,
                                                     double tk, double t0, double p0q0,
                                                     double w, int c) {
  const double lnC = 0.3466 * (double)ex;
  if (dd_min * g_inv4k_min + kRecombFar > lnC) return 0.0;  // group-uniform
  Geom<double> G;
  geometry_p(pk, hRn, q, G);
  const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const double dd[2] = {G.r2[0] - pk.eps2(0), G.r2[1] - pk.eps2(1)};
  const double np_ = n[0] * p[0] + n[1] * p[1] + n[2] * p[2];
  const double bzr = p[2] * d.inv_gamma;
  const double nbr = np_ * d.inv_gamma;
  const double bb_re_p = pp * d.inv_gamma2;
  const double ppg = pp * d.half_inv_gamma;
  double rr = 0.0, ri = 0.0;
  for (int j = c; j < d.n_shell; j += kGroup) {
    const int ce = j < d.n_shell0 ? 0 : 1;
    const double dz = -G.dz[ce];
    const double pd = -(p[0] * G.dx[ce] + p[1] * G.dy[ce] + p[2] * G.dz[ce]);
    const double nd = -(n[0] * G.dx[ce] + n[1] * G.dy[ce] + n[2] * G.dz[ce]);
    const double i4 = d.sh_inv4k[j], i2 = 2.0 * i4;
    const double er = (bb_re_p - dd[ce]) * i4 - ppg;
    if (er + lnC < kRecombFar) continue;
    const double ei = 2.0 * pd * d.inv_gamma * i4;
    const double gm = exp_neg(-er);
    double sn, cs;
    sincos_k(ei, sn, cs);
    const double Gr = gm * cs, Gi = gm * sn;
    double Xr = d.sh_ns[j] * bzr * i2, Xi = d.sh_ns[j] * dz * i2;
    if (d.sh_np[j] != 0.0) {
      const double ur = n[2] * i2 + (bzr * nbr - dz * nd) * i2 * i2;
      const double ui = (bzr * nd + dz * nbr) * i2 * i2;
      Xr -= d.sh_np[j] * ui;
      Xi += d.sh_np[j] * ur;
    }
    rr += Gr * Xr - Gi * Xi;
    ri += Gr * Xi + Gi * Xr;
  }
  const double phi = S - d.Ip * (tk - t0) + p0q0;
  double sp, cp;
  sincos_k(phi, sp, cp);
  rr = group_sum(rr);
  ri = group_sum(ri);
  if (rr == 0.0 && ri == 0.0) return 0.0;
  const double er_ = Cre * cp - Cim * sp, ei_ = Cre * sp + Cim * cp;
  return -w * (er_ * rr - ei_ * ri);
}

template <int M>
struct PipeRing {
  static constexpr int T = pipe_traj<M>();
  double K[2][4][6][T];  // slot, RK4 stage, Hessian entry, trajectory
  double st[2][8][T];    // slot, (q, p, S, dd_min) at the step, trajectory
  double dep[kWave][T];  // Re a of the last 64 steps (step mod 64, trajectory)
};

template <int M>
__device__ __forceinline__ void run_pipe_unit(const Desc* __restrict__ descs,
                                              const double* __restrict__ field, const EnsPtrs& e,
                                              const int32_t* __restrict__ dep_from,
                                              double* __restrict__ accum, int prob,
                                              uint32_t unit_pos, PipeRing<M>& ring) {
  const Desc& d = descs[prob];
  const int N = d.N;
  const int wave = threadIdx.x / kWave;  // 0: orbit, 1 ..: monodromy
  const bool orbit_wave = wave == 0;
  const int lane = threadIdx.x & (kWave - 1);
  const int mw0 = orbit_wave ? 0 : (wave - 1) * kPerWave;  // first trajectory of the wavefront
  const int g = orbit_wave ? lane >> 1 : mw0 + lane / kGroup;  // trajectory of the unit
  const int c = lane & (kGroup - 1);                           // monodromy column
  const uint32_t pos = unit_pos + (uint32_t)g;
  const bool valid = g < pipe_traj<M>() && pos < e.live_count[prob];
  const uint32_t slot = valid ? e.order[e.live_start[prob] + pos] : 0u;
  const int k0 = valid ? e.k0[slot] : N + 1;
  // the unit's first trajectory is born first (sorted by birth step)
  const int kmin = e.k0[e.order[e.live_start[prob] + unit_pos]];
  const double h = d.rk.h, hh = d.rk.hh, h6 = d.rk.h6;
  double q[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  double p[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
  double S = 0.0;

  if (orbit_wave) {
    // Lanes 2g and 2g + 1 both hold trajectory g's (q, p, S).  RK4's stages
    // 1 and 2 are evaluated at q and q + h/2 p, so they depend on (q, p)
    // only; stage 3's point needs stage 1's force only, stage 4's stage 2's.
    // Lane j of the pair evaluates stages 1 + j and 3 + j (j = 0: q, then
    // q + h/2 (p + h/2 F1); j = 1: q + h/2 p, then q + h (p + h/2 F2)), writes
    // their Hessians, and the pair exchanges the four gradients and
    // potentials; both lanes then combine the stages in the classical order,
    // with the same operations as a one-lane step.
    const int j = lane & 1;
    const double* __restrict__ fe = field + d.field_off;
    const ExpK ekv = make_expk();
    // the potential's constants in VGPRs for the whole loop (opaque, so the
    // compiler neither reloads them from the descriptor nor keeps them in
    // scarce SGPRs)
    PotK<double> pk = pot_k<double>(d);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int ce = 0; ce < 2; ++ce) asm volatile("" : "+v"(pk.v[r][ce]));
    const double cA = j ? hh : 0.0, cB = j ? h : hh;
    for (int i = kmin; i <= N + 1; ++i) {
      if (valid && i <= N) {
        const int sl = i & 1;
        double yq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) yq[a] = q[a] + cA * p[a];  // lane 0: q exactly
        Geom<double> G;
        geometry_p(pk, hRn, yq, G);
        if (j == 0) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            ring.st[sl][a][g] = q[a];
            ring.st[sl][3 + a][g] = p[a];
          }
          ring.st[sl][6][g] = S;
          // the recombination gate's nearest-centre squared distance at q
          ring.st[sl][7][g] = fmin(G.r2[0] - pk.eps2(0), G.r2[1] - pk.eps2(1));
        }
        if (i >= k0 && i < N) {
          const double Ek = fe[2 * i], Eh = fe[2 * i + 1], E1 = fe[2 * i + 2];
          double yp[3], VA, VB, gA[3], gB[3], K[6];
          potential_p(pk, G, VA, gA, K, &ekv);
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) ring.K[sl][j][jj][g] = K[jj];
          {
            const double EA = j ? Eh : Ek;
            const double kp[3] = {-gA[0], -gA[1], -gA[2] - EA};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              yp[a] = p[a] + hh * kp[a];  // p at stage 2 (lane 0), stage 3 (lane 1)
              yq[a] = q[a] + cB * yp[a];  // stage 3 (lane 0), stage 4 (lane 1)
            }
          }
          geometry_p(pk, hRn, yq, G);
          potential_p(pk, G, VB, gB, K, &ekv);
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) ring.K[sl][2 + j][jj][g] = K[jj];
          // stage s's gradient and potential on both lanes: from lane
          // (s - 1) & 1 of the pair (quad permutations [0,0,2,2], [1,1,3,3])
          double gr[4][3], V[4];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            gr[0][a] = dpp64<0xA0>(gA[a]);
            gr[1][a] = dpp64<0xF5>(gA[a]);
            gr[2][a] = dpp64<0xA0>(gB[a]);
            gr[3][a] = dpp64<0xF5>(gB[a]);
          }
          V[0] = dpp64<0xA0>(VA);
          V[1] = dpp64<0xF5>(VA);
          V[2] = dpp64<0xA0>(VB);
          V[3] = dpp64<0xF5>(VB);
          double sq[3], sp3[3], sS;
          {
            const double kp[3] = {-gr[0][0], -gr[0][1], -gr[0][2] - Ek};
            sS = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - V[0] - q[2] * Ek;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              sq[a] = p[a];
              sp3[a] = kp[a];
              yq[a] = q[a] + hh * p[a];
              yp[a] = p[a] + hh * kp[a];
            }
          }
          {
            const double kp[3] = {-gr[1][0], -gr[1][1], -gr[1][2] - Eh};
            sS += 2.0 * (0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V[1] - yq[2] * Eh);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double kq = yp[a];
              sq[a] += 2.0 * kq;
              sp3[a] += 2.0 * kp[a];
              yq[a] = q[a] + hh * kq;
              yp[a] = p[a] + hh * kp[a];
            }
          }
          {
            const double kp[3] = {-gr[2][0], -gr[2][1], -gr[2][2] - Eh};
            sS += 2.0 * (0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V[2] - yq[2] * Eh);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double kq = yp[a];
              sq[a] += 2.0 * kq;
              sp3[a] += 2.0 * kp[a];
              yq[a] = q[a] + h * kq;
              yp[a] = p[a] + h * kp[a];
            }
          }
          {
            const double kp[3] = {-gr[3][0], -gr[3][1], -gr[3][2] - E1};
            sS += 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V[3] - yq[2] * E1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              sq[a] += yp[a];
              sp3[a] += kp[a];
              q[a] = q[a] + h6 * sq[a];
              p[a] = p[a] + h6 * sp3[a];
            }
            S = S + h6 * sS;
          }
        }
      }
      __syncthreads();
    }
    return;
  }

  // monodromy wavefront
  const int kdep = (dep_from != nullptr && valid) ? dep_from[slot] : 0;
  const double w = e.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  const double p0q0 = p[0] * q[0] + p[1] * q[1] + p[2] * q[2] + e.dph[slot];
  double x[3], v[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    x[r] = (c == r) ? 1.0 : 0.0;
    v[r] = (c == r + 3) ? 1.0 : 0.0;
  }
  double Cre = 1.0, Cim = 0.0, flips = 0.0;
  double* __restrict__ acc = accum + d.acc_off;
  const double gamma = d.gamma, inv_gamma = d.inv_gamma;
  int kend = N + 1;
  // per-step constants in registers for the whole loop (opaque: neither
  // reloaded from the descriptor nor rematerialised)
  PotK<double> pk = pot_k<double>(d);
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int ce = 0; ce < 2; ++ce) asm volatile("" : "+v"(pk.v[r][ce]));
  double c_max2 = d.c_max2, g_inv4k_min = d.g_inv4k_min;
  asm volatile("" : "+v"(c_max2), "+v"(g_inv4k_min));
  int capped = __builtin_amdgcn_readfirstlane(d.c_max2 > 0.0 ? 1 : 0);
  asm volatile("" : "+s"(capped));
  __syncthreads();  // iteration kmin: the orbit wavefront writes step kmin
  for (int k = kmin; k <= N; ++k) {
    const int sl = k & 1;
    bool live = k >= k0 && k < kend;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q[a] = ring.st[sl][a][g];
      p[a] = ring.st[sl][3 + a][g];
    }
    S = ring.st[sl][6][g];
    const double dd_min = ring.st[sl][7][g];
    double x3[3], v3[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      x3[r] = from_lane_plus<3>(x[r]);
      v3[r] = from_lane_plus<3>(v[r]);
    }
    double rr[3], ri[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      rr[r] = x[r] + v3[r];
      ri[r] = fma(inv_gamma, v[r], -gamma * x3[r]);
    }
    // det 2R by the cyclic cofactor expansion along row 0: lane c < 3 takes
    // the term of column c, its minor from columns c + 1 and c + 2 (mod 3)
    // of rows 1 and 2 (quad permutations [1,2,0,3] and [2,0,1,3]); lane 3's
    // term is zero, and two quad exchanges sum the terms on lane 0
    const double a1r = dpp64<0xC9>(rr[1]), a1i = dpp64<0xC9>(ri[1]);  // R[1][c+1]
    const double a2r = dpp64<0xC9>(rr[2]), a2i = dpp64<0xC9>(ri[2]);  // R[2][c+1]
    const double b1r = dpp64<0xD2>(rr[1]), b1i = dpp64<0xD2>(ri[1]);  // R[1][c+2]
    const double b2r = dpp64<0xD2>(rr[2]), b2i = dpp64<0xD2>(ri[2]);  // R[2][c+2]
    const double mr = fma(a1r, b2r, fma(-a1i, b2i, fma(-b1r, a2r, b1i * a2i)));
    const double mi = fma(a1r, b2i, fma(a1i, b2r, fma(-b1r, a2i, -(b1i * a2r))));
    double tr = c < 3 ? fma(rr[0], mr, -(ri[0] * mi)) : 0.0;
    double ti = c < 3 ? fma(rr[0], mi, ri[0] * mr) : 0.0;
    tr += dpp64<0xB1>(tr);
    ti += dpp64<0xB1>(ti);
    tr += dpp64<0x4E>(tr);
    ti += dpp64<0x4E>(ti);
    double re_a = 0.0;
    if (live && c == 0) {
      sqrt_continued(0.125 * tr, 0.125 * ti, Cre, Cim, flips);
      if (capped && Cre * Cre + Cim * Cim > c_max2) kend = k;
    }
    if (capped) {  // the cap decision of lane 0 holds for its whole group
      kend = __shfl(kend, lane & ~(kGroup - 1), kWave);
      live = k >= k0 && k < kend;
    }
    if (live && k >= kdep) {  // group-uniform
      // the binary exponent of 1 + |C|^2 of lane 0 for the gate
      const double cc = 1.0 + Cre * Cre + Cim * Cim;
      const int ex = group_bcast0(((int)(__double_as_longlong(cc) >> 52) & 0x7ff) - 1022);
      const double a = amplitude_re_group(d, pk, g_inv4k_min, hRn, n, q, p, dd_min, ex, Cre, Cim,
                                          S, d.t_first + (double)k * h, t0, p0q0, w, c);
      re_a = c == 0 ? a : 0.0;
    }
    // deposit: each trajectory's Re a_k goes to LDS (no cross-lane sum per
    // step); every 64 steps, and at the last, lane j adds the 8 values of
    // step (k & ~63) + j and flushes them with one coalesced atomic
    if (c == 0) ring.dep[k & (kWave - 1)][g] = re_a;
    if ((k & (kWave - 1)) == kWave - 1 || k == N) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int kb = k & ~(kWave - 1);
      if (lane <= (k & (kWave - 1)) && kb + lane >= kmin) {
        double tot = 0.0;
#pragma unroll
        for (int t = 0; t < kPerWave; ++t) tot += ring.dep[lane][mw0 + t];
        if (tot != 0.0) unsafeAtomicAdd(&acc[kb + lane], tot);
      }
    }
    if (k < N && live) {
      double sx[3], sv[3], xs[3], vs[3], kv[3], K[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) K[j] = ring.K[sl][0][j][g];
      neg_hess_times(K, x, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sx[a] = v[a];
        sv[a] = kv[a];
        xs[a] = x[a] + hh * v[a];
        vs[a] = v[a] + hh * kv[a];
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) K[j] = ring.K[sl][1][j][g];
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double kx = vs[a];
        sx[a] += 2.0 * kx;
        sv[a] += 2.0 * kv[a];
        xs[a] = x[a] + hh * kx;
        vs[a] = v[a] + hh * kv[a];
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) K[j] = ring.K[sl][2][j][g];
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double kx = vs[a];
        sx[a] += 2.0 * kx;
        sv[a] += 2.0 * kv[a];
        xs[a] = x[a] + h * kx;
        vs[a] = v[a] + h * kv[a];
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) K[j] = ring.K[sl][3][j][g];
      neg_hess_times(K, xs, kv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sx[a] += vs[a];
        sv[a] += kv[a];
        x[a] = x[a] + h6 * sx[a];
        v[a] = v[a] + h6 * sv[a];
      }
    }
    __syncthreads();
  }
}

template <int M>
__global__ void __launch_bounds__(pipe_threads<M>())
propagate_pipe_kernel(const Desc* __restrict__ descs, int n_prob,
                      const double* __restrict__ field, EnsPtrs e,
                      const int32_t* __restrict__ dep_from, double* __restrict__ accum) {
  __shared__ PipeRing<M> ring;
  constexpr int kU = pipe_units_per_pack<M>();
  int prob;
  uint32_t unit_pos;
  if (!find_unit<pipe_traj<M>()>(e, n_prob, blockIdx.x / kU, blockIdx.x % kU, prob, unit_pos))
    return;
  run_pipe_unit<M>(descs, field, e, dep_from, accum, prob, unit_pos, ring);
}

// Persistent form: a fixed grid of workgroups pulls units (pack
// queue[u / units per pack], unit u % units per pack of it) through an
// atomic counter until all are taken.
template <int M>
__global__ void __launch_bounds__(pipe_threads<M>())
propagate_pipe_persistent(const Desc* __restrict__ descs, int n_prob,
                          const double* __restrict__ field, EnsPtrs e,
                          const int32_t* __restrict__ dep_from, double* __restrict__ accum,
                          const uint32_t* __restrict__ queue, uint32_t* __restrict__ counter) {
  __shared__ PipeRing<M> ring;
  __shared__ uint32_t next;
  constexpr int kU = pipe_units_per_pack<M>();
  const uint32_t total = e.pack_start[n_prob] * (uint32_t)kU;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t u = next;
    __syncthreads();  // every thread has read `next` before thread 0 rewrites it
    if (u >= total) break;
    int prob;
    uint32_t unit_pos;
    if (!find_unit<pipe_traj<M>()>(e, n_prob, queue[u / kU], u % kU, prob, unit_pos)) continue;
    run_pipe_unit<M>(descs, field, e, dep_from, accum, prob, unit_pos, ring);
  }
}

template <int M>
hipError_t launch_pipe(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                       const int32_t* dep_from, uint32_t max_packs, double* accum, hipStream_t s,
                       const LaunchCfg& cfg) {
  if (cfg.persistent) {
    // cfg.grid counts wavefronts: 1 + M per workgroup
    const uint32_t grid = cfg.grid / (1 + M) > 0 ? cfg.grid / (1 + M) : 1;
    hipLaunchKernelGGL(propagate_pipe_persistent<M>, dim3(grid), dim3(pipe_threads<M>()), 0, s,
                       descs, n_prob, field, e, dep_from, accum, cfg.queue, cfg.counter);
  } else {
    const uint32_t units = (uint32_t)((uint64_t)max_packs * pipe_units_per_pack<M>());
    hipLaunchKernelGGL(propagate_pipe_kernel<M>, dim3(units), dim3(pipe_threads<M>()), 0, s,
                       descs, n_prob, field, e, dep_from, accum);
  }
  return hipGetLastError();
}

template <bool Track>
__global__ void __launch_bounds__(kWave)
propagate_latency_kernel(const Desc* __restrict__ descs, int n_prob,
                         const double* __restrict__ field, EnsPtrs e,
                         const int32_t* __restrict__ dep_from, double* __restrict__ accum,
                         Records rec) {
  int prob;
  uint32_t unit_pos;
  if (!find_unit(e, n_prob, blockIdx.x / kPerWave, blockIdx.x % kPerWave, prob, unit_pos)) return;
  run_unit<Track>(descs, field, e, dep_from, accum, rec, prob, unit_pos, threadIdx.x);
}

}  // namespace

hipError_t launch_propagate_latency(const Desc* descs, int n_prob, const double* field,
                                    EnsPtrs e, const int32_t* dep_from, uint32_t max_packs,
                                    double* accum, const Records& rec, hipStream_t s,
                                    const LaunchCfg& cfg) {
  if (max_packs == 0) return hipSuccess;
  if (rec.any()) {  // records: the one-wavefront form
    const uint32_t units = (uint32_t)((uint64_t)max_packs * kPerWave);
    hipLaunchKernelGGL(propagate_latency_kernel<true>, dim3(units), dim3(kWave), 0, s, descs,
                       n_prob, field, e, dep_from, accum, rec);
    return hipGetLastError();
  }
  return cfg.pipe_mono == 2
             ? launch_pipe<2>(descs, n_prob, field, e, dep_from, max_packs, accum, s, cfg)
             : launch_pipe<1>(descs, n_prob, field, e, dep_from, max_packs, accum, s, cfg);
}

}  // namespace sfhk
