// FP64 trajectory kernel: one trajectory per lane, one 64-lane pack of
// trajectories of one problem (sorted by birth step) per wavefront.
//
// Per step, for every live lane: HK prefactor from the monodromy matrix,
// coherent-state recombination amplitude, wave-reduced Re a added to the
// dipole accumulator, then one classical RK4 step of (q, p, S) and of the
// six monodromy columns.  State lives in VGPRs for the whole pulse.
#include "sfhk_internal.h"

namespace sfhk {
namespace {

// 1/sqrt(x), x > 0: the hardware estimate (relative error ~2^-24) refined by
// the second-order expansion of (1 - e)^(-1/2), e = 1 - x y^2 (error < 2 ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Far-field cut-offs.  Screening: for alpha*rho > kScreenFar the terms of
// dZ e^{-alpha rho} in V, V' and V'' are below 1e-21 of the Z_inf terms, far
// under one rounding unit, so they are not evaluated.  Recombination: a GTO
// primitive whose Gaussian exponent satisfies er + ln(1 + |C|) < kRecombFar
// contributes less than 1e-30 to a dipole sample (|b|-dependent factors and
// norms are bounded by 1e4), so its exp and sincos are not evaluated.
constexpr double kScreenFar = 60.0;
constexpr double kRecombFar = -75.0;

// Two-centre potential of Eq. 7 with softened distance (per centre
// V_i = -Z_i(rho)/rho, Z_i = Zinf + dZ e^{-alpha rho}, rho^2 = |q-R_i|^2 + eps2):
// value, gradient and the symmetric Hessian K (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ void potential(const Desc& d, const double hRn[3], const double q[3],
                                          double& V, double g[3], double K[6]) {
  V = 0.0;
  g[0] = g[1] = g[2] = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) K[a] = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double s = c == 0 ? 1.0 : -1.0;
    const double dx = q[0] - s * hRn[0];
    const double dy = q[1] - s * hRn[1];
    const double dz = q[2] - s * hRn[2];
    const double r2 = dx * dx + dy * dy + dz * dz + d.eps2[c];
    const double inv = rsqrt_nr(r2);
    double Z = d.Zinf[c];
    double f1 = Z * inv * inv;
    double f2 = -2.0 * Z * inv * inv * inv;
    if (d.screened) {
      const double ar = d.alpha[c] * (r2 * inv);
      if (ar < kScreenFar) {
        const double ex = exp(-ar);
        const double adx = d.alpha[c] * d.dZ[c] * ex;
        Z += d.dZ[c] * ex;
        f1 = (Z * inv + adx) * inv;
        f2 = -(2.0 * Z * inv * inv + 2.0 * adx * inv + d.alpha[c] * adx) * inv;
      }
    }
    V -= Z * inv;
    const double c1 = f1 * inv;                 // f'/rho
    const double c2 = (f2 - c1) * inv * inv;    // (f'' - f'/rho)/rho^2
    g[0] += c1 * dx;
    g[1] += c1 * dy;
    g[2] += c1 * dz;
    K[0] += c2 * dx * dx + c1;
    K[1] += c2 * dy * dy + c1;
    K[2] += c2 * dz * dz + c1;
    K[3] += c2 * dx * dy;
    K[4] += c2 * dx * dz;
    K[5] += c2 * dy * dz;
  }
}

// y = K x for the symmetric 3x3 K
__device__ __forceinline__ void symmul(const double K[6], const double x[3], double y[3]) {
  y[0] = K[0] * x[0] + K[3] * x[1] + K[4] * x[2];
  y[1] = K[3] * x[0] + K[1] * x[1] + K[5] * x[2];
  y[2] = K[4] * x[0] + K[5] * x[1] + K[2] * x[2];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Monodromy matrix storage: element-major, lane-minor in LDS, one 18 KB
// slice per wavefront (workgroup = one wavefront), so that every ds access
// of a wavefront touches 64 consecutive doubles.
constexpr int kMonoElems = 36;  // row-major 6x6, rows (q, p), columns (q0, p0)

__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2, 2)))
propagate_f64_kernel(const Desc* __restrict__ descs, int n_prob, const double* __restrict__ field,
                     EnsPtrs e, double* __restrict__ accum, double* __restrict__ final_state,
                     uint64_t capacity) {
  __shared__ double mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  const uint32_t pack = blockIdx.x;
  if (pack >= e.pack_start[n_prob]) return;
  int lo = 0, hi = n_prob;  // pack_start[lo] <= pack < pack_start[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (e.pack_start[mid] <= pack) lo = mid; else hi = mid;
  }
  const Desc& d = descs[lo];
  const int N = d.N;
  const uint32_t pos = (pack - e.pack_start[lo]) * kWave + lane;
  const bool valid = pos < e.live_count[lo];
  const uint32_t slot = valid ? e.order[e.live_start[lo] + pos] : 0u;

  // initial conditions
  const int k0 = valid ? e.k0[slot] : N + 1;
  double q[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  double p[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double w = e.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  const double p0q0 = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < kMonoElems; ++i) mono[i][lane] = (i % 7 == 0) ? 1.0 : 0.0;
  // HK matrix R = 1/2 (Mqq + Mpp - i g Mqp + (i/g) Mpq) of the current M
  double Rr[3][3], Ri[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Rr[a][b] = a == b ? 1.0 : 0.0;
      Ri[a][b] = 0.0;
    }
  double Cre = 1.0, Cim = 0.0;
  double flips = 0.0;

  const double h = d.dt;
  const double* __restrict__ fe = field + d.field_off;
  double* __restrict__ acc = accum + d.acc_off;
  const int kmin = __builtin_amdgcn_readfirstlane(k0);
  double acc_reg = 0.0;

  for (int k = kmin;; ++k) {
    const bool live = k >= k0;
    double re_a = 0.0;
    if (live) {
      // --- HK prefactor C = sqrt(det R), continued branch
      const double c0r = Rr[1][1] * Rr[2][2] - Ri[1][1] * Ri[2][2] - (Rr[1][2] * Rr[2][1] - Ri[1][2] * Ri[2][1]);
      const double c0i = Rr[1][1] * Ri[2][2] + Ri[1][1] * Rr[2][2] - (Rr[1][2] * Ri[2][1] + Ri[1][2] * Rr[2][1]);
      const double c1r = Rr[1][0] * Rr[2][2] - Ri[1][0] * Ri[2][2] - (Rr[1][2] * Rr[2][0] - Ri[1][2] * Ri[2][0]);
      const double c1i = Rr[1][0] * Ri[2][2] + Ri[1][0] * Rr[2][2] - (Rr[1][2] * Ri[2][0] + Ri[1][2] * Rr[2][0]);
      const double c2r = Rr[1][0] * Rr[2][1] - Ri[1][0] * Ri[2][1] - (Rr[1][1] * Rr[2][0] - Ri[1][1] * Ri[2][0]);
      const double c2i = Rr[1][0] * Ri[2][1] + Ri[1][0] * Rr[2][1] - (Rr[1][1] * Ri[2][0] + Ri[1][1] * Rr[2][0]);
      const double Dr = (Rr[0][0] * c0r - Ri[0][0] * c0i) - (Rr[0][1] * c1r - Ri[0][1] * c1i) +
                        (Rr[0][2] * c2r - Ri[0][2] * c2i);
      const double Di = (Rr[0][0] * c0i + Ri[0][0] * c0r) - (Rr[0][1] * c1i + Ri[0][1] * c1r) +
                        (Rr[0][2] * c2i + Ri[0][2] * c2r);
      // principal square root: u = (|D| + |Dr|)/2, sqrt(u) and Di/(2 sqrt(u))
      // from one reciprocal square root each (|D| >= 1 for symplectic M)
      const double m2 = Dr * Dr + Di * Di;
      const double mag = m2 * rsqrt_nr(m2);
      const double u = 0.5 * (mag + fabs(Dr));
      const double ru = rsqrt_nr(u);
      const double big = u * ru, small = 0.5 * Di * ru;
      double sr, si;
      if (Dr >= 0.0) {
        sr = big;
        si = small;
      } else {
        sr = fabs(small);
        si = Di < 0.0 ? -big : big;
      }
      // continued branch: the root whose ratio to the previous C has Re >= 0;
      // arg(D_k / D_{k-1}) = 2 arg(C_k / C_{k-1}) leaves (-pi/2, pi/2] exactly
      // when |Im(C_k conj C_{k-1})| > Re(C_k conj C_{k-1})
      double xr = sr * Cre + si * Cim;
      const double xi = si * Cre - sr * Cim;
      if (xr < 0.0) {
        sr = -sr;
        si = -si;
        xr = -xr;
      }
      if (fabs(xi) > xr) flips += 1.0;
      Cre = sr;
      Cim = si;

      // --- recombination <psi0|k_z|p,q> (Gaussian moments of the GTO primitives)
      const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      const double np_ = n[0] * p[0] + n[1] * p[1] + n[2] * p[2];
      double dd[2], pd[2], nd[2], dz[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double s = c == 0 ? d.half_R : -d.half_R;
        const double x = s * n[0] - q[0], y = s * n[1] - q[1], z = s * n[2] - q[2];
        dd[c] = x * x + y * y + z * z;
        pd[c] = p[0] * x + p[1] * y + p[2] * z;
        nd[c] = n[0] * x + n[1] * y + n[2] * z;
        dz[c] = z;
      }
      const double bzr = p[2] * d.inv_gamma;
      const double bb_re_p = pp * d.inv_gamma2;
      // ln(1 + |C|) bound from the binary exponent of 1 + |C|^2
      const double cc = 1.0 + Cre * Cre + Cim * Cim;
      const double lnC = 0.3466 * (double)(((int)(__double_as_longlong(cc) >> 52) & 0x7ff) - 1022);
      double rr = 0.0, ri = 0.0;
      for (int j = 0; j < d.n_gto; ++j) {
        const int c = d.g_sgn[j] > 0.0 ? 0 : 1;
        const double ddc = c == 0 ? dd[0] : dd[1];
        const double pdc = c == 0 ? pd[0] : pd[1];
        const double dzc = c == 0 ? dz[0] : dz[1];
        const double i4 = d.g_inv4k[j], i2 = d.g_inv2k[j];
        const double er = (bb_re_p - ddc) * i4 - pp * d.half_inv_gamma;
        if (er + lnC < kRecombFar) continue;
        const double ei = 2.0 * pdc * d.inv_gamma * i4;
        const double gm = d.g_norm[j] * exp(er);
        double sn, cs;
        sincos(ei, &sn, &cs);
        const double Gr = gm * cs, Gi = gm * sn;
        double Xr, Xi;
        if (d.g_l[j] == 0) {
          Xr = bzr * i2;
          Xi = dzc * i2;
        } else {
          const double ndc = c == 0 ? nd[0] : nd[1];
          const double nbr = np_ * d.inv_gamma, nbi = ndc;
          // i/(2a) [n_z/(2k) + b_z (n.b)/(4k^2)]
          const double ur = n[2] * i2 + (bzr * nbr - dzc * nbi) * i2 * i2;
          const double ui = (bzr * nbi + dzc * nbr) * i2 * i2;
          Xr = -ui * d.g_i2a[j];
          Xi = ur * d.g_i2a[j];
        }
        rr += Gr * Xr - Gi * Xi;
        ri += Gr * Xi + Gi * Xr;
      }
      // --- amplitude a = -w C e^{i Phi} rho, Phi = S - Ip (t_k - t0) + p0.q0
      if (rr != 0.0 || ri != 0.0) {
        const double tk = d.t_first + (double)k * h;
        const double phi = S - d.Ip * (tk - t0) + p0q0;
        double sp, cp;
        sincos(phi, &sp, &cp);
        const double er_ = Cre * cp - Cim * sp, ei_ = Cre * sp + Cim * cp;
        re_a = -w * (er_ * rr - ei_ * ri);
      }
    }
    // wave sum of Re a; lane (k mod 64) keeps it, and every 64 steps the
    // wavefront adds its 64 sums to the accumulator in one coalesced atomic
    if (__ballot(re_a != 0.0)) {
      const double tot = wave_sum(re_a);
      if (lane == (k & (kWave - 1))) acc_reg += tot;
    }
    if ((k & (kWave - 1)) == kWave - 1 || k >= N) {
      if (acc_reg != 0.0) unsafeAtomicAdd(&acc[(k & ~(kWave - 1)) + lane], acc_reg);
      acc_reg = 0.0;
    }
    if (k >= N) break;
    if (!live) continue;

    // --- classical RK4 step t_k -> t_{k+1}
    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
    const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
    double K1[6], K2[6], K3[6], K4[6];
    double V, g[3];
    double sq[3], sp3[3], sS;  // RK4 weighted sums of the q, p and S slopes
    double yq[3], yp[3];

    potential(d, hRn, q, V, g, K1);
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
    potential(d, hRn, yq, V, g, K2);
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
    potential(d, hRn, yq, V, g, K3);
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
    potential(d, hRn, yq, V, g, K4);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - E1};
      const double kS = 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * E1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += yp[a];
        sp3[a] += kp[a];
        q[a] = q[a] + (h / 6.0) * sq[a];
        p[a] = p[a] + (h / 6.0) * sp3[a];
      }
      sS += kS;
      S = S + (h / 6.0) * sS;
    }
    // monodromy: each column (x, v) = (dq/dx0_c, dp/dx0_c) obeys x' = v,
    // v' = -K(q(t)) x with the stage Hessians K1..K4 of this RK4 step.
    // Columns c and c + 3 give column c of R.
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      __builtin_amdgcn_sched_barrier(0);
      const double x0[3] = {mono[c][lane], mono[6 + c][lane], mono[12 + c][lane]};
      const double v0[3] = {mono[18 + c][lane], mono[24 + c][lane], mono[30 + c][lane]};
      double a[3], xs[3], vs[3], sx[3], sv[3];
      symmul(K1, x0, a);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        sx[r] = v0[r];
        sv[r] = -a[r];
        xs[r] = x0[r] + 0.5 * h * v0[r];
        vs[r] = v0[r] + 0.5 * h * (-a[r]);
      }
      symmul(K2, xs, a);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double kx = vs[r];
        sx[r] += 2.0 * kx;
        sv[r] += 2.0 * (-a[r]);
        xs[r] = x0[r] + 0.5 * h * kx;
        vs[r] = v0[r] + 0.5 * h * (-a[r]);
      }
      symmul(K3, xs, a);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double kx = vs[r];
        sx[r] += 2.0 * kx;
        sv[r] += 2.0 * (-a[r]);
        xs[r] = x0[r] + h * kx;
        vs[r] = v0[r] + h * (-a[r]);
      }
      symmul(K4, xs, a);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        sx[r] += vs[r];
        sv[r] += -a[r];
        const double xn = x0[r] + (h / 6.0) * sx[r];
        const double vn = v0[r] + (h / 6.0) * sv[r];
        mono[6 * r + c][lane] = xn;
        mono[18 + 6 * r + c][lane] = vn;
        if (c < 3) {  // x = Mqq[:, c], v = Mpq[:, c]
          Rr[r][c] = 0.5 * xn;
          Ri[r][c] = 0.5 * d.inv_gamma * vn;
        } else {      // x = Mqp[:, c-3], v = Mpp[:, c-3]
          Rr[r][c - 3] += 0.5 * vn;
          Ri[r][c - 3] -= 0.5 * d.gamma * xn;
        }
      }
    }
  }

  if (final_state != nullptr && valid) {
    double* f = final_state + slot;
    const uint64_t st = capacity;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[(SFHK_FS_Q + a) * st] = q[a];
      f[(SFHK_FS_P + a) * st] = p[a];
    }
#pragma unroll
    for (int i = 0; i < kMonoElems; ++i) f[(SFHK_FS_M + i) * st] = mono[i][lane];
    f[SFHK_FS_S * st] = S;
    f[SFHK_FS_CRE * st] = Cre;
    f[SFHK_FS_CIM * st] = Cim;
    f[SFHK_FS_FLIPS * st] = flips;
  }
}

}  // namespace

hipError_t launch_propagate_f64(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                                uint32_t max_packs, double* accum, double* final_state,
                                uint64_t capacity, hipStream_t s) {
  if (max_packs == 0) return hipSuccess;
  hipLaunchKernelGGL(propagate_f64_kernel, dim3(max_packs), dim3(kWave), 0, s, descs, n_prob,
                     field, e, accum, final_state, capacity);
  return hipGetLastError();
}

}  // namespace sfhk
