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
    const double rho = sqrt(r2);
    const double inv = 1.0 / rho;
    double Z = d.Zinf[c], f1, f2;
    if (d.screened) {
      const double ex = exp(-d.alpha[c] * rho);
      const double adx = d.alpha[c] * d.dZ[c] * ex;
      Z += d.dZ[c] * ex;
      f1 = (Z * inv + adx) * inv;
      f2 = -(2.0 * Z * inv * inv + 2.0 * adx * inv + d.alpha[c] * adx) * inv;
    } else {
      f1 = Z * inv * inv;
      f2 = -2.0 * Z * inv * inv * inv;
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

__global__ void __launch_bounds__(kWave)
propagate_f64_kernel(const Desc* __restrict__ descs, int n_prob, const double* __restrict__ field,
                     EnsPtrs e, double* __restrict__ accum, double* __restrict__ final_state,
                     uint64_t capacity) {
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
  const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
  const double t0 = d.t_first + (double)k0 * d.dt;
  const double p0q0 = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
  double S = 0.0;
  // monodromy columns: mq[r][c] = dq_r/dx0_c, mp[r][c] = dp_r/dx0_c
  double mq[3][6], mp[3][6];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      mq[r][c] = (c == r) ? 1.0 : 0.0;
      mp[r][c] = (c == r + 3) ? 1.0 : 0.0;
    }
  double Cre = 1.0, Cim = 0.0, Dre_prev = 1.0, Dim_prev = 0.0;
  double flips = 0.0;

  const double h = d.dt;
  const double* __restrict__ fe = field + d.field_off;
  double* __restrict__ acc = accum + d.acc_off;
  const int kmin = __builtin_amdgcn_readfirstlane(k0);

  for (int k = kmin;; ++k) {
    const bool live = k >= k0;
    double re_a = 0.0;
    if (live) {
      // --- HK prefactor: R = 1/2 (Mqq + Mpp - i g Mqp + (i/g) Mpq), C = sqrt(det R)
      double Rr[3][3], Ri[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          Rr[a][b] = 0.5 * (mq[a][b] + mp[a][3 + b]);
          Ri[a][b] = 0.5 * (d.inv_gamma * mp[a][b] - d.gamma * mq[a][3 + b]);
        }
      // cofactors of row 0
      double c0r = Rr[1][1] * Rr[2][2] - Ri[1][1] * Ri[2][2] - (Rr[1][2] * Rr[2][1] - Ri[1][2] * Ri[2][1]);
      double c0i = Rr[1][1] * Ri[2][2] + Ri[1][1] * Rr[2][2] - (Rr[1][2] * Ri[2][1] + Ri[1][2] * Rr[2][1]);
      double c1r = Rr[1][0] * Rr[2][2] - Ri[1][0] * Ri[2][2] - (Rr[1][2] * Rr[2][0] - Ri[1][2] * Ri[2][0]);
      double c1i = Rr[1][0] * Ri[2][2] + Ri[1][0] * Rr[2][2] - (Rr[1][2] * Ri[2][0] + Ri[1][2] * Rr[2][0]);
      double c2r = Rr[1][0] * Rr[2][1] - Ri[1][0] * Ri[2][1] - (Rr[1][1] * Rr[2][0] - Ri[1][1] * Ri[2][0]);
      double c2i = Rr[1][0] * Ri[2][1] + Ri[1][0] * Rr[2][1] - (Rr[1][1] * Ri[2][0] + Ri[1][1] * Rr[2][0]);
      const double Dr = (Rr[0][0] * c0r - Ri[0][0] * c0i) - (Rr[0][1] * c1r - Ri[0][1] * c1i) +
                        (Rr[0][2] * c2r - Ri[0][2] * c2i);
      const double Di = (Rr[0][0] * c0i + Ri[0][0] * c0r) - (Rr[0][1] * c1i + Ri[0][1] * c1r) +
                        (Rr[0][2] * c2i + Ri[0][2] * c2r);
      // principal square root, then the branch closest to the previous C
      const double mag = sqrt(Dr * Dr + Di * Di);
      double sr, si;
      if (Dr >= 0.0) {
        sr = sqrt(0.5 * (mag + Dr));
        si = sr > 0.0 ? Di / (2.0 * sr) : 0.0;
      } else {
        si = sqrt(0.5 * (mag - Dr));
        if (Di < 0.0) si = -si;
        sr = Di / (2.0 * si);
      }
      if (sr * Cre + si * Cim < 0.0) {
        sr = -sr;
        si = -si;
      }
      if (Dr * Dre_prev + Di * Dim_prev < 0.0) flips += 1.0;
      Cre = sr;
      Cim = si;
      Dre_prev = Dr;
      Dim_prev = Di;

      // --- recombination <psi0|k_z|p,q> (Gaussian moments of the GTO primitives)
      const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      const double np_ = n[0] * p[0] + n[1] * p[1] + n[2] * p[2];
      double dd[2], pd[2], nd[2], dz[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double s = c == 0 ? 1.0 : -1.0;
        const double x = s * hRn[0] - q[0], y = s * hRn[1] - q[1], z = s * hRn[2] - q[2];
        dd[c] = x * x + y * y + z * z;
        pd[c] = p[0] * x + p[1] * y + p[2] * z;
        nd[c] = n[0] * x + n[1] * y + n[2] * z;
        dz[c] = z;
      }
      const double bzr = p[2] * d.inv_gamma;
      const double bb_re_p = pp * d.inv_gamma2;
      double rr = 0.0, ri = 0.0;
      for (int j = 0; j < d.n_gto; ++j) {
        const int c = d.g_sgn[j] > 0.0 ? 0 : 1;
        const double ddc = c == 0 ? dd[0] : dd[1];
        const double pdc = c == 0 ? pd[0] : pd[1];
        const double dzc = c == 0 ? dz[0] : dz[1];
        const double i4 = d.g_inv4k[j], i2 = d.g_inv2k[j];
        const double er = (bb_re_p - ddc) * i4 - pp * d.half_inv_gamma;
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
      const double tk = d.t_first + (double)k * h;
      const double phi = S - d.Ip * (tk - t0) + p0q0;
      double sp, cp;
      sincos(phi, &sp, &cp);
      const double er_ = Cre * cp - Cim * sp, ei_ = Cre * sp + Cim * cp;
      re_a = -w * (er_ * rr - ei_ * ri);
    }
    const double tot = wave_sum(re_a);
    if (lane == 0) unsafeAtomicAdd(&acc[k], tot);
    if (k >= N) break;
    if (!live) continue;

    // --- classical RK4 step t_k -> t_{k+1}
    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
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
    // monodromy: each column (mq, mp) obeys d mq/dt = mp, d mp/dt = -K(q(t)) mq
    // with the stage Hessians K1..K4 of the same RK4 step
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double x0[3] = {mq[0][c], mq[1][c], mq[2][c]};
      const double v0[3] = {mp[0][c], mp[1][c], mp[2][c]};
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
        mq[r][c] = x0[r] + (h / 6.0) * sx[r];
        mp[r][c] = v0[r] + (h / 6.0) * sv[r];
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
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        f[(SFHK_FS_M + 6 * r + c) * st] = mq[r][c];
        f[(SFHK_FS_M + 6 * (3 + r) + c) * st] = mp[r][c];
      }
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
