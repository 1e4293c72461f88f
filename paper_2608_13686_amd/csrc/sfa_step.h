// Exact SFA ionisation step of the sampler (Sec. II.A, Eq. 1-2), one
// trajectory per lane.
//
// The pulse A(t) = -(E0/w) cos^2(pi t/tau) sin(w t + cep) is written as three
// carriers, A = -a0 sum_j c_j sin(w_j t + cep) with a0 = E0/w, c = (1/2, 1/4,
// 1/4), w_j = (w, w + W, w - W), W = 2 pi/tau, which continues it to complex
// time and gives closed antiderivatives of A and A^2.  On the path
// t = t0 + i s every carrier splits into real hyperbolic functions of w_j s,
// so the saddle point, the tunnel exit, the tunnelling action and the
// matrix element below are real arithmetic on cos/sin(w_j t0 + cep) and
// sinh/cosh(w_j t_t); cosh - 1 is taken as 2 sinh^2(x/2).
#pragma once

#include "sfhk_internal.h"

namespace sfhk {

struct SfaBirth {
  double kz;   // longitudinal momentum at birth (p0_z)
  double q0z;  // tunnel exit Re int_{t_s}^{t0} A dt
  double w;    // |m e^{i S}| over the k_perp proposal, in units of the
               // peak-field tunnelling factor e^{-kappa^3/(3 E0)}
  double dph;  // Re S - I_p t0 + arg m
};

// Principal square root of x + i y.
__device__ __forceinline__ void csqrt_principal(double x, double y, double& sr, double& si) {
  const double r = hypot(x, y);
  if (x >= 0.0) {
    const double s = sqrt(0.5 * (r + x));
    sr = s;
    si = s > 0.0 ? y / (2.0 * s) : 0.0;
  } else {
    const double s = sqrt(0.5 * (r - x));
    sr = fabs(y) / (2.0 * s);
    si = copysign(s, y);
  }
}

// Saddle point t_s = t0 + i t_t of [k + A(t_s) - A(t0)]^2/2 + I_p = 0 for
// real k: Im A(t0 + i t_t) = -sgn E(t0) sqrt(2 I_p + k_perp^2) fixes t_t (the
// smallest positive root: unit steps from 0 to 150 a.u. to the first
// crossing, then Newton steps kept inside the bracket), and
// k_z = A(t0) - Re A(t_s).  Then the tunnel exit, the action
//   S = I_p t_s - int_{t_s}^{t0} [k + A - A(t0)]^2 / 2 dt
// from the antiderivatives, and the amplitude
//   m = <kappa_s| z E(t_s) |psi_0> / sqrt(E(t_s) kappa_z),
// kappa_s = (k_perp, i Im A(t_s)), from the Gaussian integrals of the GTO
// primitives.  Returns false when there is no saddle point.
__device__ inline bool sfa_birth(const Desc& d, double t0, double kx, double ky,
                                 const double n[3], SfaBirth& o) {
  const double a0 = d.E0 / d.omega;
  const double Om = 2.0 * kPi / d.tau;
  const double wj[3] = {d.omega, d.omega + Om, d.omega - Om};
  const double cj[3] = {0.5, 0.25, 0.25};
  double Cj[3], Sj[3];
  double Et0 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    sincos(wj[j] * t0 + d.cep, &Sj[j], &Cj[j]);
    Et0 += cj[j] * wj[j] * Cj[j];
  }
  Et0 *= a0;
  // no birth where the field vanishes (the pulse ends, where E = 0 exactly)
  if (!(fabs(Et0) > 1e-12 * d.E0)) return false;
  const double kp2 = kx * kx + ky * ky;
  const double kap0 = sqrt(2.0 * d.Ip + kp2);
  const double sg = Et0 > 0.0 ? 1.0 : -1.0;
  // h(s) = sg a0 sum_j c_j C_j sinh(w_j s) - kap0, h(0) = -kap0 < 0
  auto h = [&](double s) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) v += cj[j] * Cj[j] * sinh(wj[j] * s);
    return sg * a0 * v - kap0;
  };
  auto dh = [&](double s) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) v += cj[j] * Cj[j] * wj[j] * cosh(wj[j] * s);
    return sg * a0 * v;
  };
  double lo = 0.0, hi = -1.0;
  for (int i = 1; i <= 150; ++i) {
    const double s = (double)i;
    if (h(s) >= 0.0) {
      hi = s;
      break;
    }
    lo = s;
  }
  if (hi < 0.0) return false;
  double tt = 0.5 * (lo + hi);
  for (int it = 0; it < 100; ++it) {
    const double f = h(tt);
    if (f >= 0.0) hi = tt;
    else lo = tt;
    double nx = tt - f / dh(tt);
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    if (nx == tt || hi - lo <= 1e-15 * hi) break;
    tt = nx;
  }

  // SFHK2: the modified equation (k_z + A(t_s) - A(t0))^2 + k_perp^2 + 2 I_p
  // + 2 sgn E(t0) D E(t_s) = 0, D = (R/2)|n_z| (the extra term -eta E(t_s).r0
  // with eta chosen so that it raises the binding energy), solved for
  // (t_t, k_z) by Newton steps with the analytic Jacobian, starting from the
  // unmodified root for I_p + |E(t0)| D.
  const bool modified = d.ionization == SFHK_ION_SADDLE_MODIFIED;
  const double Dm = modified ? d.half_R * fabs(n[2]) : 0.0;
  double kz_m = 0.0;
  if (modified) {
    const double kap1 = sqrt(2.0 * (d.Ip + fabs(Et0) * Dm) + kp2);
    auto h1 = [&](double s) { return h(s) + kap0 - kap1; };
    lo = 0.0;
    hi = -1.0;
    for (int i = 1; i <= 150; ++i) {
      const double s = (double)i;
      if (h1(s) >= 0.0) {
        hi = s;
        break;
      }
      lo = s;
    }
    if (hi < 0.0) return false;
    tt = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
      const double f = h1(tt);
      if (f >= 0.0) hi = tt;
      else lo = tt;
      double nx = tt - f / dh(tt);
      if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
      if (nx == tt || hi - lo <= 1e-15 * hi) break;
      tt = nx;
    }
    // k_z of the unmodified relation, then Newton on the complex equation
    kz_m = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double s2 = sinh(0.5 * wj[j] * tt);
      kz_m += cj[j] * Sj[j] * 2.0 * s2 * s2;
    }
    kz_m *= a0;
    bool conv = false;
    for (int it = 0; it < 40 && !conv; ++it) {
      // A(t_s) - A(t0), E(t_s), E'(t_s) on the path t0 + i tt
      double dAr = 0.0, dAi = 0.0, Er = 0.0, Ei = 0.0, Dr = 0.0, Di = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double x = wj[j] * tt;
        const double shx = sinh(x), s2 = sinh(0.5 * x), c1x = 2.0 * s2 * s2;
        dAr -= cj[j] * Sj[j] * c1x;
        dAi -= cj[j] * Cj[j] * shx;
        Er += cj[j] * wj[j] * Cj[j] * (1.0 + c1x);
        Ei -= cj[j] * wj[j] * Sj[j] * shx;
        Dr -= cj[j] * wj[j] * wj[j] * Sj[j] * (1.0 + c1x);
        Di -= cj[j] * wj[j] * wj[j] * Cj[j] * shx;
      }
      dAr *= a0; dAi *= a0; Er *= a0; Ei *= a0; Dr *= a0; Di *= a0;
      const double kr = kz_m + dAr, ki = dAi;                // kappa_z
      const double fr = kr * kr - ki * ki + kp2 + 2.0 * d.Ip + 2.0 * sg * Dm * Er;
      const double fi = 2.0 * kr * ki + 2.0 * sg * Dm * Ei;
      // df/dk_z = 2 kappa_z; df/dt_t = -2 i kappa_z E(t_s) + 2 i sgn D E'(t_s)
      const double gkr = 2.0 * kr, gki = 2.0 * ki;
      const double ptr = 2.0 * (kr * Ei + ki * Er) - 2.0 * sg * Dm * Di;
      const double pti = -2.0 * (kr * Er - ki * Ei) + 2.0 * sg * Dm * Dr;
      const double det = ptr * gki - gkr * pti;
      if (det == 0.0) return false;
      const double d0 = (-fr * gki + fi * gkr) / det;   // step in t_t
      const double d1 = (-fi * ptr + fr * pti) / det;   // step in k_z
      tt += d0;
      kz_m += d1;
      conv = fabs(d0) < 1e-13 * (1.0 + fabs(tt)) && fabs(d1) < 1e-13 * (1.0 + fabs(kz_m));
    }
    if (!conv || !(tt > 0.0)) return false;
  }

  double sh[3], ch1[3], chh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double x = wj[j] * tt;
    sh[j] = sinh(x);
    const double s2 = sinh(0.5 * x);
    ch1[j] = 2.0 * s2 * s2;  // cosh(x) - 1
    chh[j] = 1.0 + ch1[j];
  }
  double kz = 0.0, q0z = 0.0, At0 = 0.0, ImAs = 0.0, Esr = 0.0, Esi = 0.0;
  double dAr_s = 0.0;  // Re A(t_s) - A(t0)
  double dFr = 0.0, dFi = 0.0;  // F(t0) - F(t_s), F = int A dt
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    kz += cj[j] * Sj[j] * ch1[j];
    dAr_s -= cj[j] * Sj[j] * ch1[j];
    q0z -= cj[j] / wj[j] * Cj[j] * ch1[j];
    At0 -= cj[j] * Sj[j];
    ImAs -= cj[j] * Cj[j] * sh[j];
    Esr += cj[j] * wj[j] * Cj[j] * chh[j];
    Esi -= cj[j] * wj[j] * Sj[j] * sh[j];
    dFr -= cj[j] / wj[j] * Cj[j] * ch1[j];
    dFi += cj[j] / wj[j] * Sj[j] * sh[j];
  }
  kz *= a0;
  dAr_s *= a0;
  if (modified) kz = kz_m;
  q0z *= a0;
  At0 *= a0;
  ImAs *= a0;
  Esr *= a0;
  Esi *= a0;
  dFr *= a0;
  dFi *= a0;
  // G(t0) - G(t_s), G = int A^2 dt = a0^2/2 sum_ij c_i c_j [D_ij(t) -
  // sin((w_i + w_j) t + 2 cep)/(w_i + w_j)], D_ii = t, D_ij = sin((w_i - w_j) t)/(w_i - w_j)
  double dGr = 0.0, dGi = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double wt = (i == j ? 1.0 : 2.0) * cj[i] * cj[j];
      double Dr, Di;
      if (i == j) {
        Dr = 0.0;
        Di = -tt;
      } else {
        const double del = wj[i] - wj[j];
        double sd, cd;
        sincos(del * t0, &sd, &cd);
        const double s2 = sinh(0.5 * del * tt);
        Dr = -sd * 2.0 * s2 * s2 / del;
        Di = -cd * sinh(del * tt) / del;
      }
      const double sig = wj[i] + wj[j];
      double sp, cp;
      sincos(sig * t0 + 2.0 * d.cep, &sp, &cp);
      const double s2 = sinh(0.5 * sig * tt);
      const double Qr = -sp * 2.0 * s2 * s2 / sig;
      const double Qi = -cp * sinh(sig * tt) / sig;
      dGr += wt * (Dr - Qr);
      dGi += wt * (Di - Qi);
    }
  dGr *= 0.5 * a0 * a0;
  dGi *= 0.5 * a0 * a0;
  // int_{t_s}^{t0} kappa^2/2 dt = 1/2 [(k_perp^2 + c^2)(-i t_t) + 2 c dF + dG], c = k_z - A(t0)
  const double c = kz - At0;
  const double Tr = 0.5 * (2.0 * c * dFr + dGr);
  const double Ti = 0.5 * (-(kp2 + c * c) * tt + 2.0 * c * dFi + dGi);
  double ImS = d.Ip * tt - Ti;
  double ReS_minus = -Tr;  // Re S - I_p t0
  // kappa_z(t_s) = k_z + A(t_s) - A(t0): purely imaginary on the unmodified
  // saddle point, complex on the modified one
  const double kzr = modified ? kz + dAr_s : 0.0, kzi = ImAs;
  if (modified) {  // SFHK2 action term eta r0_z (A(t_s) - A(t0)), eta r0_z = -sgn D
    ReS_minus -= sg * Dm * dAr_s;
    ImS -= sg * Dm * ImAs;
  }

  // matrix element at kappa = (kx, ky, kzr + i kzi)
  const double k2r = kp2 + kzr * kzr - kzi * kzi, k2i = 2.0 * kzr * kzi;  // kappa.kappa
  double mr = 0.0, mi = 0.0;
  for (int j = 0; j < d.n_gto; ++j) {
    const double sgn = (d.g_l[j] & 2) ? -1.0 : 1.0;
    const double Rx = sgn * d.half_R * n[0], Ry = sgn * d.half_R * n[1],
                 Rz = sgn * d.half_R * n[2];
    const double i2a = d.g_i2a[j];
    // G = c (2a)^{-3/2} exp(-kappa^2/(4a) - i kappa.R)
    const double Er = -0.5 * k2r * i2a + kzi * Rz;
    const double Ei = -0.5 * k2i * i2a - (kx * Rx + ky * Ry + kzr * Rz);
    double se, ce;
    sincos(Ei, &se, &ce);
    const double gm = d.g_ion[j] * exp(Er);
    const double Gr = gm * ce, Gi = gm * se;
    double fr, fi;
    if ((d.g_l[j] & 1) == 0) {  // Rz - i kappa_z/(2a)
      fr = Rz + kzi * i2a;
      fi = -kzr * i2a;
    } else {  // -i Rz (n.kappa)/(2a) + n_z/(2a) - (n.kappa) kappa_z/(4a^2)
      const double nkr = n[0] * kx + n[1] * ky + n[2] * kzr, nki = n[2] * kzi;
      fr = Rz * i2a * nki + n[2] * i2a - (nkr * kzr - nki * kzi) * i2a * i2a;
      fi = -Rz * i2a * nkr - (nkr * kzi + nki * kzr) * i2a * i2a;
    }
    mr += Gr * fr - Gi * fi;
    mi += Gr * fi + Gi * fr;
  }
  // times E(t_s), over sqrt(E(t_s) kappa_z)
  const double er = mr * Esr - mi * Esi, ei = mr * Esi + mi * Esr;
  double qr, qi;
  csqrt_principal(Esr * kzr - Esi * kzi, Esr * kzi + Esi * kzr, qr, qi);
  const double q2 = qr * qr + qi * qi;
  const double m_r = (er * qr + ei * qi) / q2, m_i = (ei * qr - er * qi) / q2;
  const double am = hypot(m_r, m_i);
  if (!(am > 0.0)) return false;
  o.kz = kz;
  o.q0z = q0z;
  const double comp = d.sigma > 0.0 ? kp2 / (2.0 * d.sigma * d.sigma) : 0.0;
  o.w = am * exp(-ImS + d.kcube3 * d.inv_E0 + comp);
  o.dph = ReS_minus + atan2(m_i, m_r);
  return true;
}

}  // namespace sfhk
