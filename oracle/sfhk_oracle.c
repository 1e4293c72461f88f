/*
 * SFHK oracle -- plain scalar FP64 implementation of the strong-field
 * Herman-Kluk estimator of the molecular dipole velocity (arXiv 2608.13686).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  No code,
 * header or table is shared with the HIP implementation.
 *
 * Every function follows one passage of the paper and is written for
 * reading, not speed: the full 43-component state is stepped by textbook
 * RK4, the monodromy derivative is a plain 6x6 matrix product, complex
 * arithmetic is C99 <complex.h>, and the transcendental functions are libm.
 * Where the paper is silent the reading used is stated next to the code.
 *
 * Parity unpinned: the overall sign of the amplitude (the minus sign of the
 * dipole formula of Sec. II.A), to which every computed observable (spectra,
 * yields, Gabor maps) is blind, and the synthetic GTO tables, which stand in
 * for the paper's fitted orbitals.
 */
#include "sfhk_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
/* hc in hartree*nm (hc = 1239.84198 eV nm, E_h = 27.211386245988 eV) */
#define ORC_HC_HARTREE_NM 45.56335252912
/* atomic unit of intensity 0.5 eps0 c E_au^2 in W/cm^2 */
#define ORC_I_AU_WCM2 3.50944552058977e16

/* ------------------------------------------------------------------ laser */
/* Linearly z-polarised pulse with a sin^2 envelope of n_cycles optical
 * cycles and carrier-envelope phase cep (Sec. II.D and III.A give the
 * envelope, cycles and CEP but not the formula).  Reading: the pulse is
 * centred at t = 0, A(t) = -(E0/w) cos^2(pi t/tau) sin(w t + cep) for
 * |t| <= tau/2 and 0 outside, and E = -dA/dt, so that A vanishes at both
 * ends and the field has no DC component. */
void orc_laser(const orc_problem* P, double* omega, double* E0, double* tau, int32_t* N) {
  double w = ORC_HC_HARTREE_NM / P->lambda_nm;
  double e0 = sqrt(P->intensity_wcm2 / ORC_I_AU_WCM2);
  double T = P->n_cycles * 2.0 * ORC_PI / w;
  if (omega) *omega = w;
  if (E0) *E0 = e0;
  if (tau) *tau = T;
  if (N) *N = P->n_steps > 0 ? P->n_steps : (int32_t)lround(T / P->dt);
}

/* The step grid of the same reading: t_k = -tau/2 + k dt, k = 0..N. */
double orc_time(const orc_problem* P, int32_t k) {
  double tau;
  orc_laser(P, NULL, NULL, &tau, NULL);
  return -0.5 * tau + (double)k * P->dt;
}

void orc_field(const orc_problem* P, double t, double* E, double* A) {
  double w, e0, tau;
  orc_laser(P, &w, &e0, &tau, NULL);
  if (fabs(t) > 0.5 * tau) {
    if (E) *E = 0.0;
    if (A) *A = 0.0;
    return;
  }
  double env = cos(ORC_PI * t / tau);
  double ph = w * t + P->cep;
  if (A) *A = -(e0 / w) * env * env * sin(ph);
  /* E = -dA/dt */
  if (E)
    *E = e0 * env * env * cos(ph) - (e0 * ORC_PI / (w * tau)) * sin(2.0 * ORC_PI * t / tau) * sin(ph);
}

/* -------------------------------------------------------------- potential */
/* Two-centre single-active-electron potential, Eq. (7) with Table I
 * parameters: each centre contributes -[Z_inf + (Z_0 - Z_inf) e^{-alpha r}]/r
 * with r the distance to the centre.  Reading: the distance is softened,
 * r -> rho = sqrt(|q - R_i|^2 + eps^2), in every occurrence (eps^2 = 0 is
 * Eq. (7) itself; dZ = 0 gives the soft-core form).  Centre 0 sits at
 * +R/2 n and centre 1 at -R/2 n for the molecular axis n (Sec. II.C). */
void orc_potential(const orc_problem* P, const double n[3], const double q[3], double* V,
                   double grad[3], double hess[9]) {
  double v = 0.0;
  double g[3] = {0.0, 0.0, 0.0};
  double h[9] = {0.0};
  for (int i = 0; i < 2; ++i) {
    double sgn = (i == 0) ? 1.0 : -1.0;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = q[a] - sgn * 0.5 * P->R * n[a];
    double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + P->eps2[i]);
    double ex = exp(-P->alpha[i] * rho);
    double Z = P->Zinf[i] + P->dZ[i] * ex;
    /* f(rho) = -Z(rho)/rho and its first two derivatives in rho */
    double f = -Z / rho;
    double f1 = Z / (rho * rho) + P->alpha[i] * P->dZ[i] * ex / rho;
    double f2 = -2.0 * Z / (rho * rho * rho) - 2.0 * P->alpha[i] * P->dZ[i] * ex / (rho * rho) -
                P->alpha[i] * P->alpha[i] * P->dZ[i] * ex / rho;
    v += f;
    for (int a = 0; a < 3; ++a) g[a] += f1 * d[a] / rho;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        h[3 * a + b] += (f2 - f1 / rho) * d[a] * d[b] / (rho * rho) + (a == b ? f1 / rho : 0.0);
  }
  if (V) *V = v;
  if (grad) memcpy(grad, g, sizeof g);
  if (hess) memcpy(hess, h, sizeof h);
}

/* ---------------------------------------------------------- recombination */
/* <psi_0 | k_z | p, q> with psi_0 a sum of GTO primitives (Sec. II.A) and
 * the coherent state <x|p,q> = (gamma/pi)^{3/4} exp[-gamma/2 |x-q|^2 +
 * i p.(x-q)], whose momentum form is (pi gamma)^{-3/4} exp[-|k-p|^2/(2 gamma)
 * - i k.q] (fixed width gamma, Sec. II.A).  Each primitive's Fourier
 * transform is Gaussian, so the momentum integral int d^3k phi~*(k) k_z
 * <k|p,q> is a Gaussian moment:
 *   s primitive c e^{-a|x-Ra|^2}:  phi~* = c (2a)^{-3/2} e^{-k^2/4a + i k.Ra}
 *   p primitive c n.(x-Ra) e^{-a|x-Ra|^2}: phi~* gains the factor i n.k/(2a)
 * With kappa2 = 1/(4a) + 1/(2 gamma), b = p/gamma + i (Ra - q):
 *   int d^3k k_z e^{-kappa2 k^2 + b.k} = (pi/kappa2)^{3/2} b_z/(2 kappa2) e^{b.b/(4 kappa2)}
 * and the p-type moment is its derivative along n with respect to b. */
void orc_recombination(const orc_problem* P, const double n[3], const double p[3],
                       const double q[3], double* re, double* im) {
  double complex rho = 0.0;
  double g = P->gamma;
  double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  for (int j = 0; j < P->n_gto; ++j) {
    double a = P->gto_a[j];
    double sgn = (P->gto_center[j] == 0) ? 1.0 : -1.0;
    double kap = 1.0 / (4.0 * a) + 1.0 / (2.0 * g);
    double complex b[3];
    for (int c = 0; c < 3; ++c) b[c] = p[c] / g + I * (sgn * 0.5 * P->R * n[c] - q[c]);
    double complex bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double complex G = P->gto_c[j] * pow(2.0 * a, -1.5) * pow(ORC_PI * g, -0.75) *
                       pow(ORC_PI / kap, 1.5) * cexp(bb / (4.0 * kap) - pp / (2.0 * g));
    if (P->gto_l[j] == 0) {
      rho += G * b[2] / (2.0 * kap);
    } else {
      double complex nb = n[0] * b[0] + n[1] * b[1] + n[2] * b[2];
      rho += G * (I / (2.0 * a)) * (n[2] / (2.0 * kap) + b[2] * nb / (4.0 * kap * kap));
    }
  }
  *re = creal(rho);
  *im = cimag(rho);
}

/* -------------------------------------------------------------- prefactor */
/* Herman-Kluk prefactor (Sec. II.A; its explicit form is deferred to an
 * earlier paper).  Reading: the standard HK form for the coherent-state
 * convention above, C = sqrt(det R) with
 *   R = 1/2 (M_qq + M_pp - i gamma M_qp + (i/gamma) M_pq),
 * M_xy = d x_t / d y_0 the blocks of the monodromy matrix. */
static double complex det3(double complex m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

static double complex hk_det(const double M[36], double g) {
  double complex R[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double Mqq = M[6 * a + b], Mqp = M[6 * a + 3 + b];
      double Mpq = M[6 * (3 + a) + b], Mpp = M[6 * (3 + a) + 3 + b];
      R[a][b] = 0.5 * (Mqq + Mpp - I * g * Mqp + (I / g) * Mpq);
    }
  return det3(R);
}

void orc_prefactor_det(const double M[36], double gamma, double* re, double* im) {
  double complex d = hk_det(M, gamma);
  *re = creal(d);
  *im = cimag(d);
}

/* ------------------------------------------------- SFA ionisation step */
/* The laser continued to complex time: the inside-pulse formula of the
 * laser reading above, A(t) = -(E0/w) cos^2(pi t/tau) sin(w t + cep) and
 * E = -dA/dt, evaluated for complex t (the saddle point t_s = t0 + i t_t of
 * Eq. (2) has its real part inside the pulse). */
static double complex vecpot_c(const orc_problem* P, double complex t) {
  double w, e0, tau;
  orc_laser(P, &w, &e0, &tau, NULL);
  double complex env = ccos(ORC_PI * t / tau);
  return -(e0 / w) * env * env * csin(w * t + P->cep);
}

static double complex field_c(const orc_problem* P, double complex t) {
  double w, e0, tau;
  orc_laser(P, &w, &e0, &tau, NULL);
  double complex env = ccos(ORC_PI * t / tau);
  double complex ph = w * t + P->cep;
  return e0 * env * env * ccos(ph) -
         (e0 * ORC_PI / (w * tau)) * csin(2.0 * ORC_PI * t / tau) * csin(ph);
}

void orc_field_complex(const orc_problem* P, double tr, double ti, double* A_re, double* A_im,
                       double* E_re, double* E_im) {
  double complex t = tr + I * ti;
  double complex A = vecpot_c(P, t), E = field_c(P, t);
  if (A_re) *A_re = creal(A);
  if (A_im) *A_im = cimag(A);
  if (E_re) *E_re = creal(E);
  if (E_im) *E_im = cimag(E);
}

/* Legendre polynomial P_n(z) and its derivative, by the three-term recurrence */
static void legendre(int n, double z, double* p, double* dp) {
  double p0 = 1.0, p1 = z;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  *dp = n * (z * p1 - p0) / (z * z - 1.0);
}

/* 16-point Gauss-Legendre nodes (roots of P_16, by Newton's method) and
 * weights 2 / ((1 - z^2) P_16'(z)^2) on [-1, 1] */
static void gauss_legendre16(double x[16], double wt[16]) {
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, &p, &dp);
      double dz = p / dp;
      z -= dz;
      if (fabs(dz) < 1e-15) break;
    }
    legendre(n, z, &p, &dp);
    x[i] = z;
    wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Saddle point of Eq. (2) for birth time t0 = Re t_s and transverse momentum
 * k_perp: [k + A(t_s) - A(t0)]^2 / 2 + I_p = 0 with k real.  Writing
 * kappa_z(t) = k_z + A(t) - A(t0), the equation is
 * kappa_z(t_s) = -/+ i sqrt(2 I_p + k_perp^2), i.e. two real conditions:
 *   Im A(t0 + i t_t) = -sgn E(t0) sqrt(2 I_p + k_perp^2)   (fixes t_t > 0),
 *   k_z = A(t0) - Re A(t0 + i t_t)                           (fixes k_z).
 * Reading: the root with the smallest t_t > 0 (the saddle point closest to
 * the real axis), found by stepping t_t by 1 a.u. from 0 up to 150 a.u. to
 * the first crossing, then bisection.  No crossing, or a vanishing field at
 * t0: no saddle point.
 *
 * Then (Sec. II.A):
 *   tunnel exit q0 = Re int_{t_s}^{t0} A dt (along z),
 *   S_down^0 = I_p t_s - int_{t_s}^{t0} [k + A(t) - A(t0)]^2 / 2 dt,
 * both integrals along the straight path t = t0 + i s, s from t_t to 0, by
 * composite 16-point Gauss-Legendre quadrature on panels no wider than
 * 0.5 a.u.; and the ionisation matrix element of Eq. (1)
 *   m = <kappa_s| z E(t_s) |psi_0> / sqrt(E(t_s) kappa_z(t_s)),
 * kappa_s = k + A(t_s) - A(t0) complex.  Reading: <kappa| is the plane wave
 * (2 pi)^{-3/2} e^{i kappa.x} continued analytically in kappa (no complex
 * conjugation of the complex part, as for real momenta), the square root is
 * the principal one, and psi_0 is the GTO sum of the recombination element.
 * For a primitive c e^{-a|x-Ra|^2} (times n.(x-Ra) for p) the Gaussian
 * integral gives, with kappa^2 = kappa.kappa and
 * G = c (2a)^{-3/2} e^{-kappa^2/(4a) - i kappa.Ra}:
 *   s:  G (Ra_z - i kappa_z/(2a))
 *   p:  G (-i Ra_z n.kappa/(2a) + n_z/(2a) - n.kappa kappa_z/(4a^2)). */
int orc_sfa_step(const orc_problem* P, double t0, const double kperp[2], const double n[3],
                 double out[7]) {
  double E0r, A0r, Epk;
  orc_field(P, t0, &E0r, &A0r);
  orc_laser(P, NULL, &Epk, NULL, NULL);
  for (int i = 0; i < 7; ++i) out[i] = 0.0;
  /* Reading: no birth where the field vanishes (|E(t0)| <= 1e-12 E0, e.g. at
   * the pulse ends, where E = 0 exactly and rounding would pick the sign that
   * selects the saddle point) */
  if (!(fabs(E0r) > 1e-12 * Epk)) return -1;
  double kp2 = kperp[0] * kperp[0] + kperp[1] * kperp[1];
  double kap0 = sqrt(2.0 * P->Ip + kp2);
  double sg = E0r > 0.0 ? 1.0 : -1.0;
  /* h(s) = -sgn E(t0) Im A(t0 + i s) - kap0 starts at -kap0 < 0 */
  double lo = 0.0, hi = -1.0;
  for (int i = 1; i <= 150; ++i) {
    double s = (double)i;
    double h = -sg * cimag(vecpot_c(P, t0 + I * s)) - kap0;
    if (h >= 0.0) {
      hi = s;
      break;
    }
    lo = s;
  }
  if (hi < 0.0) return -1;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double h = -sg * cimag(vecpot_c(P, t0 + I * mid)) - kap0;
    if (h >= 0.0) hi = mid;
    else lo = mid;
  }
  double tt = 0.5 * (lo + hi);
  double complex ts = t0 + I * tt;
  double complex As = vecpot_c(P, ts);
  double kz = A0r - creal(As);

  /* SFHK2 (Sec. III.C, modified saddle-point equation): an extra term
   * -eta E(t_s).r0 with r0 = R/2.  Reading: eta is the sign for which the
   * term raises the effective binding energy, as the paper states it does,
   * so -eta E(t_s).r0 = sgn E(t0) E(t_s) D with D = (R/2)|n_z| (zero at 90
   * degrees, largest at 0); the tunnelling action gains eta r0.(A(t_s) -
   * A(t0)), the term whose stationarity in t_s gives the extra term.  The
   * saddle point is the root (t_t, k_z) of the complex equation
   *   (k_z + A(t_s) - A(t0))^2 + k_perp^2 + 2 I_p + 2 sgn E(t0) D E(t_s) = 0
   * reached by Newton steps on the two real unknowns (finite-difference
   * Jacobian) from the unmodified root for I_p + |E(t0)| D. */
  double Dm = 0.0;
  if (P->ionization == ORC_ION_SADDLE_MODIFIED) {
    Dm = 0.5 * P->R * fabs(n[2]);
    double kap1 = sqrt(2.0 * (P->Ip + fabs(E0r) * Dm) + kp2);
    lo = 0.0;
    hi = -1.0;
    for (int i = 1; i <= 150; ++i) {
      double s = (double)i;
      double h = -sg * cimag(vecpot_c(P, t0 + I * s)) - kap1;
      if (h >= 0.0) {
        hi = s;
        break;
      }
      lo = s;
    }
    if (hi < 0.0) return -1;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      double h = -sg * cimag(vecpot_c(P, t0 + I * mid)) - kap1;
      if (h >= 0.0) hi = mid;
      else lo = mid;
    }
    tt = 0.5 * (lo + hi);
    kz = A0r - creal(vecpot_c(P, t0 + I * tt));
    int converged = 0;
    for (int it = 0; it < 60 && !converged; ++it) {
      double x[2] = {tt, kz};
      double complex f0 = 0.0, fd[2];
      for (int v = 0; v < 3; ++v) {
        double xx[2] = {x[0], x[1]};
        double hstep = 1e-7 * (1.0 + fabs(x[v == 2 ? 1 : 0]));
        if (v > 0) xx[v - 1] += hstep;
        double complex t = t0 + I * xx[0];
        double complex kzt = xx[1] + vecpot_c(P, t) - A0r;
        double complex f = kzt * kzt + kp2 + 2.0 * P->Ip + 2.0 * sg * Dm * field_c(P, t);
        if (v == 0) f0 = f;
        else fd[v - 1] = (f - f0) / hstep;
      }
      /* solve [Re fd0 Re fd1; Im fd0 Im fd1] d = -(Re f0, Im f0) */
      double a11 = creal(fd[0]), a12 = creal(fd[1]), a21 = cimag(fd[0]), a22 = cimag(fd[1]);
      double det = a11 * a22 - a12 * a21;
      if (det == 0.0) return -1;
      double d0 = (-creal(f0) * a22 + cimag(f0) * a12) / det;
      double d1 = (-cimag(f0) * a11 + creal(f0) * a21) / det;
      tt += d0;
      kz += d1;
      if (fabs(d0) < 1e-13 * (1.0 + fabs(tt)) && fabs(d1) < 1e-13 * (1.0 + fabs(kz)))
        converged = 1;
    }
    if (!converged || !(tt > 0.0)) return -1;
    ts = t0 + I * tt;
    As = vecpot_c(P, ts);
  }

  /* integrals from t_s to t0 along t = t0 + i s: int_{t_s}^{t0} f dt =
   * -i int_0^{t_t} f(t0 + i s) ds */
  double gx[16], gw[16];
  gauss_legendre16(gx, gw);
  int panels = (int)ceil(tt / 0.5);
  if (panels < 1) panels = 1;
  double width = tt / panels;
  double complex intA = 0.0, intK2 = 0.0;
  for (int pnl = 0; pnl < panels; ++pnl) {
    double a = pnl * width;
    for (int j = 0; j < 16; ++j) {
      double s = a + 0.5 * width * (gx[j] + 1.0);
      double complex A = vecpot_c(P, t0 + I * s);
      double complex kz_t = kz + A - A0r;
      intA += 0.5 * width * gw[j] * A;
      intK2 += 0.5 * width * gw[j] * (kp2 + kz_t * kz_t);
    }
  }
  intA *= -I;
  intK2 *= -I;
  double q0z = creal(intA);
  double complex S = P->Ip * ts - 0.5 * intK2;
  /* SFHK2: eta r0_z (A(t_s) - A(t0)) with eta r0_z = -sgn E(t0) D */
  S += -sg * Dm * (As - A0r);

  /* matrix element and its denominator */
  double complex Es = field_c(P, ts);
  double complex kzs = kz + As - A0r;
  double complex kap[3] = {kperp[0], kperp[1], kzs};
  double complex k2 = kap[0] * kap[0] + kap[1] * kap[1] + kap[2] * kap[2];
  double complex nk = n[0] * kap[0] + n[1] * kap[1] + n[2] * kap[2];
  double complex me = 0.0;
  for (int j = 0; j < P->n_gto; ++j) {
    double a = P->gto_a[j];
    double sgn = (P->gto_center[j] == 0) ? 1.0 : -1.0;
    double Ra[3] = {sgn * 0.5 * P->R * n[0], sgn * 0.5 * P->R * n[1], sgn * 0.5 * P->R * n[2]};
    double complex kR = kap[0] * Ra[0] + kap[1] * Ra[1] + kap[2] * Ra[2];
    double complex G = P->gto_c[j] * pow(2.0 * a, -1.5) * cexp(-k2 / (4.0 * a) - I * kR);
    if (P->gto_l[j] == 0)
      me += G * (Ra[2] - I * kzs / (2.0 * a));
    else
      me += G * (-I * Ra[2] * nk / (2.0 * a) + n[2] / (2.0 * a) - nk * kzs / (4.0 * a * a));
  }
  me *= Es;
  double complex m = me / csqrt(Es * kzs);
  out[0] = tt;
  out[1] = kz;
  out[2] = q0z;
  out[3] = creal(S);
  out[4] = cimag(S);
  out[5] = creal(m);
  out[6] = cimag(m);
  return 0;
}

/* ----------------------------------------------------------------- Philox */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications
 * with a fixed word permutation, the key bumped by the Weyl constants
 * between rounds. */
static uint32_t mul_hi_lo(uint32_t a, uint32_t b, uint32_t* hi) {
  uint64_t prod = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(prod >> 32);
  return (uint32_t)prod;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, hi1;
    uint32_t lo0 = mul_hi_lo(M0, x0, &hi0);
    uint32_t lo1 = mul_hi_lo(M1, x2, &hi1);
    uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* --------------------------------------------------------------- sampling */
/* Initial conditions at the tunnel exit (Sec. II.A, Eq. (2) and the
 * tunnel-exit condition; Sec. II.B for the joint alignment sampling).
 * Readings (the paper samples by the full SFA amplitude; the measured
 * workloads draw the ionisation time uniformly, weight it by an ADK-like
 * factor and draw p_perp from a Gaussian):
 *  - random numbers: trajectory j draws two Philox4x32-10 blocks with key
 *    (seed lo, seed hi) and counter (j lo, j hi, 0, block);
 *  - birth step k0 uniform on 0..N-1, t0 = t_k0;
 *  - p0 = (sigma g1, sigma g2, 0), g from Box-Muller; p_par = 0;
 *  - axis: fixed (theta, phi), or cos(beta) with density ~ cos^(2m) beta
 *    sin beta (odd root of a uniform on [-1,1]) and alpha uniform;
 *  - Eq. (2) expanded to first order about t0 (A(t0 + i y) ~ A(t0) - i y E)
 *    gives the tunnel exit q0 = Re int_{ts}^{t0} A = -(Ip + p0^2/2)/E(t0) z
 *    and |exp(i S_down)| = exp(-(2 Ip + p^2)^{3/2} / (3|E|)); the weight is
 *    its p = 0 value normalised at the peak field F0 = E0, with the static
 *    Coulomb-corrected power law of the amplitude:
 *    w = (F0/F)^{(2/kappa - 1)/2} exp(-(kappa^3/3)(1/F - 1/F0)), kappa = sqrt(2 Ip);
 *  - w < w_cut: the trajectory is dropped (w = 0) but still counted. */
static double unit_open(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

static void sample_one(const orc_problem* P, uint64_t seed, uint64_t j, int32_t N, double E0,
                       int32_t* k0, double q0[3], double p0[3], double nax[3], double* w,
                       double* dph) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t c0[4] = {(uint32_t)j, (uint32_t)(j >> 32), 0u, 0u};
  uint32_t c1[4] = {(uint32_t)j, (uint32_t)(j >> 32), 0u, 1u};
  uint32_t x[4], y[4];
  orc_philox4x32_10(c0, key, x);
  orc_philox4x32_10(c1, key, y);

  int32_t k = (int32_t)(((uint64_t)x[0] * (uint64_t)N) >> 32);
  double u1 = unit_open(x[1]), u2 = unit_open(x[2]);
  double r = sqrt(-2.0 * log(u1));
  p0[0] = P->sigma_perp * r * cos(2.0 * ORC_PI * u2);
  p0[1] = P->sigma_perp * r * sin(2.0 * ORC_PI * u2);
  p0[2] = 0.0;

  if (P->align_kind == ORC_ALIGN_FIXED) {
    nax[0] = sin(P->theta) * cos(P->phi);
    nax[1] = sin(P->theta) * sin(P->phi);
    nax[2] = cos(P->theta);
  } else {
    double c = 2.0 * unit_open(x[3]) - 1.0;
    double cb = (c < 0.0 ? -1.0 : 1.0) * pow(fabs(c), 1.0 / (2.0 * P->align_m + 1.0));
    double sb = sqrt(1.0 - cb * cb);
    double al = 2.0 * ORC_PI * unit_open(y[0]);
    nax[0] = sb * cos(al);
    nax[1] = sb * sin(al);
    nax[2] = cb;
  }

  double E;
  orc_field(P, orc_time(P, k), &E, NULL);
  double F = fabs(E);
  double ww = 0.0;
  q0[0] = q0[1] = q0[2] = 0.0;
  *dph = 0.0;
  if (P->ionization == ORC_ION_SADDLE || P->ionization == ORC_ION_SADDLE_MODIFIED) {
    /* Monte Carlo over the ionisation amplitude of Eq. (1): t0 uniform on
     * the grid, k_perp from the Gaussian above, the axis from its density;
     * weight |m e^{i S}| over the k_perp density, in units of the
     * tunnelling factor e^{-kappa^3/(3 E0)} at the peak field (kappa^2 =
     * 2 I_p), and the birth phase beyond I_p t0 + p0.q0 in dph. */
    double t0 = orc_time(P, k), out[7];
    if (orc_sfa_step(P, t0, p0, nax, out) == 0) {
      double kap = sqrt(2.0 * P->Ip);
      double kp2 = p0[0] * p0[0] + p0[1] * p0[1];
      double complex m = out[5] + I * out[6];
      p0[2] = out[1];
      q0[2] = out[2];
      /* sigma_perp = 0: k_perp = 0, no proposal density to divide out */
      double comp = P->sigma_perp > 0.0 ? kp2 / (2.0 * P->sigma_perp * P->sigma_perp) : 0.0;
      ww = cabs(m) * exp(-out[4] + kap * kap * kap / (3.0 * E0) + comp);
      *dph = (out[3] - P->Ip * t0) + carg(m);
    }
  } else if (F > 0.0) {
    double kap = sqrt(2.0 * P->Ip);
    ww = pow(E0 / F, 0.5 * (2.0 / kap - 1.0)) *
         exp(-(kap * kap * kap / 3.0) * (1.0 / F - 1.0 / E0));
    q0[2] = -(P->Ip + 0.5 * (p0[0] * p0[0] + p0[1] * p0[1] + p0[2] * p0[2])) / E;
  }
  if (!(ww >= P->w_cut)) ww = 0.0;
  if (ww == 0.0) *dph = 0.0;
  *k0 = k;
  *w = ww;
}

/* Trajectories first .. first + n - 1 of a problem, each drawn as above. */
void orc_sample(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n, int32_t* k0,
                double* q0, double* p0, double* nax, double* w, double* dph) {
  double E0;
  int32_t N;
  orc_laser(P, NULL, &E0, NULL, &N);
  for (uint64_t i = 0; i < n; ++i)
    sample_one(P, seed, first + i, N, E0, &k0[i], &q0[3 * i], &p0[3 * i], &nax[3 * i], &w[i],
               &dph[i]);
}

/* ------------------------------------------------------------- propagation */
/* State y = (q[3], p[3], M[36] row-major 6x6, S).  Hamilton's equations for
 * the coherent-state centre in the length gauge with electron charge -1
 * (Sec. II.A; H = p^2/2 + V(q) + q.E(t)), the monodromy (stability) matrix
 * dM/dt = [[0, I], [-Hess V, 0]] M with M(t0) = 1, and the continuum action
 * dS/dt = p.qdot - H = p^2/2 - V - q_z E (Sec. II.A, S_->). */
enum { NY = 43 };

static void rhs(const orc_problem* P, const double n[3], double E, const double y[NY],
                double f[NY]) {
  double V, g[3], H[9];
  orc_potential(P, n, y, &V, g, H);
  const double* p = y + 3;
  const double* M = y + 6;
  for (int a = 0; a < 3; ++a) f[a] = p[a];
  f[3] = -g[0];
  f[4] = -g[1];
  f[5] = -g[2] - E;
  double A[6][6] = {{0.0}};
  for (int a = 0; a < 3; ++a) {
    A[a][3 + a] = 1.0;
    for (int b = 0; b < 3; ++b) A[3 + a][b] = -H[3 * a + b];
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      double s = 0.0;
      for (int m = 0; m < 6; ++m) s += A[r][m] * M[6 * m + c];
      f[6 + 6 * r + c] = s;
    }
  f[42] = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - V - y[2] * E;
}

/* Classical fourth-order Runge-Kutta from t_k to t_{k+1} = t_k + dt for the
 * whole 43-component state (Hamilton's equations of Sec. II.A with the
 * monodromy and the action); the paper states no integrator for the
 * trajectories (it uses this scheme for the TDSE of Sec. II.D), so this is a
 * reading, with the field at t_k, t_k + dt/2 and t_{k+1}. */
static void rk4_step(const orc_problem* P, const double n[3], int32_t k, double y[NY]) {
  double h = P->dt;
  double tk = orc_time(P, k);
  double Ek, Eh, E1;
  orc_field(P, tk, &Ek, NULL);
  orc_field(P, tk + 0.5 * h, &Eh, NULL);
  orc_field(P, orc_time(P, k + 1), &E1, NULL);
  double k1[NY], k2[NY], k3[NY], k4[NY], yt[NY];
  rhs(P, n, Ek, y, k1);
  for (int i = 0; i < NY; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
  rhs(P, n, Eh, yt, k2);
  for (int i = 0; i < NY; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
  rhs(P, n, Eh, yt, k3);
  for (int i = 0; i < NY; ++i) yt[i] = y[i] + h * k3[i];
  rhs(P, n, E1, yt, k4);
  for (int i = 0; i < NY; ++i) y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* One trajectory's contribution a_k = -w C_k e^{i Phi_k} <psi_0|k_z|p_k,q_k>
 * to the dipole velocity (Sec. II.A: v_z ~ -<psi_0 e^{i Ip t}|k_z|psi_c> + c.c.;
 * Eq. (1) for psi_c).  Readings: the phase is Phi = S_-> + Re S_down^0 - Ip t
 * with Re S_down^0 = Ip t0 at first order, plus p0.q0 from Eq. (1); the
 * square root of det R is continued along the trajectory (C_{k0} = 1, each
 * step takes the root closer to the previous C).  Optional prefactor cap
 * (not in the paper, whose prefactor is fully included; off when c_max <= 0):
 * from the first step with |C_k| > c_max on, the trajectory contributes
 * nothing and is not propagated further. */
static int traj_core(const orc_problem* P, int32_t k0, int32_t k_end, const double q0[3],
                     const double p0[3], const double n[3], double w, double dph,
                     double* amp_re, double* amp_im, double* c_re, double* c_im, double* accum,
                     double* final_state) {
  int32_t N;
  orc_laser(P, NULL, NULL, NULL, &N);
  if (k0 < 0 || k_end < k0 || k_end > N) return -1;
  double y[NY] = {0.0};
  for (int a = 0; a < 3; ++a) {
    y[a] = q0[a];
    y[3 + a] = p0[a];
  }
  for (int a = 0; a < 6; ++a) y[6 + 6 * a + a] = 1.0;
  double complex C = 1.0, Dprev = 1.0;
  double flips = 0.0;
  double mmax = 0.0; /* largest |M_ij| over the steps reached */
  double t0 = orc_time(P, k0);
  double p0q0 = p0[0] * q0[0] + p0[1] * q0[1] + p0[2] * q0[2];
  for (int32_t k = k0;; ++k) {
    for (int i = 0; i < 36; ++i)
      if (fabs(y[6 + i]) > mmax) mmax = fabs(y[6 + i]);
    double complex D = hk_det(y + 6, P->gamma);
    double complex c = csqrt(D);
    if (creal(c * conj(C)) < 0.0) c = -c;
    if (fabs(carg(D / Dprev)) > 0.5 * ORC_PI) flips += 1.0;
    C = c;
    Dprev = D;
    if (c_re) c_re[k] = creal(C);
    if (c_im) c_im[k] = cimag(C);
    if (P->c_max > 0.0 && cabs(C) > P->c_max) break;
    double phi = y[42] - P->Ip * (orc_time(P, k) - t0) + p0q0 + dph;
    double rre, rim;
    orc_recombination(P, n, y + 3, y, &rre, &rim);
    double complex a = -w * C * cexp(I * phi) * (rre + I * rim);
    if (amp_re) amp_re[k] = creal(a);
    if (amp_im) amp_im[k] = cimag(a);
    if (accum) accum[k] += creal(a);
    if (k == k_end) break;
    rk4_step(P, n, k, y);
  }
  if (final_state) {
    memcpy(final_state, y, NY * sizeof(double));
    final_state[ORC_F_CRE] = creal(C);
    final_state[ORC_F_CIM] = cimag(C);
    final_state[ORC_F_FLIPS] = flips;
    final_state[ORC_F_MMAX] = mmax;
  }
  return 0;
}

/* One trajectory from its birth step k0 to k_end (Sec. II.A), as above. */
int orc_trajectory(const orc_problem* P, int32_t k0, int32_t k_end, const double q0[3],
                   const double p0[3], const double nax[3], double w, double dph,
                   double* amp_re, double* amp_im, double* c_re, double* c_im,
                   double* final_state) {
  return traj_core(P, k0, k_end, q0, p0, nax, w, dph, amp_re, amp_im, c_re, c_im, NULL,
                   final_state);
}

/* ------------------------------------------------------------ returns */
/* Classical return of the trajectory to the molecule (Sec. III.C: long and
 * short trajectories born in successive half-cycles return in the same time
 * window).  Reading: a return is the first entry into the sphere of radius
 * r_ret around the molecular centre after the trajectory has been outside
 * it; the return energy is the kinetic energy there (the photon energy is
 * that plus I_p).  The full state is stepped by the same RK4 as above. */
void orc_return_step(const orc_problem* P, int32_t k0, const double q0[3], const double p0[3],
                     const double nax[3], double r_ret, int32_t* k_ret, double* e_ret) {
  int32_t N;
  orc_laser(P, NULL, NULL, NULL, &N);
  double y[NY] = {0.0};
  for (int a = 0; a < 3; ++a) {
    y[a] = q0[a];
    y[3 + a] = p0[a];
  }
  for (int a = 0; a < 6; ++a) y[6 + 6 * a + a] = 1.0;
  *k_ret = -1;
  *e_ret = 0.0;
  int outside = 0;
  for (int32_t k = k0;; ++k) {
    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    if (r >= r_ret) {
      outside = 1;
    } else if (outside) {
      *k_ret = k;
      *e_ret = 0.5 * (y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
      return;
    }
    if (k >= N) return;
    rk4_step(P, nax, k, y);
  }
}

/* ------------------------------------------------------------ the ensemble */
/* Monte Carlo sum over independent trajectories (Sec. II.A-B, Eq. (4)-(6)):
 * accum[k] = sum_j Re a_jk; the dipole velocity is v_k = (2/N_s) accum[k]
 * for N_s sampled trajectories (the "+ c.c." doubles the real part).  Each
 * thread takes one contiguous index range; partial sums are added in thread
 * order. */
typedef struct {
  const orc_problem* P;
  uint64_t seed, first, n;
  double* accum;
  uint64_t live_steps, n_live;
} orc_job;

static void* run_range(void* arg) {
  orc_job* J = (orc_job*)arg;
  double E0;
  int32_t N;
  orc_laser(J->P, NULL, &E0, NULL, &N);
  for (uint64_t i = 0; i < J->n; ++i) {
    int32_t k0;
    double q0[3], p0[3], nax[3], w, dph;
    sample_one(J->P, J->seed, J->first + i, N, E0, &k0, q0, p0, nax, &w, &dph);
    if (w == 0.0) continue;
    traj_core(J->P, k0, N, q0, p0, nax, w, dph, NULL, NULL, NULL, NULL, J->accum, NULL);
    J->live_steps += (uint64_t)(N - k0);
    J->n_live += 1;
  }
  return NULL;
}

int orc_run(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n, int32_t nthreads,
            double* accum, uint64_t* live_steps, uint64_t* n_live) {
  int32_t N;
  orc_laser(P, NULL, NULL, NULL, &N);
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > n && n > 0) nthreads = (int32_t)n;
  orc_job* jobs = (orc_job*)calloc((size_t)nthreads, sizeof(orc_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) {
    free(jobs);
    free(th);
    return -1;
  }
  uint64_t base = 0;
  for (int32_t t = 0; t < nthreads; ++t) {
    uint64_t cnt = n / (uint64_t)nthreads + ((uint64_t)t < n % (uint64_t)nthreads ? 1 : 0);
    jobs[t].P = P;
    jobs[t].seed = seed;
    jobs[t].first = first + base;
    jobs[t].n = cnt;
    jobs[t].accum = (double*)calloc((size_t)N + 1, sizeof(double));
    base += cnt;
  }
  for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_range, &jobs[t]);
  for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  uint64_t ls = 0, nl = 0;
  for (int32_t k = 0; k <= N; ++k) accum[k] = 0.0;
  for (int32_t t = 0; t < nthreads; ++t) {
    for (int32_t k = 0; k <= N; ++k) accum[k] += jobs[t].accum[k];
    ls += jobs[t].live_steps;
    nl += jobs[t].n_live;
    free(jobs[t].accum);
  }
  if (live_steps) *live_steps = ls;
  if (n_live) *n_live = nl;
  free(jobs);
  free(th);
  return 0;
}

/* The same sum split by each trajectory's largest monodromy entry.  Near a
 * nucleus a trajectory can grow its monodromy matrix by many orders of
 * magnitude; rounding differences between two correct FP64 evaluations grow
 * with it, so comparisons across implementations treat these trajectories
 * apart.  A trajectory's amplitudes go into a buffer of its own first and
 * are then added to accum_all, and to accum_regular if its largest entry is
 * <= m_regular; per thread in index order, threads in order (the same
 * additions as orc_run, so accum_all equals orc_run's accum). */
typedef struct {
  const orc_problem* P;
  uint64_t seed, first, n;
  double m_regular;
  double *all, *regular, *finals;
  uint64_t live_steps, n_live;
} orc_split_job;

static void* run_split_range(void* arg) {
  orc_split_job* J = (orc_split_job*)arg;
  double E0;
  int32_t N;
  orc_laser(J->P, NULL, &E0, NULL, &N);
  double* buf = (double*)calloc((size_t)N + 1, sizeof(double));
  double fin[ORC_NFINAL];
  if (!buf) return (void*)1;
  for (uint64_t i = 0; i < J->n; ++i) {
    int32_t k0;
    double q0[3], p0[3], nax[3], w, dph;
    sample_one(J->P, J->seed, J->first + i, N, E0, &k0, q0, p0, nax, &w, &dph);
    double* row = J->finals ? J->finals + i * (uint64_t)ORC_NFINAL : NULL;
    if (w == 0.0) {
      if (row) memset(row, 0, sizeof(double) * ORC_NFINAL);
      continue;
    }
    for (int32_t k = k0; k <= N; ++k) buf[k] = 0.0;
    traj_core(J->P, k0, N, q0, p0, nax, w, dph, buf, NULL, NULL, NULL, NULL, fin);
    const int regular = fin[ORC_F_MMAX] <= J->m_regular;
    for (int32_t k = k0; k <= N; ++k) {
      J->all[k] += buf[k];
      if (regular) J->regular[k] += buf[k];
    }
    if (row) memcpy(row, fin, sizeof fin);
    J->live_steps += (uint64_t)(N - k0);
    J->n_live += 1;
  }
  free(buf);
  return NULL;
}

int orc_run_ensemble(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n,
                     int32_t nthreads, double m_regular, double* accum_all,
                     double* accum_regular, double* finals, uint64_t* live_steps,
                     uint64_t* n_live) {
  int32_t N;
  orc_laser(P, NULL, NULL, NULL, &N);
  if (!accum_all || !accum_regular) return -1;
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > n && n > 0) nthreads = (int32_t)n;
  orc_split_job* jobs = (orc_split_job*)calloc((size_t)nthreads, sizeof(orc_split_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  int fail = !jobs || !th;
  uint64_t base = 0;
  for (int32_t t = 0; !fail && t < nthreads; ++t) {
    uint64_t cnt = n / (uint64_t)nthreads + ((uint64_t)t < n % (uint64_t)nthreads ? 1 : 0);
    jobs[t].P = P;
    jobs[t].seed = seed;
    jobs[t].first = first + base;
    jobs[t].n = cnt;
    jobs[t].m_regular = m_regular;
    jobs[t].all = (double*)calloc((size_t)N + 1, sizeof(double));
    jobs[t].regular = (double*)calloc((size_t)N + 1, sizeof(double));
    jobs[t].finals = finals ? finals + base * (uint64_t)ORC_NFINAL : NULL;
    if (!jobs[t].all || !jobs[t].regular) fail = 1;
    base += cnt;
  }
  if (!fail) {
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_split_range, &jobs[t]);
    for (int32_t t = 0; t < nthreads; ++t) {
      void* r = NULL;
      pthread_join(th[t], &r);
      if (r) fail = 1;
    }
  }
  uint64_t ls = 0, nl = 0;
  for (int32_t k = 0; k <= N; ++k) accum_all[k] = accum_regular[k] = 0.0;
  for (int32_t t = 0; jobs && t < nthreads; ++t) {
    if (!fail) {
      for (int32_t k = 0; k <= N; ++k) {
        accum_all[k] += jobs[t].all[k];
        accum_regular[k] += jobs[t].regular[k];
      }
      ls += jobs[t].live_steps;
      nl += jobs[t].n_live;
    }
    free(jobs[t].all);
    free(jobs[t].regular);
  }
  if (live_steps) *live_steps = ls;
  if (n_live) *n_live = nl;
  free(jobs);
  free(th);
  return fail ? -1 : 0;
}

/* --------------------------------------------------------------- spectrum */
/* Hanning-windowed Fourier transform of the dipole velocity (Eq. (3)):
 * V(w) = dt sum_k v_k W_H(t_k) e^{i w t_k}, W_H = (1 + cos(pi t/tau_H))/2
 * for |t| <= tau_H (0 outside); the harmonic yield is |V|^2 w^2 (Sec. II.A). */
void orc_spectrum(const double* v, int32_t n_t, double t_first, double dt, double tau_H,
                  const double* omega, int32_t n_omega, double* V_re, double* V_im,
                  double* yield) {
  for (int32_t m = 0; m < n_omega; ++m) {
    double complex s = 0.0;
    for (int32_t k = 0; k < n_t; ++k) {
      double t = t_first + (double)k * dt;
      double wh = fabs(t) <= tau_H ? 0.5 * (1.0 + cos(ORC_PI * t / tau_H)) : 0.0;
      s += v[k] * wh * cexp(I * omega[m] * t);
    }
    s *= dt;
    V_re[m] = creal(s);
    V_im[m] = cimag(s);
    yield[m] = omega[m] * omega[m] * (creal(s) * creal(s) + cimag(s) * cimag(s));
  }
}

/* ------------------------------------------------------------------ Gabor */
/* Time-frequency analysis of the dipole (Sec. III.C, Fig. 8: the Gabor
 * transform locates the emission of long and short trajectories in time).
 * The paper does not give the window; reading: a Gaussian window of
 * standard deviation sigma (the caller's choice, 1/(3 w_laser) by default in
 * the front end), the plain sum over every grid point, and the yield
 * w^2 |G|^2 of the velocity form, as for the spectrum. */
void orc_gabor(const double* v, int32_t n_t, double t_first, double dt, double sigma,
               const double* t_c, int32_t n_c, const double* omega, int32_t n_omega,
               double* G_re, double* G_im, double* yield) {
  for (int32_t a = 0; a < n_c; ++a)
    for (int32_t b = 0; b < n_omega; ++b) {
      double complex g = 0.0;
      for (int32_t k = 0; k < n_t; ++k) {
        double t = t_first + k * dt;
        double x = (t - t_c[a]) / sigma;
        g += v[k] * exp(-0.5 * x * x) * cexp(I * omega[b] * t);
      }
      g *= dt;
      G_re[(size_t)a * n_omega + b] = creal(g);
      G_im[(size_t)a * n_omega + b] = cimag(g);
      yield[(size_t)a * n_omega + b] = omega[b] * omega[b] * creal(g * conj(g));
    }
}
