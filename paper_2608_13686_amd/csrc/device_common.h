// Device building blocks shared by the FP64 and the mixed-precision trajectory
// kernels: reciprocal square roots, the two-centre potential with gradient and
// Hessian, the HK prefactor step, the recombination amplitude and the dipole
// deposit.
#pragma once

#include "sfhk_internal.h"

namespace sfhk {

// 1/sqrt(x), x > 0: the hardware estimate (relative error ~2^-24) refined by
// the second-order expansion of (1 - e)^(-1/2), e = 1 - x y^2 (error < 2 ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt_nr(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }
__device__ __forceinline__ float exp_t(float x) { return __expf(x); }

// Far-field cut-offs.  Screening: for alpha*rho > kScreenFar the terms of
// dZ e^{-alpha rho} in V, V' and V'' are below 1e-21 of the Z_inf terms, far
// under one rounding unit, so they are not evaluated.  Recombination: a GTO
// primitive whose Gaussian exponent satisfies er + ln(1 + |C|) < kRecombFar
// contributes less than 1e-30 to a dipole sample (|b|-dependent factors and
// norms are bounded by 1e4), so its exp and sincos are not evaluated.
constexpr double kScreenFar = 60.0;
constexpr double kRecombFar = -75.0;

template <typename T> struct PotConst;
template <> struct PotConst<double> {
  __device__ static double Zinf(const Desc& d, int c) { return d.Zinf[c]; }
  __device__ static double dZ(const Desc& d, int c) { return d.dZ[c]; }
  __device__ static double alpha(const Desc& d, int c) { return d.alpha[c]; }
  __device__ static double eps2(const Desc& d, int c) { return d.eps2[c]; }
};
template <> struct PotConst<float> {
  __device__ static float Zinf(const Desc& d, int c) { return d.fZinf[c]; }
  __device__ static float dZ(const Desc& d, int c) { return d.fdZ[c]; }
  __device__ static float alpha(const Desc& d, int c) { return d.falpha[c]; }
  __device__ static float eps2(const Desc& d, int c) { return d.feps2[c]; }
};

// Two-centre potential of Eq. 7 with softened distance (per centre
// V_i = -Z_i(rho)/rho, Z_i = Zinf + dZ e^{-alpha rho}, rho^2 = |q-R_i|^2 + eps2):
// value, gradient and the symmetric Hessian K (xx, yy, zz, xy, xz, yz).
template <typename T>
__device__ __forceinline__ void potential(const Desc& d, const T hRn[3], const T q[3], T& V,
                                          T g[3], T K[6]) {
  using PC = PotConst<T>;
  V = T(0);
  g[0] = g[1] = g[2] = T(0);
#pragma unroll
  for (int a = 0; a < 6; ++a) K[a] = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T dx = c == 0 ? q[0] - hRn[0] : q[0] + hRn[0];
    const T dy = c == 0 ? q[1] - hRn[1] : q[1] + hRn[1];
    const T dz = c == 0 ? q[2] - hRn[2] : q[2] + hRn[2];
    const T r2 = dx * dx + dy * dy + dz * dz + PC::eps2(d, c);
    const T inv = rsqrt_t(r2);
    T Z = PC::Zinf(d, c);
    T f1 = Z * inv * inv;
    T f2 = T(-2) * Z * inv * inv * inv;
    if (d.screened) {
      const T ar = PC::alpha(d, c) * (r2 * inv);
      if (ar < T(kScreenFar)) {
        const T ex = exp_t(-ar);
        const T adx = PC::alpha(d, c) * PC::dZ(d, c) * ex;
        Z += PC::dZ(d, c) * ex;
        f1 = (Z * inv + adx) * inv;
        f2 = -(T(2) * Z * inv * inv + T(2) * adx * inv + PC::alpha(d, c) * adx) * inv;
      }
    }
    V -= Z * inv;
    const T c1 = f1 * inv;               // f'/rho
    const T c2 = (f2 - c1) * inv * inv;  // (f'' - f'/rho)/rho^2
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
template <typename T>
__device__ __forceinline__ void symmul(const T K[6], const T x[3], T y[3]) {
  y[0] = K[0] * x[0] + K[3] * x[1] + K[4] * x[2];
  y[1] = K[3] * x[0] + K[1] * x[1] + K[5] * x[2];
  y[2] = K[4] * x[0] + K[5] * x[1] + K[2] * x[2];
}

// Index of element (r, c) of a symmetric 3x3 matrix in the 6-element storage
// used by symmul: xx, yy, zz, xy, xz, yz.
__device__ __forceinline__ constexpr int sym_idx(int r, int c) {
  return r == c ? r : (r + c == 1 ? 3 : (r + c == 2 ? 4 : 5));
}

// Step matrix of one RK4 step of the monodromy equation.  M' = A(t) M with
// A = [[0, I], [-K, 0]] is linear, so RK4 with the stage Hessians K1..K4 maps
// M to P M exactly; expanding the four stages (a product of two A's is block
// diagonal) gives
//   P11 = I - h^2/6 (K1 + K2 + K3) + h^4/24 K3 K1
//   P12 = h I - h^3/12 (K2 + K3)                       (symmetric)
//   P21 = -h/6 (K1 + 2 K2 + 2 K3 + K4) + h^3/12 (K3 K1 + K4 K2)
//   P22 = I - h^2/6 (K2 + K3 + K4) + h^4/24 K4 K2.
// Building P once and applying it to the six columns takes fewer operations
// than running RK4 on every column.
template <typename T>
struct StepMatrix {
  T a[3][3];  // P11
  T b[6];     // P12, symmetric storage
  T c[3][3];  // P21
  T d[3][3];  // P22
};

// With Inc = true the identity is left out of P11 and P22 (the step is then
// applied as an increment, apply_step_increment), so that their small
// O(h^2 K) parts keep full relative precision in FP32.
template <typename T, bool Inc = false>
__device__ __forceinline__ void rk4_step_matrix(const T K1[6], const T K2[6], const T K3[6],
                                                const T K4[6], T h, StepMatrix<T>& P) {
  const T c2 = h * h / T(6), c3 = h * h * h / T(12), c4 = h * h * h * h / T(24), c1 = h / T(6);
  T s23[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) s23[i] = K2[i] + K3[i];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T q31 = K3[sym_idx(r, 0)] * K1[sym_idx(0, c)] + K3[sym_idx(r, 1)] * K1[sym_idx(1, c)] +
                    K3[sym_idx(r, 2)] * K1[sym_idx(2, c)];
      const T q42 = K4[sym_idx(r, 0)] * K2[sym_idx(0, c)] + K4[sym_idx(r, 1)] * K2[sym_idx(1, c)] +
                    K4[sym_idx(r, 2)] * K2[sym_idx(2, c)];
      const int i = sym_idx(r, c);
      const T dl = (r == c && !Inc) ? T(1) : T(0);
      P.a[r][c] = dl - c2 * (K1[i] + s23[i]) + c4 * q31;
      P.d[r][c] = dl - c2 * (s23[i] + K4[i]) + c4 * q42;
      P.c[r][c] = c3 * (q31 + q42) - c1 * (K1[i] + K4[i] + T(2) * s23[i]);
    }
#pragma unroll
  for (int i = 0; i < 6; ++i) P.b[i] = (i < 3 ? h : T(0)) - c3 * s23[i];
}

// One monodromy column through a step matrix built with Inc = true:
// (x, v) + (P11 - I, P12; P21, P22 - I)(x, v).
template <typename T>
__device__ __forceinline__ void apply_step_increment(const StepMatrix<T>& P, const T x[3],
                                                     const T v[3], T xn[3], T vn[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T dx = P.a[r][0] * x[0] + P.a[r][1] * x[1] + P.a[r][2] * x[2] +
                 P.b[sym_idx(r, 0)] * v[0] + P.b[sym_idx(r, 1)] * v[1] + P.b[sym_idx(r, 2)] * v[2];
    const T dv = P.c[r][0] * x[0] + P.c[r][1] * x[1] + P.c[r][2] * x[2] + P.d[r][0] * v[0] +
                 P.d[r][1] * v[1] + P.d[r][2] * v[2];
    xn[r] = x[r] + dx;
    vn[r] = v[r] + dv;
  }
}

// One monodromy column (x, v) = (dq/dz_c, dp/dz_c) through the step matrix.
template <typename T>
__device__ __forceinline__ void apply_step_matrix(const StepMatrix<T>& P, const T x[3],
                                                  const T v[3], T xn[3], T vn[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    xn[r] = P.a[r][0] * x[0] + P.a[r][1] * x[1] + P.a[r][2] * x[2] + P.b[sym_idx(r, 0)] * v[0] +
            P.b[sym_idx(r, 1)] * v[1] + P.b[sym_idx(r, 2)] * v[2];
    vn[r] = P.c[r][0] * x[0] + P.c[r][1] * x[1] + P.c[r][2] * x[2] + P.d[r][0] * v[0] +
            P.d[r][1] * v[1] + P.d[r][2] * v[2];
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// The pack a wavefront works on: problem index, lane validity and slot.
struct Pack {
  int prob;
  bool valid;
  uint32_t slot;
};

__device__ __forceinline__ bool find_pack(const EnsPtrs& e, int n_prob, uint32_t pack, int lane,
                                          Pack& out) {
  if (pack >= e.pack_start[n_prob]) return false;
  int lo = 0, hi = n_prob;  // pack_start[lo] <= pack < pack_start[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (e.pack_start[mid] <= pack) lo = mid; else hi = mid;
  }
  const uint32_t pos = (pack - e.pack_start[lo]) * kWave + lane;
  out.prob = lo;
  out.valid = pos < e.live_count[lo];
  out.slot = out.valid ? e.order[e.live_start[lo] + pos] : 0u;
  return true;
}

// det R of the complex 3x3 R = Rr + i Ri (cofactor expansion along row 0).
template <typename T>
__device__ __forceinline__ void det3c(const T Rr[3][3], const T Ri[3][3], T& Dr, T& Di) {
  const T c0r = Rr[1][1] * Rr[2][2] - Ri[1][1] * Ri[2][2] - (Rr[1][2] * Rr[2][1] - Ri[1][2] * Ri[2][1]);
  const T c0i = Rr[1][1] * Ri[2][2] + Ri[1][1] * Rr[2][2] - (Rr[1][2] * Ri[2][1] + Ri[1][2] * Rr[2][1]);
  const T c1r = Rr[1][0] * Rr[2][2] - Ri[1][0] * Ri[2][2] - (Rr[1][2] * Rr[2][0] - Ri[1][2] * Ri[2][0]);
  const T c1i = Rr[1][0] * Ri[2][2] + Ri[1][0] * Rr[2][2] - (Rr[1][2] * Ri[2][0] + Ri[1][2] * Rr[2][0]);
  const T c2r = Rr[1][0] * Rr[2][1] - Ri[1][0] * Ri[2][1] - (Rr[1][1] * Rr[2][0] - Ri[1][1] * Ri[2][0]);
  const T c2i = Rr[1][0] * Ri[2][1] + Ri[1][0] * Rr[2][1] - (Rr[1][1] * Ri[2][0] + Ri[1][1] * Rr[2][0]);
  Dr = (Rr[0][0] * c0r - Ri[0][0] * c0i) - (Rr[0][1] * c1r - Ri[0][1] * c1i) +
       (Rr[0][2] * c2r - Ri[0][2] * c2i);
  Di = (Rr[0][0] * c0i + Ri[0][0] * c0r) - (Rr[0][1] * c1i + Ri[0][1] * c1r) +
       (Rr[0][2] * c2i + Ri[0][2] * c2r);
}

// HK prefactor C = sqrt(D), D = det R: the principal root continued along
// the trajectory (the root whose ratio to the previous C has a non-negative
// real part).  flips counts the steps at which arg(D_k / D_{k-1}) =
// 2 arg(C_k / C_{k-1}) leaves (-pi/2, pi/2], i.e.
// |Im(C_k conj C_{k-1})| > Re(C_k conj C_{k-1}).
__device__ __forceinline__ void sqrt_continued(double Dr, double Di, double& Cre, double& Cim,
                                               double& flips) {
  // principal root: u = (|D| + |Dr|)/2, sqrt(u) and Di/(2 sqrt(u)) from one
  // reciprocal square root each (|D| >= 1 for a symplectic M)
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
}

__device__ __forceinline__ void prefactor_step(const double Rr[3][3], const double Ri[3][3],
                                               double& Cre, double& Cim, double& flips) {
  double Dr, Di;
  det3c(Rr, Ri, Dr, Di);
  sqrt_continued(Dr, Di, Cre, Cim, flips);
}

// Re a_k of the amplitude a = -w C e^{i Phi} <psi0|k_z|p,q>,
// Phi = S - Ip (t_k - t0) + p0.q0 (Sec. II.A; Eq. 4), with the recombination
// element as a sum of Gaussian moments of the GTO primitives.  Primitives
// below the far-field cut are skipped (their terms are < 1e-30).
__device__ __forceinline__ double amplitude_re(const Desc& d, const double n[3],
                                               const double p[3], const double q[3],
                                               double Cre, double Cim, double S, double tk,
                                               double t0, double p0q0, double w) {
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
  // ln(1 + |C|) bound from the binary exponent of 1 + |C|^2
  const double cc = 1.0 + Cre * Cre + Cim * Cim;
  const double lnC = 0.3466 * (double)(((int)(__double_as_longlong(cc) >> 52) & 0x7ff) - 1022);
  // every primitive's exponent er <= -|R_a - q|^2 / (4 kappa2) <= -dd g_inv4k_min
  // (the |p|^2 coefficient of er is <= 0): the whole sum is below the cut
  if (fmin(dd[0], dd[1]) * d.g_inv4k_min + kRecombFar > lnC) return 0.0;
  const double bzr = p[2] * d.inv_gamma;
  const double bb_re_p = pp * d.inv_gamma2;
  double rr = 0.0, ri = 0.0;
  for (int j = 0; j < d.n_gto; ++j) {
    const int c = (d.g_l[j] >> 1) & 1;
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
    if ((d.g_l[j] & 1) == 0) {
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
  if (rr == 0.0 && ri == 0.0) return 0.0;
  const double phi = S - d.Ip * (tk - t0) + p0q0;
  double sp, cp;
  sincos(phi, &sp, &cp);
  const double er_ = Cre * cp - Cim * sp, ei_ = Cre * sp + Cim * cp;
  return -w * (er_ * rr - ei_ * ri);
}

// Dipole deposit: the wavefront sum of Re a_k is kept by lane (k mod 64);
// every 64 steps (and at the last step) the wavefront adds its 64 sums to the
// accumulator with one coalesced atomic.  Uniform control flow required.
__device__ __forceinline__ void deposit(double re_a, int k, int N, int lane, double& acc_reg,
                                        double* __restrict__ acc) {
  if (__ballot(re_a != 0.0)) {
    const double tot = wave_sum(re_a);
    if (lane == (k & (kWave - 1))) acc_reg += tot;
  }
  if ((k & (kWave - 1)) == kWave - 1 || k >= N) {
    if (acc_reg != 0.0) unsafeAtomicAdd(&acc[(k & ~(kWave - 1)) + lane], acc_reg);
    acc_reg = 0.0;
  }
}

}  // namespace sfhk
