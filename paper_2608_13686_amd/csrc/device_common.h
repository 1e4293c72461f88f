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

// Arithmetic with double constants that are built in an SGPR pair where
// they are used.  The step loops leave no registers for long-lived
// constants: the compiler hoists plain literals out of the loop and then
// spills them to scratch or copies them into VGPRs at every use (it prefers
// the two-address FMAC form, whose addend must be a VGPR).  Here the scalar
// moves are volatile (never hoisted) and the FMA is the three-address VOP3
// form, which reads the SGPR pair directly.
constexpr uint64_t dbits(double x) { return __builtin_bit_cast(uint64_t, x); }
template <uint64_t B>
__device__ __forceinline__ double sconst() {
  uint32_t lo, hi;
  asm volatile("s_mov_b32 %0, %1" : "=s"(lo) : "i"((uint32_t)(B & 0xffffffffu)));
  asm volatile("s_mov_b32 %0, %1" : "=s"(hi) : "i"((uint32_t)(B >> 32)));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// VOP3 arithmetic with one operand k held in an SGPR pair.
__device__ __forceinline__ double fma_s(double a, double b, double k) {  // a b + k
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(k));
  return d;
}
__device__ __forceinline__ double fnma_s(double a, double k, double c) {  // c - a k
  double d;
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(d) : "v"(a), "s"(k), "v"(c));
  return d;
}
__device__ __forceinline__ double fnms_s(double a, double k, double b) {  // -a k - b
  double d;
  asm("v_fma_f64 %0, -%1, %2, -%3" : "=v"(d) : "v"(a), "s"(k), "v"(b));
  return d;
}
__device__ __forceinline__ double mul_s(double a, double k) {
  double d;
  asm("v_mul_f64 %0, %1, %2" : "=v"(d) : "v"(a), "s"(k));
  return d;
}
__device__ __forceinline__ double add_s(double a, double k) {
  double d;
  asm("v_add_f64 %0, %1, %2" : "=v"(d) : "v"(a), "s"(k));
  return d;
}
template <uint64_t C>
__device__ __forceinline__ double fma_k(double a, double b) { return fma_s(a, b, sconst<C>()); }
template <uint64_t C>
__device__ __forceinline__ double fnma_k(double a, double c) { return fnma_s(a, sconst<C>(), c); }
template <uint64_t C>
__device__ __forceinline__ double fnms_k(double a, double b) { return fnms_s(a, sconst<C>(), b); }
template <uint64_t C>
__device__ __forceinline__ double mul_k(double a) { return mul_s(a, sconst<C>()); }
template <uint64_t C>
__device__ __forceinline__ double add_k(double a) { return add_s(a, sconst<C>()); }
// one Horner step q <- q r + C of two independent evaluations sharing C
template <uint64_t C>
__device__ __forceinline__ void horner2(double& q0, double& q1, double r0, double r1) {
  const double k = sconst<C>();
  q0 = fma_s(q0, r0, k);
  q1 = fma_s(q1, r1, k);
}

// e^{-y} for 0 <= y <= 708.  -y = n ln2 + r with n = rint(-y / ln2) and
// |r| <= ln2/2 (the first FMA of the reduction is exact; the low part of
// ln2 corrects the rest); e^r = 1 + r (1 + r q(r)) with q a degree-9
// Chebyshev fit of (e^r - 1 - r) / r^2 on |r| <= ln2/2; 2^n by ldexp.
// Error < 0.7 ulp for results in the normal range; no range checks.
// exp_neg2 evaluates two arguments in lock step (shared constants,
// interleaved dependency chains).
__device__ __forceinline__ void exp_neg2(double y0, double y1, double& e0, double& e1) {
  double k = sconst<dbits(-1.4426950408889634)>();
  const double n0 = __builtin_rint(mul_s(y0, k)), n1 = __builtin_rint(mul_s(y1, k));
  k = sconst<dbits(0.6931471805599453)>();
  double r0 = fnms_s(n0, k, y0), r1 = fnms_s(n1, k, y1);
  k = sconst<dbits(2.3190468138462996e-17)>();
  r0 = fnma_s(n0, k, r0);
  r1 = fnma_s(n1, k, r1);
  k = sconst<dbits(2.5100375832561234e-08)>();
  double q0 = mul_s(r0, k), q1 = mul_s(r1, k);
  k = sconst<dbits(2.7620075879983367e-07)>();
  q0 = add_s(q0, k);
  q1 = add_s(q1, k);
  horner2<dbits(2.7557268480310024e-06)>(q0, q1, r0, r1);
  horner2<dbits(2.4801521322368692e-05)>(q0, q1, r0, r1);
  horner2<dbits(0.00019841269863040545)>(q0, q1, r0, r1);
  horner2<dbits(0.0013888888917196719)>(q0, q1, r0, r1);
  horner2<dbits(0.008333333333330065)>(q0, q1, r0, r1);
  horner2<dbits(0.041666666666624164)>(q0, q1, r0, r1);
  horner2<dbits(0.16666666666666669)>(q0, q1, r0, r1);
  horner2<dbits(0.5000000000000001)>(q0, q1, r0, r1);
  q0 = fma(q0, r0, 1.0);
  q1 = fma(q1, r1, 1.0);
  q0 = fma(q0, r0, 1.0);
  q1 = fma(q1, r1, 1.0);
  e0 = __builtin_amdgcn_ldexp(q0, (int)n0);
  e1 = __builtin_amdgcn_ldexp(q1, (int)n1);
}
__device__ __forceinline__ double exp_neg(double y) {
  const double n = __builtin_rint(mul_k<dbits(-1.4426950408889634)>(y));
  double r = fnms_k<dbits(0.6931471805599453)>(n, y);
  r = fnma_k<dbits(2.3190468138462996e-17)>(n, r);
  double q = add_k<dbits(2.7620075879983367e-07)>(mul_k<dbits(2.5100375832561234e-08)>(r));
  q = fma_k<dbits(2.7557268480310024e-06)>(q, r);
  q = fma_k<dbits(2.4801521322368692e-05)>(q, r);
  q = fma_k<dbits(0.00019841269863040545)>(q, r);
  q = fma_k<dbits(0.0013888888917196719)>(q, r);
  q = fma_k<dbits(0.008333333333330065)>(q, r);
  q = fma_k<dbits(0.041666666666624164)>(q, r);
  q = fma_k<dbits(0.16666666666666669)>(q, r);
  q = fma_k<dbits(0.5000000000000001)>(q, r);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return __builtin_amdgcn_ldexp(q, (int)n);
}
// The same constants held in VGPRs for a whole kernel, for kernels with
// registers to spare: made opaque once (so that the compiler neither folds
// them back into literals nor rematerialises them), then read by VOP3 FMAs
// with no scalar moves at the point of use.
struct ExpK {
  double c[13];
};
__device__ __forceinline__ ExpK make_expk() {
  ExpK k;
  const double v[13] = {-1.4426950408889634, 0.6931471805599453, 2.3190468138462996e-17,
                        2.5100375832561234e-08, 2.7620075879983367e-07, 2.7557268480310024e-06,
                        2.4801521322368692e-05, 0.00019841269863040545, 0.0013888888917196719,
                        0.008333333333330065, 0.041666666666624164, 0.16666666666666669,
                        0.5000000000000001};
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    k.c[i] = v[i];
    asm volatile("" : "+v"(k.c[i]));
  }
  return k;
}
__device__ __forceinline__ double fma_vvv(double a, double b, double c) {  // a b + c
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
// exp_neg2 with the constants of k, in the same operation order
__device__ __forceinline__ void exp_neg2_v(double y0, double y1, double& e0, double& e1,
                                           const ExpK& k) {
  const double n0 = __builtin_rint(y0 * k.c[0]), n1 = __builtin_rint(y1 * k.c[0]);
  double r0, r1;
  asm("v_fma_f64 %0, -%1, %2, -%3" : "=v"(r0) : "v"(n0), "v"(k.c[1]), "v"(y0));
  asm("v_fma_f64 %0, -%1, %2, -%3" : "=v"(r1) : "v"(n1), "v"(k.c[1]), "v"(y1));
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r0) : "v"(n0), "v"(k.c[2]), "v"(r0));
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r1) : "v"(n1), "v"(k.c[2]), "v"(r1));
  double q0 = fma_vvv(r0, k.c[3], k.c[4]), q1 = fma_vvv(r1, k.c[3], k.c[4]);
#pragma unroll
  for (int i = 5; i < 13; ++i) {
    q0 = fma_vvv(q0, r0, k.c[i]);
    q1 = fma_vvv(q1, r1, k.c[i]);
  }
  q0 = fma(q0, r0, 1.0);
  q1 = fma(q1, r1, 1.0);
  q0 = fma(q0, r0, 1.0);
  q1 = fma(q1, r1, 1.0);
  e0 = __builtin_amdgcn_ldexp(q0, (int)n0);
  e1 = __builtin_amdgcn_ldexp(q1, (int)n1);
}

// sin x and cos x for |x| < 2^31.  x = n pi/2 + r with n = rint(2x/pi) and
// |r| <= pi/4 (pi/2 in two parts; the first FMA is exact); on |r| <= pi/4,
// sin r = r + r z S(z) and cos r = 1 - z/2 + z^2 C(z), z = r^2, with S and C
// degree-5 Chebyshev fits of (sin r / r - 1) / z and (cos r - 1 + z/2) / z^2;
// the quadrant n mod 4 swaps and negates.  Absolute error < 2^-52.
__device__ __forceinline__ void sincos_k(double x, double& sn, double& cs) {
  const double n = __builtin_rint(mul_k<dbits(0.6366197723675814)>(x));
  double r = fnma_k<dbits(1.5707963267948966)>(n, x);
  r = fnma_k<dbits(6.123233995736766e-17)>(n, r);
  const double z = r * r;
  double ps = add_k<dbits(-2.5051131845003624e-08)>(mul_k<dbits(1.5918129294866608e-10)>(z));
  ps = fma_k<dbits(2.755731610255244e-06)>(ps, z);
  ps = fma_k<dbits(-0.00019841269836758574)>(ps, z);
  ps = fma_k<dbits(0.008333333333330948)>(ps, z);
  ps = fma_k<dbits(-0.16666666666666666)>(ps, z);
  double pc = add_k<dbits(2.08761462684032e-09)>(mul_k<dbits(-1.1382632425521717e-11)>(z));
  pc = fma_k<dbits(-2.7557317271729793e-07)>(pc, z);
  pc = fma_k<dbits(2.480158729876569e-05)>(pc, z);
  pc = fma_k<dbits(-0.0013888888888887398)>(pc, z);
  pc = fma_k<dbits(0.041666666666666664)>(pc, z);
  const double s_r = fma(r * z, ps, r);
  const double c_r = fma(z * z, pc, fma(z, -0.5, 1.0));
  const int q = (int)n;
  const bool swap = (q & 1) != 0;
  const double s0 = swap ? c_r : s_r, c0 = swap ? s_r : c_r;
  // sin changes sign in quadrants 2, 3; cos in quadrants 1, 2
  const uint64_t ss = (uint64_t)(q & 2) << 62, cc = (uint64_t)((q + 1) & 2) << 62;
  sn = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, s0) ^ ss);
  cs = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, c0) ^ cc);
}
// FP32 (mixed kernel): the hardware exponential
__device__ __forceinline__ void exp_neg2(float y0, float y1, float& e0, float& e1) {
  e0 = __expf(-y0);
  e1 = __expf(-y1);
}

// Far-field cut-offs.  Screening: for alpha*rho > kScreenFar at both centres
// the terms of dZ e^{-alpha rho} in V, V' and V'' are at most
// (alpha rho)^2 e^{-alpha rho} dZ / (2 Z_inf) < 2.9e-17 dZ/Z_inf of the Z_inf
// terms (4e-16 for N2's Table I values), at the rounding level, so they are
// not evaluated; when
// they are, the exponent is capped at kScreenCap (e^{-700} is nothing next to
// Z_inf, and the cap keeps the exponential in its range).  Recombination: a
// shell whose Gaussian exponent satisfies er + ln(1 + |C|) < kRecombFar
// contributes less than e^-45 1e4 = 3e-16 to a dipole sample (|b|-dependent
// factors and norms are bounded by 1e4): below one rounding unit of an O(1)
// amplitude, so its exp and sincos are not evaluated.
constexpr double kScreenFar = 45.0;
constexpr double kScreenCap = 700.0;
constexpr double kRecombFar = -45.0;

template <typename T> struct PotConst;
template <> struct PotConst<double> {
  __device__ static double Zinf(const Desc& d, int c) { return d.Zinf[c]; }
  __device__ static double dZ(const Desc& d, int c) { return d.dZ[c]; }
  __device__ static double alpha(const Desc& d, int c) { return d.alpha[c]; }
  __device__ static double eps2(const Desc& d, int c) { return d.eps2[c]; }
  __device__ static double adZ(const Desc& d, int c) { return d.adZ[c]; }
  __device__ static double a2dZ(const Desc& d, int c) { return d.a2dZ[c]; }
};
template <> struct PotConst<float> {
  __device__ static float Zinf(const Desc& d, int c) { return d.fZinf[c]; }
  __device__ static float dZ(const Desc& d, int c) { return d.fdZ[c]; }
  __device__ static float alpha(const Desc& d, int c) { return d.falpha[c]; }
  __device__ static float eps2(const Desc& d, int c) { return d.feps2[c]; }
  __device__ static float adZ(const Desc& d, int c) { return d.fadZ[c]; }
  __device__ static float a2dZ(const Desc& d, int c) { return d.fa2dZ[c]; }
};

// Sources of the potential's constants: the problem descriptor, read at
// each use (PotDesc), or values a kernel keeps in registers for a whole
// loop (PotK: the FP64 constants, or their FP32 roundings).
template <typename T>
struct PotDesc {
  const Desc& d;
  __device__ T Zinf(int c) const { return PotConst<T>::Zinf(d, c); }
  __device__ T dZ(int c) const { return PotConst<T>::dZ(d, c); }
  __device__ T alpha(int c) const { return PotConst<T>::alpha(d, c); }
  __device__ T eps2(int c) const { return PotConst<T>::eps2(d, c); }
  __device__ T adZ(int c) const { return PotConst<T>::adZ(d, c); }
  __device__ T a2dZ(int c) const { return PotConst<T>::a2dZ(d, c); }
  __device__ bool screened() const { return d.screened != 0; }
};
template <typename T>
struct PotK {
  T v[6][2];  // Zinf, dZ, alpha, eps2, adZ, a2dZ of both centres
  bool scr;
  __device__ T Zinf(int c) const { return v[0][c]; }
  __device__ T dZ(int c) const { return v[1][c]; }
  __device__ T alpha(int c) const { return v[2][c]; }
  __device__ T eps2(int c) const { return v[3][c]; }
  __device__ T adZ(int c) const { return v[4][c]; }
  __device__ T a2dZ(int c) const { return v[5][c]; }
  __device__ bool screened() const { return scr; }
};
template <typename T>
__device__ __forceinline__ PotK<T> pot_k(const Desc& d) {
  const PotDesc<T> s{d};
  PotK<T> k;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    k.v[0][c] = s.Zinf(c);
    k.v[1][c] = s.dZ(c);
    k.v[2][c] = s.alpha(c);
    k.v[3][c] = s.eps2(c);
    k.v[4][c] = s.adZ(c);
    k.v[5][c] = s.a2dZ(c);
  }
  k.scr = s.screened();
  return k;
}

// Two-centre potential of Eq. 7 with softened distance (per centre
// V_i = -Z_i(rho)/rho, Z_i = Zinf + dZ u, u = e^{-alpha rho},
// rho^2 = |q-R_i|^2 + eps2): value, gradient and the symmetric Hessian K
// (xx, yy, zz, xy, xz, yz).  With s = 1/rho and A = alpha dZ:
//   V_i' = s t,  t = Z s + A u,
//   V_i'' = -2 Z s^3 - 2 A u s^2 - alpha A u s,
// so that grad V_i = s^2 t d and
//   Hess V_i = s^2 t I + c2 d d^T,  c2 = (V_i'' - V_i'/rho) s^2
//                                      = -s^3 (3 s t + alpha A u).
// Position relative to both nuclei: d_c = q - R_c (centre 0 at +R/2 n,
// hRn = R/2 n) and the softened squared distances r2_c = |d_c|^2 + eps2_c.
// Computed once per step at q_k for the recombination amplitude and the
// first RK4 stage.
template <typename T>
struct Geom {
  T dx[2], dy[2], dz[2], r2[2];
};

template <typename T, typename P>
__device__ __forceinline__ void geometry_p(const P& k, const T hRn[3], const T q[3],
                                           Geom<T>& G) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    G.dx[c] = c == 0 ? q[0] - hRn[0] : q[0] + hRn[0];
    G.dy[c] = c == 0 ? q[1] - hRn[1] : q[1] + hRn[1];
    G.dz[c] = c == 0 ? q[2] - hRn[2] : q[2] + hRn[2];
    G.r2[c] = fma(G.dz[c], G.dz[c], fma(G.dy[c], G.dy[c], fma(G.dx[c], G.dx[c], k.eps2(c))));
  }
}
template <typename T>
__device__ __forceinline__ void geometry(const Desc& d, const T hRn[3], const T q[3],
                                         Geom<T>& G) {
  geometry_p(PotDesc<T>{d}, hRn, q, G);
}

// ek: the exponential's constants in VGPRs (FP64 only; null: built in
// SGPRs at their use).
template <typename T, typename P>
__device__ __forceinline__ void potential_p(const P& k, const Geom<T>& G, T& V, T g[3], T K[6],
                                            const ExpK* ek = nullptr) {
  const T* dx = G.dx;
  const T* dy = G.dy;
  const T* dz = G.dz;
  const T* r2 = G.r2;
  T s[2], u[2] = {T(0), T(0)};
#pragma unroll
  for (int c = 0; c < 2; ++c) s[c] = rsqrt_t(r2[c]);
  if (k.screened()) {
    // both centres' screening factors at once (an electron far from one
    // centre is far from the other); the argument is capped where e^{-y}
    // is far below a rounding unit of Z_inf
    const T ar0 = k.alpha(0) * (r2[0] * s[0]), ar1 = k.alpha(1) * (r2[1] * s[1]);
    if (ar0 < T(kScreenFar) || ar1 < T(kScreenFar)) {
      const T y0 = fmin(ar0, T(kScreenCap)), y1 = fmin(ar1, T(kScreenCap));
      if constexpr (sizeof(T) == sizeof(double)) {
        if (ek)
          exp_neg2_v(y0, y1, u[0], u[1], *ek);
        else
          exp_neg2(y0, y1, u[0], u[1]);
      } else {
        exp_neg2(y0, y1, u[0], u[1]);
      }
    }
  }
  V = T(0);
  g[0] = g[1] = g[2] = T(0);
#pragma unroll
  for (int a = 0; a < 6; ++a) K[a] = T(0);
  T diag = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T Z = k.Zinf(c) + k.dZ(c) * u[c];
    const T t = Z * s[c] + k.adZ(c) * u[c];
    const T s2 = s[c] * s[c];
    const T c1 = s2 * t;  // V_i'/rho
    // c2 = -s^3 (3 s t + alpha^2 dZ u) = -s^2 (3 c1 + alpha^2 dZ u s)
    const T c2 = -s2 * fma(T(3), c1, k.a2dZ(c) * u[c] * s[c]);
    V -= Z * s[c];
    g[0] += c1 * dx[c];
    g[1] += c1 * dy[c];
    g[2] += c1 * dz[c];
    diag += c1;
    const T ex = c2 * dx[c], ey = c2 * dy[c];
    K[0] += ex * dx[c];
    K[1] += ey * dy[c];
    K[2] += c2 * dz[c] * dz[c];
    K[3] += ex * dy[c];
    K[4] += ex * dz[c];
    K[5] += ey * dz[c];
  }
  K[0] += diag;
  K[1] += diag;
  K[2] += diag;
}

template <typename T>
__device__ __forceinline__ void potential(const Desc& d, const Geom<T>& G, T& V, T g[3],
                                          T K[6], const ExpK* ek = nullptr) {
  potential_p(PotDesc<T>{d}, G, V, g, K, ek);
}
template <typename T>
__device__ __forceinline__ void potential(const Desc& d, const T hRn[3], const T q[3], T& V,
                                          T g[3], T K[6], const ExpK* ek = nullptr) {
  Geom<T> G;
  geometry(d, hRn, q, G);
  potential(d, G, V, g, K, ek);
}

// Index of element (r, c) of a symmetric 3x3 matrix in its 6-element
// storage: xx, yy, zz, xy, xz, yz.
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
                                                const T K4[6], const RkCoef<T>& rk,
                                                StepMatrix<T>& P) {
  const T h = rk.h, c2 = rk.c2, c3 = rk.c3, c4 = rk.c4, c1 = rk.h6;
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

// M <- P M for the monodromy held in LDS (element-major, lane-minor: row-major
// 6x6, rows (q, p), columns (q0, p0)), one column at a time, and
// R2 = 2R = Mqq + Mpp - i g Mqp + (i/g) Mpq rebuilt from the new columns
// (column c < 3 holds Mqq[:, c] and Mpq[:, c], column c + 3 holds Mqp[:, c]
// and Mpp[:, c]).  The next column is loaded before the current one is
// computed, so that the LDS latency is hidden behind its arithmetic; the
// scheduling barrier per column bounds the registers in flight.
// With Track, mmax is raised to the largest |entry| of the new matrix.
template <int W, bool Track = false>
__device__ __forceinline__ void monodromy_step(const StepMatrix<double>& P, double (*mono)[W],
                                               int lane, double gamma, double inv_gamma,
                                               double Rr[3][3], double Ri[3][3],
                                               double* mmax = nullptr) {
  double x[3] = {mono[0][lane], mono[6][lane], mono[12][lane]};
  double v[3] = {mono[18][lane], mono[24][lane], mono[30][lane]};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    __builtin_amdgcn_sched_barrier(0);
    double xl[3] = {0.0, 0.0, 0.0}, vl[3] = {0.0, 0.0, 0.0};
    if (c < 5) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        xl[r] = mono[6 * r + c + 1][lane];
        vl[r] = mono[18 + 6 * r + c + 1][lane];
      }
    }
    double xn[3], vn[3];
    apply_step_matrix(P, x, v, xn, vn);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      mono[6 * r + c][lane] = xn[r];
      mono[18 + 6 * r + c][lane] = vn[r];
      if (c < 3) {
        Rr[r][c] = xn[r];
        Ri[r][c] = inv_gamma * vn[r];
      } else {
        Rr[r][c - 3] += vn[r];
        Ri[r][c - 3] -= gamma * xn[r];
      }
      if constexpr (Track) *mmax = fmax(*mmax, fmax(fabs(xn[r]), fabs(vn[r])));
      x[r] = xl[r];
      v[r] = vl[r];
    }
  }
}

// One per-slot record (SFHK_FS_* layout, field-major with stride st) of the
// state at one grid step; M is read from the LDS monodromy (element-major,
// lane-minor) of either precision.
template <typename TM, typename TS>
__device__ __forceinline__ void write_record(double* __restrict__ f, uint64_t st,
                                             const TS q[3], const TS p[3], TM (*mono)[kWave],
                                             int lane, double S, double Cre, double Cim,
                                             double flips, double mmax, double n_near) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f[(SFHK_FS_Q + a) * st] = (double)q[a];
    f[(SFHK_FS_P + a) * st] = (double)p[a];
  }
#pragma unroll
  for (int i = 0; i < 36; ++i) f[(SFHK_FS_M + i) * st] = (double)mono[i][lane];
  f[SFHK_FS_S * st] = S;
  f[SFHK_FS_CRE * st] = Cre;
  f[SFHK_FS_CIM * st] = Cim;
  f[SFHK_FS_FLIPS * st] = flips;
  f[SFHK_FS_MMAX * st] = mmax;
  f[SFHK_FS_NEAR * st] = n_near;
}

// First snapshot step at or after k: the next multiple of every.
__device__ __forceinline__ int first_snap_step(int k, int every) {
  return ((k + every - 1) / every) * every;
}

// x from lane (lane ^ m) within each 32-lane half (ds_swizzle, bit-mask
// mode: and 0x1f, or 0, xor m); the pattern is an immediate, no address VGPR
template <int M>
__device__ __forceinline__ double swizzle_xor(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)b, (M << 10) | 0x1f);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), (M << 10) | 0x1f);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += __shfl_xor(v, 32, kWave);
  v += swizzle_xor<16>(v);
  v += swizzle_xor<8>(v);
  v += swizzle_xor<4>(v);
  v += swizzle_xor<2>(v);
  v += swizzle_xor<1>(v);
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

// det R of the complex 3x3 R = Rr + i Ri (cofactor expansion along row 0),
// each term one multiply-add chain.
template <typename T>
__device__ __forceinline__ void det3c(const T Rr[3][3], const T Ri[3][3], T& Dr, T& Di) {
  // complex 2x2 minors of rows 1, 2: m_j = R[1][a] R[2][b] - R[1][b] R[2][a]
  T mr[3], mi[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int a = j == 0 ? 1 : 0, b = j == 2 ? 1 : 2;
    mr[j] = fma(Rr[1][a], Rr[2][b],
                fma(-Ri[1][a], Ri[2][b], fma(-Rr[1][b], Rr[2][a], Ri[1][b] * Ri[2][a])));
    mi[j] = fma(Rr[1][a], Ri[2][b],
                fma(Ri[1][a], Rr[2][b], fma(-Rr[1][b], Ri[2][a], -(Ri[1][b] * Rr[2][a]))));
  }
  Dr = fma(Rr[0][0], mr[0], fma(-Ri[0][0], mi[0], fma(-Rr[0][1], mr[1],
       fma(Ri[0][1], mi[1], fma(Rr[0][2], mr[2], -(Ri[0][2] * mi[2]))))));
  Di = fma(Rr[0][0], mi[0], fma(Ri[0][0], mr[0], fma(-Rr[0][1], mi[1],
       fma(-Ri[0][1], mr[1], fma(Rr[0][2], mi[2], Ri[0][2] * mr[2])))));
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
  // a square root (either sign: the continuation below picks it): (big,
  // small) for Dr >= 0, (small, big) for Dr < 0, each free of cancellation
  const double big = u * ru, small = 0.5 * Di * ru;
  const bool pos = Dr >= 0.0;
  double sr = pos ? big : small;
  double si = pos ? small : big;
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

// One prefactor step from R2 = 2R (kept doubled: the factors 1/2 are left out
// of its entries, and det R = det R2 / 8 exactly, a power-of-two scaling).
__device__ __forceinline__ void prefactor_step(const double R2r[3][3], const double R2i[3][3],
                                               double& Cre, double& Cim, double& flips) {
  double Dr, Di;
  det3c(R2r, R2i, Dr, Di);
  sqrt_continued(0.125 * Dr, 0.125 * Di, Cre, Cim, flips);
}

// Re a_k of the amplitude a = -w C e^{i Phi} <psi0|k_z|p,q>,
// Phi = S - Ip (t_k - t0) + p0.q0 (Sec. II.A; Eq. 4), with the recombination
// element as a sum of Gaussian moments of the GTO primitives, taken shell by
// shell (the primitives of one centre and exponent share the Gaussian
// factor).  Shells below the far-field cut are skipped (their terms are
// < 3e-16).
// near is set when at least one shell passes the far-field cut (the step
// evaluates the recombination sum).
__device__ __forceinline__ double amplitude_re(const Desc& d, const double n[3],
                                               const double p[3], const Geom<double>& G,
                                               double Cre, double Cim, double S, double tk,
                                               double t0, double p0q0, double w, bool& near) {
  near = false;
  const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  // |R_a - q|^2 from the softened distances of the geometry at q
  const double dd[2] = {G.r2[0] - d.eps2[0], G.r2[1] - d.eps2[1]};
  // ln(1 + |C|) bound from the binary exponent of 1 + |C|^2
  const double cc = 1.0 + Cre * Cre + Cim * Cim;
  const double lnC = 0.3466 * (double)(((int)(__double_as_longlong(cc) >> 52) & 0x7ff) - 1022);
  // every shell's exponent er <= -|R_a - q|^2 / (4 kappa2) <= -dd g_inv4k_min
  // (the |p|^2 coefficient of er is <= 0): the whole sum is below the cut
  if (fmin(dd[0], dd[1]) * d.g_inv4k_min + kRecombFar > lnC) return 0.0;
  const double np_ = n[0] * p[0] + n[1] * p[1] + n[2] * p[2];
  const double bzr = p[2] * d.inv_gamma;
  const double nbr = np_ * d.inv_gamma;
  const double bb_re_p = pp * d.inv_gamma2;
  const double ppg = pp * d.half_inv_gamma;
  double rr = 0.0, ri = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    // R_a - q = -d_c
    const double dz = -G.dz[c];
    const double pd = -(p[0] * G.dx[c] + p[1] * G.dy[c] + p[2] * G.dz[c]);  // p.(R_a - q)
    const double nd = -(n[0] * G.dx[c] + n[1] * G.dy[c] + n[2] * G.dz[c]);  // n.(R_a - q)
    const double ddc = dd[c];
    const int j0 = c == 0 ? 0 : d.n_shell0, j1 = c == 0 ? d.n_shell0 : d.n_shell;
    for (int j = j0; j < j1; ++j) {
      const double i4 = d.sh_inv4k[j], i2 = 2.0 * i4;
      const double er = (bb_re_p - ddc) * i4 - ppg;  // <= 0
      if (er + lnC < kRecombFar) continue;
      near = true;
      const double ei = 2.0 * pd * d.inv_gamma * i4;
      const double gm = exp_neg(-er);
      double sn, cs;
      sincos_k(ei, sn, cs);
      const double Gr = gm * cs, Gi = gm * sn;
      // s primitives: b_z / (2 kappa2); p primitives:
      // i/(2a) [n_z/(2 kappa2) + b_z (n.b)/(4 kappa2^2)], b = p/gamma + i (R_a - q)
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
  }
  if (rr == 0.0 && ri == 0.0) return 0.0;
  const double phi = S - d.Ip * (tk - t0) + p0q0;
  double sp, cp;
  sincos_k(phi, sp, cp);
  const double er_ = Cre * cp - Cim * sp, ei_ = Cre * sp + Cim * cp;
  return -w * (er_ * rr - ei_ * ri);
}

// Dipole deposit: the wavefront sum of Re a_k (one cross-half exchange, then
// five swizzle levels) is kept by lane (k mod 64);
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
