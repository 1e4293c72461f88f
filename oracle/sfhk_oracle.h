/*
 * SFHK oracle: a plain, slow, scalar FP64 CPU implementation of the
 * strong-field Herman-Kluk (SFHK) dipole-velocity estimator for molecular
 * high-harmonic generation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It
 * shares no code, header, table or constant generator with the HIP path.
 *
 * Atomic units throughout, except the laser (nm, W/cm^2, cycles, rad).
 */
#ifndef SFHK_ORACLE_H
#define SFHK_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_GTO 64

/* Per-trajectory final-state record written by orc_trajectory (doubles). */
enum {
  ORC_F_Q = 0,      /* q_t   [3]                                            */
  ORC_F_P = 3,      /* p_t   [3]                                            */
  ORC_F_M = 6,      /* monodromy 6x6 row-major, rows (q,p), cols (q0,p0)    */
  ORC_F_S = 42,     /* continuum action S                                   */
  ORC_F_CRE = 43,   /* HK prefactor C, real part                            */
  ORC_F_CIM = 44,   /* HK prefactor C, imaginary part                       */
  ORC_F_FLIPS = 45, /* steps where arg(D_k / D_{k-1}) exceeded pi/2        */
  ORC_F_MMAX = 46,  /* largest |M_ij| over the grid steps reached (>= 1)   */
  ORC_NFINAL = 47
};

enum { ORC_ALIGN_FIXED = 0, ORC_ALIGN_COS2M = 1 };
/* ionisation step: first-order tunnel exit with an ADK-like weight, or the
 * complex saddle point of Eq. (2) with the matrix element of Eq. (1) */
enum { ORC_ION_FIRST_ORDER = 0, ORC_ION_SADDLE = 1, ORC_ION_SADDLE_MODIFIED = 2 };

typedef struct {
  /* laser: linear polarisation along z, sin^2 envelope */
  double lambda_nm, intensity_wcm2, n_cycles, cep;
  /* target: internuclear distance R, binding energy Ip (hartree) */
  double R, Ip;
  /* per-centre potential parameters; centre 0 at +R/2 n, centre 1 at -R/2 n */
  double Zinf[2], dZ[2], alpha[2], eps2[2];
  /* GTO expansion of psi_0: centre index, l (0 = s, 1 = p along the axis) */
  int32_t n_gto;
  int32_t gto_center[ORC_MAX_GTO];
  int32_t gto_l[ORC_MAX_GTO];
  double gto_a[ORC_MAX_GTO];
  double gto_c[ORC_MAX_GTO];
  /* alignment: fixed (theta, phi) or cos^(2m) beta axis density */
  int32_t align_kind, align_m;
  double theta, phi;
  /* time step, coherent-state width, weight cut, transverse momentum sigma */
  double dt, gamma, w_cut, sigma_perp;
  int32_t n_steps; /* 0 = round(tau / dt) */
  double c_max;    /* > 0: a trajectory stops contributing once |C| > c_max */
  int32_t ionization; /* ORC_ION_FIRST_ORDER or ORC_ION_SADDLE */
} orc_problem;

/* laser constants: omega, peak field E0, pulse length tau, steps N */
void orc_laser(const orc_problem* P, double* omega, double* E0, double* tau, int32_t* N);
/* grid time t_k = -tau/2 + k dt */
double orc_time(const orc_problem* P, int32_t k);
/* E(t) and A(t) of the sin^2 pulse */
void orc_field(const orc_problem* P, double t, double* E, double* A);
/* V, grad V (3) and Hessian (3x3 row-major) of the two-centre potential for axis n */
void orc_potential(const orc_problem* P, const double n[3], const double q[3], double* V,
                   double grad[3], double hess[9]);
/* recombination element <psi_0 | k_z | p, q> for axis n */
void orc_recombination(const orc_problem* P, const double n[3], const double p[3],
                       const double q[3], double* re, double* im);
/* det of the HK matrix R built from a 6x6 monodromy matrix (row-major) */
void orc_prefactor_det(const double M[36], double gamma, double* re, double* im);
/* exact SFA ionisation step for birth time t0, transverse momentum kperp and
 * axis n: out = {t_t, k_z, q0_z, Re S, Im S, Re m, Im m} with t_s = t0 + i t_t
 * the saddle point, S the tunnelling action S_down^0, q0_z the tunnel exit
 * and m = <kappa|z E(t_s)|psi_0> / sqrt(E(t_s) kappa_z).  With
 * ionization = ORC_ION_SADDLE_MODIFIED the saddle point and the action are
 * those of the modified equation (Sec. III.C, SFHK2).  Returns 0, or -1 when
 * no saddle point exists (the trajectory is not born). */
int orc_sfa_step(const orc_problem* P, double t0, const double kperp[2], const double n[3],
                 double out[7]);
/* the laser continued to complex time t = tr + i ti: A(t) and E(t) */
void orc_field_complex(const orc_problem* P, double tr, double ti, double* A_re, double* A_im,
                       double* E_re, double* E_im);
/* Philox4x32-10 block function */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* sample trajectories first..first+n-1 of a problem with a given seed; dph
 * receives each trajectory's birth phase beyond I_p t0 + p0.q0 (0 for the
 * first-order step) */
void orc_sample(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n, int32_t* k0,
                double* q0, double* p0, double* nax, double* w, double* dph);
/* propagate one trajectory from step k0 to step k_end (<= N).  amp_re/amp_im
 * (nullable, length N+1) receive a_k for k0 <= k <= k_end; c_re/c_im
 * (nullable, length N+1) the HK prefactor C_k; final (nullable) receives
 * ORC_NFINAL doubles at the last step reached.  Returns 0, or -1 on bad input. */
int orc_trajectory(const orc_problem* P, int32_t k0, int32_t k_end, const double q0[3],
                   const double p0[3], const double nax[3], double w, double dph,
                   double* amp_re, double* amp_im, double* c_re, double* c_im,
                   double* final_state);
/* whole estimator: sample trajectories first..first+n-1, propagate the live
 * ones, accum[k] = sum_j Re a_jk (length N+1).  Returns 0 or -1. */
int orc_run(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n, int32_t nthreads,
            double* accum, uint64_t* live_steps, uint64_t* n_live);
/* orc_run with the sum split by how strongly each trajectory amplifies
 * perturbations: accum_all[k] = sum_j Re a_jk over every live trajectory,
 * accum_regular[k] the same over those whose largest monodromy entry along
 * the trajectory, max_k max_ij |M_ij(t_k)|, stays <= m_regular.  finals
 * (nullable) receives ORC_NFINAL doubles per trajectory index (row i for
 * trajectory first + i; zeros for a trajectory that is not propagated).
 * Returns 0 or -1. */
int orc_run_ensemble(const orc_problem* P, uint64_t seed, uint64_t first, uint64_t n,
                     int32_t nthreads, double m_regular, double* accum_all,
                     double* accum_regular, double* finals, uint64_t* live_steps,
                     uint64_t* n_live);
/* windowed Fourier transform of v on the grid t_first + k dt, k < n_t */
void orc_spectrum(const double* v, int32_t n_t, double t_first, double dt, double tau_H,
                  const double* omega, int32_t n_omega, double* V_re, double* V_im,
                  double* yield);

/* first return of a trajectory born at step k0: the first step k > k0 with
 * |q_k| < r_ret after some step j (k0 <= j < k) with |q_j| >= r_ret;
 * *k_ret = -1 if none up to step N; *e_ret = |p|^2/2 at that step */
void orc_return_step(const orc_problem* P, int32_t k0, const double q0[3], const double p0[3],
                     const double nax[3], double r_ret, int32_t* k_ret, double* e_ret);
/* Gabor time-frequency transform of v on the grid t_first + k dt (k < n_t):
 * G(t_c, w) = dt sum_k v_k exp(-(t_k - t_c)^2 / (2 sigma^2)) e^{i w t_k},
 * yield w^2 |G|^2; outputs [n_c][n_omega] row-major */
void orc_gabor(const double* v, int32_t n_t, double t_first, double dt, double sigma,
               const double* t_c, int32_t n_c, const double* omega, int32_t n_omega,
               double* G_re, double* G_im, double* yield);

#ifdef __cplusplus
}
#endif
#endif
