/*
 * sfhk.h -- C ABI of the MI355X strong-field Herman-Kluk (SFHK) hot path.
 *
 * The library computes the SFHK estimate of the molecular dipole velocity
 * and its high-harmonic spectrum (arXiv 2608.13686, Sec. II.A-B):
 *   1. sample trajectories at the tunnel exit     -> sfhk_sample_initial
 *   2. propagate them with their monodromy, action,
 *      HK prefactor and recombination amplitude,
 *      summing Re a_jk over trajectories          -> sfhk_propagate
 *   3. normalise the sum into v_z(t_k)             -> sfhk_dipole
 *   4. Hanning-windowed Fourier transform          -> sfhk_spectrum
 *      (and its time-resolved form                 -> sfhk_gabor)
 *
 * Conventions
 *  - Atomic units, except the laser (nm, W/cm^2, optical cycles, rad).
 *  - Every pointer documented as "device" is a HIP device pointer owned by
 *    the caller; the library never allocates or frees device memory (apart
 *    from the one fixed array behind sfhk_propagate_static, reserved when
 *    the library is loaded on a GPU).
 *    "host" pointers are read during the call only.
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *    enqueued asynchronously on it; outputs are valid once it completes.
 *  - Arguments are validated before anything is enqueued: a bad argument
 *    returns SFHK_E_INVALID and enqueues nothing.  A HIP launch error returns
 *    SFHK_E_DEVICE.  sfhk_last_error() describes the last failure of the
 *    calling thread.  No C++ exception crosses this interface.
 *  - Trajectory j of problem P depends only on (seeds[P], first_index[P] + j):
 *    splitting an ensemble over calls draws the same trajectories.
 */
#ifndef SFHK_H
#define SFHK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFHK_ABI_VERSION 3
#define SFHK_MAX_GTO 64
#define SFHK_MAX_PROBLEMS 65535

typedef enum {
  SFHK_OK = 0,
  SFHK_E_INVALID = 1,     /* bad argument; nothing was enqueued            */
  SFHK_E_NOMEM = 2,       /* workspace or buffer too small                 */
  SFHK_E_DEVICE = 3,      /* HIP reported an error                          */
  SFHK_E_BUSY = 4,        /* resource in use                                */
  SFHK_E_UNSUPPORTED = 5  /* valid request the library does not implement   */
} sfhk_status;

typedef enum { SFHK_FP64 = 0, SFHK_MIXED = 1 } sfhk_precision;
typedef enum { SFHK_ALIGN_FIXED = 0, SFHK_ALIGN_COS2M = 1 } sfhk_align_kind;

/* Ionisation step of sfhk_sample_initial.  FIRST_ORDER: birth at the tunnel
 * exit of Eq. 2 expanded to first order about t0, p0 = (k_perp, 0), weight
 * from the quasi-static tunnelling rate.  SADDLE: the complex saddle point of
 * Eq. 2 for real momentum (t_s = t0 + i t_t, k_z fixed by Eq. 2), tunnel exit
 * Re int A, and the amplitude of Eq. 1 (matrix element of r.E(t_s) over
 * sqrt(E.kappa), times e^{i(S_down^0 + p0.q0)}) split into the weight w (its
 * modulus over the k_perp proposal density) and the birth phase dph. */
typedef enum {
  SFHK_ION_FIRST_ORDER = 0,
  SFHK_ION_SADDLE = 1,
  /* SADDLE with the modified equation of Sec. III.C (SFHK2): the extra term
   * -eta E(t_s).r0, r0 = R/2, with eta the sign for which it raises the
   * binding energy (sgn E(t0) E(t_s) (R/2)|n_z|), and the matching action
   * term eta r0.(A(t_s) - A(t0)) */
  SFHK_ION_SADDLE_MODIFIED = 2
} sfhk_ionization;

/* One centre of the two-centre model potential (Eq. 7, Table I):
 * V_i = -[Zinf + dZ exp(-alpha rho)] / rho, rho = sqrt(|r - R_i|^2 + eps2).
 * eps2 = 0 is Eq. 7 itself; dZ = 0 is a soft-core Coulomb centre.
 * Requires eps2 >= 0 and alpha >= 0 (a screening that decays). */
typedef struct {
  double Zinf, dZ, alpha, eps2;
} sfhk_center;

/* One GTO primitive of psi_0 (Sec. II.A, GTO expansion):
 * l = 0: c exp(-a |x - R_c|^2);  l = 1: c n.(x - R_c) exp(-a |x - R_c|^2),
 * centre 0 at +R/2 n, centre 1 at -R/2 n, n the molecular axis. */
typedef struct {
  int32_t center; /* 0 or 1          */
  int32_t l;      /* 0 (s) or 1 (p_n) */
  double a;       /* exponent > 0    */
  double c;       /* coefficient     */
} sfhk_gto;

typedef struct {
  double R;               /* internuclear distance                         */
  double Ip;              /* binding energy of psi_0 (hartree), > 0         */
  sfhk_center ctr[2];     /* ctr[0] at +R/2 n, ctr[1] at -R/2 n             */
  int32_t n_gto;          /* 1..SFHK_MAX_GTO                                */
  int32_t reserved;
  const sfhk_gto* gto;    /* host array [n_gto]                             */
} sfhk_target;

/* Linearly z-polarised pulse with a sin^2 envelope (Sec. II.D, III.A), centred
 * at t = 0: A(t) = -(E0/w) cos^2(pi t/tau) sin(w t + cep), |t| <= tau/2,
 * E = -dA/dt, w = 45.56335252912/lambda_nm, E0 = sqrt(I/3.50944552e16),
 * tau = n_cycles 2 pi / w.  intensity 0 switches the laser off. */
typedef struct {
  double lambda_nm, intensity_wcm2, n_cycles, cep;
} sfhk_laser;

/* Alignment (Sec. II.B, Eq. 5-6): FIXED axis n = (sin th cos ph, sin th sin ph,
 * cos th), or COS2M: cos(beta) with density ~ cos^(2m) beta sin beta and alpha
 * uniform, one axis per trajectory (m = 0 is isotropic). */
typedef struct {
  int32_t kind; /* sfhk_align_kind */
  int32_t m;
  double theta, phi;
} sfhk_align;

typedef struct {
  sfhk_target tgt;
  sfhk_laser las;
  sfhk_align al;
  double dt;         /* RK4 step (a.u.) > 0                                */
  double gamma_cs;   /* coherent-state width gamma (Sec. II.A uses 1)       */
  double w_cut;      /* trajectories with weight below it are not propagated */
  double sigma_perp; /* std. dev. of each transverse initial momentum       */
  int32_t n_steps;   /* 0: N = round(tau / dt); time grid t_k = -tau/2 + k dt */
  int32_t ionization; /* sfhk_ionization: how sfhk_sample_initial draws the birth */
  double c_max;      /* optional prefactor cap: > 0 stops a trajectory's contributions from
                        the first step with |C| > c_max (a filter of chaotic trajectories
                        the paper does not use); <= 0: prefactor fully included */
} sfhk_problem;

/* Sampled ensemble: structure of arrays in device memory, `capacity` slots.
 * Problem P owns slots [off_P, off_P + n_per_prob[P]) with off_P the prefix
 * sum of n_per_prob.  Filled by sfhk_sample_initial:
 *   k0    birth step (int32), prob problem index (int32),
 *   q0 = (qx,qy,qz), p0 = (px,py,pz), weight w (0 = not propagated),
 *   axis n = (nx,ny,nz), birth phase dph (the phase of the trajectory's
 *   ionisation amplitude beyond I_p t0 + p0.q0; 0 for the first-order step);
 *   order[capacity]: slot ids of the live trajectories sorted by (problem,
 *       k0), ties by slot id; entries past the live total are unspecified;
 *   live_start[n_prob], live_count[n_prob]: each problem's run in `order`;
 *   pack_start[n_prob + 1]: prefix sum of ceil(live_count / 64) (one 64-lane
 *       pack per wavefront; pack_start[n_prob] is the total). */
typedef struct {
  uint64_t capacity;
  int32_t* k0;
  int32_t* prob;
  double *qx, *qy, *qz;
  double *px, *py, *pz;
  double* w;
  double *nx, *ny, *nz;
  double* dph;
  uint32_t* order;
  uint32_t* live_start;
  uint32_t* live_count;
  uint32_t* pack_start;
} sfhk_ensemble;

/* Per-trajectory final state (optional output of sfhk_propagate): device
 * array [SFHK_FS_COUNT][capacity] (field-major), indexed by slot. */
enum {
  SFHK_FS_Q = 0,      /* q(t_N) [3]                                              */
  SFHK_FS_P = 3,      /* p(t_N) [3]                                              */
  SFHK_FS_M = 6,      /* monodromy [36], row-major 6x6, rows (q,p), cols (q0,p0) */
  SFHK_FS_S = 42,     /* continuum action S                                      */
  SFHK_FS_CRE = 43,   /* HK prefactor C (real)                                   */
  SFHK_FS_CIM = 44,   /* HK prefactor C (imaginary)                              */
  SFHK_FS_FLIPS = 45, /* steps at which arg(D_k / D_{k-1}) left (-pi/2, pi/2]      */
  SFHK_FS_MMAX = 46,  /* largest |M_ij| over the grid steps reached (>= 1): how far
                         the trajectory amplifies perturbations                  */
  SFHK_FS_NEAR = 47,  /* steps at which the kernel evaluated the recombination sum
                         (a shell of psi_0 passed its far-field cut)             */
  SFHK_FS_COUNT = 48
};

/* SFHK_ABI_VERSION of the library. */
int32_t sfhk_abi_version(void);

/* Description of the calling thread's last failure ("" if none). */
const char* sfhk_last_error(void);

/* Host only.  Number of steps N, first grid time t_0 = -tau/2 and pulse length
 * tau of a problem (Sec. II.D laser; grid t_k = t_0 + k dt, k = 0..N). */
sfhk_status sfhk_problem_steps(const sfhk_problem* p, int32_t* n_steps, double* t_first,
                               double* tau);

/* Host only.  Bytes of device workspace that sfhk_sample_initial and
 * sfhk_propagate (either precision) need for these problems and `capacity`
 * slots.  0 for invalid problems. */
size_t sfhk_workspace_bytes(const sfhk_problem* probs, int32_t n_prob, uint64_t capacity);

/* Host only.  Device bytes of the whole path for one problem of n_traj
 * trajectories at `precision` (Sec. II.A-B: the sampled ensemble and its
 * packing, the propagation's workspace, the dipole accumulator and v): the
 * sum of the 256-byte aligned arrays sfhk_ensemble (capacity n_traj, one
 * problem), a workspace of sfhk_propagate at this precision (which also
 * serves sfhk_sample_initial) and accum and v of N + 1 doubles each.  The
 * admission size of a request.  0 for an invalid problem or precision. */
size_t sfhk_footprint_bytes(const sfhk_problem* p, uint64_t n_traj, int32_t precision);

/* Sample the ensemble (Sec. II.A tunnel exit; Sec. II.B joint alignment):
 * for problem P, trajectories first_index[P] .. + n_per_prob[P] - 1 drawn
 * from the counter-based Philox4x32-10 stream keyed by seeds[P]; birth step
 * uniform, p_perp Gaussian, axis by the alignment rule, first-order tunnel
 * exit, amplitude weight; then sorts the live ones by (problem, k0) into
 * 64-lane packs.  probs, n_per_prob, seeds, first_index: host arrays
 * [n_prob]; sum(n_per_prob) <= ens->capacity; workspace: device,
 * >= sfhk_workspace_bytes. */
sfhk_status sfhk_sample_initial(const sfhk_problem* probs, int32_t n_prob,
                                const uint64_t* n_per_prob, const uint64_t* seeds,
                                const uint64_t* first_index, const sfhk_ensemble* ens,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Propagate every live trajectory of `ens` from its birth step to t_N with
 * classical RK4 (Sec. II.A Hamilton's equations in the Eq. 7 potential plus
 * the laser), its 6x6 monodromy matrix, the action S, the HK prefactor
 * C = sqrt(det R) (continued branch) and the coherent-state recombination
 * amplitude a_k = -w C exp(i[S - Ip(t_k - t0) + p0.q0]) <psi0|k_z|p_k,q_k>
 * (Sec. II.A, Eq. 4-6), and ADD sum_j Re a_jk into accum.
 *   accum: device double [sum_P (N_P + 1)], problem P at offset
 *          sum_{Q<P} (N_Q + 1); the caller zeroes it once, calls may add
 *          further ensembles into it.
 *   final_state: NULL or device double [SFHK_FS_COUNT][ens->capacity]: the
 *          record (SFHK_FS_*) of every live slot at the last step it reached.
 *   snapshots: NULL or device double [n_snap][SFHK_FS_COUNT][ens->capacity]:
 *          snapshot s (0 <= s < n_snap) is the same record at grid step
 *          k = s snap_every, written for the live slots with k0 <= k <= the
 *          last step they reach (entries of other slots and steps are left
 *          as they were; the caller fills them if it needs to tell).
 *          n_snap >= 1 and snap_every >= 1 when snapshots is non-null.
 *          Asking for either record runs the one-wavefront-per-pack kernel
 *          that keeps them (same arithmetic as without).
 *   An FP64 launch of at most 128 64-lane packs (ceil(capacity / 64) +
 *   n_prob <= 128) runs one trajectory per 8 lanes (latency form: same
 *   equations, RK4 applied per monodromy column instead of through the RK4
 *   step matrix), and so does the FP64 re-run of the mixed form.
 *   precision: SFHK_FP64 (everything FP64) or SFHK_MIXED: q, p, the
 *          potential and its derivatives, the monodromy matrix and det R in
 *          FP32; S, the root of det R with its branch, the amplitude and the
 *          sum in FP64.  A trajectory whose FP32 monodromy entry exceeds 1e4,
 *          or (c_max > 0) whose |C| passes c_max / 4, is re-run in FP64 from
 *          its birth and deposits from that step on; its records are then
 *          the FP64 ones.  The mixed result's error against FP64 is measured
 *          and stated, not bounded by the call.
 * probs/n_prob must be those given to sfhk_sample_initial for `ens`;
 * workspace: device, >= sfhk_workspace_bytes (or the precision's share
 * counted by sfhk_footprint_bytes for a single problem). */
sfhk_status sfhk_propagate(const sfhk_problem* probs, int32_t n_prob, const sfhk_ensemble* ens,
                           int32_t precision, double* accum, double* final_state,
                           double* snapshots, int32_t n_snap, int32_t snap_every,
                           void* workspace, size_t workspace_bytes, void* stream);

/* sfhk_propagate without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a 32 MiB array of the
 * library in each GPU's memory, reserved when the library is loaded on that
 * GPU and held until the process ends.  Arguments and results as for
 * sfhk_propagate; problem descriptors travel as kernel arguments.  The call
 * allocates no device memory and calls no allocating HIP or library routine.
 * Limits: at most 1024 problems, and at most 32 MiB of workspace need (that
 * of sfhk_propagate at this precision, at most sfhk_workspace_bytes: about
 * 24 B per step and problem plus, for SFHK_MIXED, 8 B per slot); beyond them
 * SFHK_E_NOMEM with a message, before anything is enqueued.  Every call on a
 * GPU uses that GPU's one array and leaves its contents behind: calls that
 * overlap on one GPU (on different streams, or from different threads
 * without ordering) race and give wrong results; calls ordered on one
 * stream do not. */
sfhk_status sfhk_propagate_static(const sfhk_problem* probs, int32_t n_prob,
                                  const sfhk_ensemble* ens, int32_t precision, double* accum,
                                  double* final_state, double* snapshots, int32_t n_snap,
                                  int32_t snap_every, void* stream);

/* Dipole velocity (Sec. II.A, Eq. 4-6): v_k = (2 / n_sampled[P]) accum_k for
 * each problem (n_sampled counts dropped trajectories too).
 * accum, v_out: device double, the accum layout; n_sampled: host [n_prob]. */
sfhk_status sfhk_dipole(const sfhk_problem* probs, int32_t n_prob, const double* accum,
                        const uint64_t* n_sampled, double* v_out, void* stream);

/* Hanning-windowed Fourier transform (Eq. 3):
 * V(w_m) = dt sum_k v_k W_H(t_k) exp(i w_m t_k), t_k = t_first + k dt,
 * W_H = (1 + cos(pi t / tau_H)) / 2 for |t| <= tau_H, else 0;
 * yield_m = w_m^2 |V(w_m)|^2 (Sec. II.A).
 * v: device [n_t]; omega: device [n_omega]; V_re, V_im, yield: device [n_omega]. */
sfhk_status sfhk_spectrum(const double* v, int32_t n_t, double t_first, double dt, double tau_H,
                          const double* omega, int32_t n_omega, double* V_re, double* V_im,
                          double* yield, void* stream);

/* Host only.  log2 of the default zero-padded transform length for n_t
 * samples: the power of two >= 8 n_t (0 for n_t < 1 or n_t > 2^25). */
int32_t sfhk_fft_log2_len(int32_t n_t);

/* Host only.  Device work bytes of sfhk_spectrum_fft at length 2^log2_len
 * (two complex double arrays of that length; 0 outside 1..28). */
size_t sfhk_spectrum_fft_work_bytes(int32_t log2_len);

/* Eq. 3 on the grid of a zero-padded FFT: the windowed dipole
 * x_k = v_k W_H(t_k) (W_H as for sfhk_spectrum; k < n_t, zeros up to
 * L = 2^log2_len), radix-2 passes of the transform with the positive
 * exponent, and for j = 0 .. L/2, w_j = 2 pi j / (L dt):
 * V_j = dt exp(i w_j t_first) sum_k x_k exp(2 pi i j k / L)
 *     = dt sum_k x_k exp(i w_j t_k),
 * the dipole acceleration's spectrum A_j = -i w_j V_j (Sec. II.A: the two
 * forms differ by that factor), yield_j = |A_j|^2 = w_j^2 |V_j|^2 and
 * phase_j = arg A_j.
 *   v: device [n_t]; log2_len: 1..28 with 2^log2_len >= n_t
 *   (sfhk_fft_log2_len gives the default); work: device, >=
 *   sfhk_spectrum_fft_work_bytes(log2_len) bytes, overwritten;
 *   V_re, V_im, yield: device [L/2 + 1]; phase: device [L/2 + 1] or NULL.
 * Errors: SFHK_E_INVALID for bad sizes or pointers, SFHK_E_NOMEM for a
 * small work buffer, before anything is enqueued. */
sfhk_status sfhk_spectrum_fft(const double* v, int32_t n_t, double t_first, double dt,
                              double tau_H, int32_t log2_len, void* work, size_t work_bytes,
                              double* V_re, double* V_im, double* yield, double* phase,
                              void* stream);

/* The dipole acceleration on the step grid (Sec. II.A: the acceleration
 * form of the dipole, whose spectrum is A = -i w V): the time derivative of
 * the windowed dipole x_k = v_k W_H(t_k) taken in the spectrum of the same
 * zero-padded transform as sfhk_spectrum_fft,
 * a_k = (1/L) sum_j (-i w_j) X_j exp(-2 pi i j k / L), k < n_t, with the
 * two-sided frequencies w_j = 2 pi j / (L dt) for j < L/2 and
 * 2 pi (j - L) / (L dt) for j > L/2 (the Nyquist term is dropped).
 *   v, a: device [n_t]; log2_len, work: as for sfhk_spectrum_fft.
 * Errors as for sfhk_spectrum_fft. */
sfhk_status sfhk_acceleration(const double* v, int32_t n_t, double t_first, double dt,
                              double tau_H, int32_t log2_len, void* work, size_t work_bytes,
                              double* a, void* stream);

/* Classical returns of a sampled ensemble (Sec. III.C: long and short
 * trajectories born in successive half-cycles return in the same window):
 * for every live slot the first step k > k0 at which |q_k| < r_return after
 * some earlier step with |q| >= r_return, and |p_k|^2/2 there (the photon
 * energy is that plus I_p); -1 and 0 for slots that never return or are not
 * live.  Only the classical orbit (q, p) is stepped, by the same RK4 as
 * sfhk_propagate.  k_ret, e_ret: device [capacity], indexed by slot;
 * workspace as for sfhk_propagate. */
sfhk_status sfhk_return_steps(const sfhk_problem* probs, int32_t n_prob,
                              const sfhk_ensemble* ens, double r_return, int32_t* k_ret,
                              double* e_ret, void* workspace, size_t workspace_bytes,
                              void* stream);

/* Gabor time-frequency transform of the dipole (Sec. III.C, the analysis of
 * long and short trajectories):
 *   G(t_c, w) = dt sum_k v_k exp(-(t_k - t_c)^2 / (2 sigma^2)) e^{i w t_k},
 * t_k = t_first + k dt, yield w^2 |G|^2.  The paper gives no window width;
 * sigma is the caller's (1/(3 w_laser) is the Python default).  Terms with
 * |t_k - t_c| > 8 sigma (weight < 2e-14) are not summed.
 * v: device [n_t]; t_c: device [n_c]; omega: device [n_omega];
 * G_re, G_im, yield: device [n_c][n_omega] row-major.  n_c or n_omega = 0 is a
 * no-op; sigma and dt must be > 0. */
sfhk_status sfhk_gabor(const double* v, int32_t n_t, double t_first, double dt, double sigma,
                       const double* t_c, int32_t n_c, const double* omega, int32_t n_omega,
                       double* G_re, double* G_im, double* yield, void* stream);

/* ------------------------------------------------------------------ plans
 * A plan runs the whole path -- sampling, packing, propagation, dipole and
 * spectrum -- for a batch of problems (alignments, intensities, CEPs, targets;
 * Eq. 5-6 averaging is a sum over such problems or over sampled axes) with one
 * enqueue, or as one recorded HIP graph.  The plan is a host object that
 * keeps pointers to caller-owned device memory; it allocates no device
 * memory.  Calls on one plan must not overlap. */

/* Launch options of the trajectory kernels (chosen by the autotuner). */
typedef struct {
  int32_t persistent;    /* 0: one wavefront per 64-lane pack, packs in (problem, birth) order;
                            1: a persistent grid pulls packs, longest first, from a device queue */
  int32_t waves_per_cu;  /* persistent grid = 256 CUs x waves_per_cu wavefronts, 1..32 (0: 8) */
  int32_t step_unroll;   /* RK4 steps per loop trip: 1, 2 or 4 (0: 1) */
  int32_t traj_per_lane; /* trajectories per lane: 1 (0: 1).  FP64: the state of one
                            trajectory fills the register budget of two wavefronts per SIMD.
                            Mixed: two FP32 trajectories per lane would pay only through
                            packed FP32 arithmetic (two lanes' worth per instruction), which
                            the library does not emit: some packed-FP32 forms have given
                            silently wrong results now and then */
  int32_t lanes_per_traj; /* lanes per trajectory of the FP64 re-run of trajectories the mixed
                            form hands over: 1, or 8 for the latency form (one monodromy column
                            per lane); 0: 8 */
} sfhk_tuning;

typedef struct sfhk_plan sfhk_plan;

/* Host only.  Device workspace bytes of a plan. */
size_t sfhk_plan_workspace_bytes(const sfhk_problem* probs, int32_t n_prob,
                                 const uint64_t* n_per_prob);

/* Create a plan and enqueue its set-up (problem tables) on `stream`.
 *   probs, n_per_prob, seeds, first_index: host [n_prob], as sfhk_sample_initial;
 *   precision: SFHK_FP64 or SFHK_MIXED (as for sfhk_propagate); tuning: NULL
 *   for the defaults;
 *   spectra on each problem's harmonic grid w_m = m h_step w_laser, m < n_omega;
 *   ens: device ensemble, capacity >= sum(n_per_prob);
 *   workspace: device, >= sfhk_plan_workspace_bytes;
 *   accum, v: device double [sum_P (N_P + 1)] (accum layout of sfhk_propagate);
 *   V_re, V_im, yield: device double [n_prob][n_omega].
 * Every run overwrites accum, v and the spectra (v = 2 accum / n_per_prob[P]). */
sfhk_status sfhk_plan_create(const sfhk_problem* probs, int32_t n_prob,
                             const uint64_t* n_per_prob, const uint64_t* seeds,
                             const uint64_t* first_index, int32_t precision,
                             const sfhk_tuning* tuning, double h_step, int32_t n_omega,
                             const sfhk_ensemble* ens, void* workspace, size_t workspace_bytes,
                             double* accum, double* v, double* V_re, double* V_im, double* yield,
                             void* stream, sfhk_plan** plan);

/* Enqueue the whole path on `stream`. */
sfhk_status sfhk_plan_run(sfhk_plan* plan, void* stream);

/* Record sfhk_plan_run into a HIP graph (stream must not be the null stream);
 * nothing is executed.  Replaces an earlier recording. */
sfhk_status sfhk_plan_capture(sfhk_plan* plan, void* stream);

/* Launch the recorded graph on `stream` (SFHK_E_INVALID if none). */
sfhk_status sfhk_plan_replay(sfhk_plan* plan, void* stream);

/* Measurement: durations in ms of the trajectory kernel (ms[0]) and, for
 * SFHK_MIXED, of the FP64 re-run of the trajectories it handed over (ms[1];
 * 0 for SFHK_FP64) in the last sfhk_plan_run of this plan, from HIP events
 * the run records around them on its stream.  Recordings and replays record
 * none.  The run must have completed; SFHK_E_INVALID if the plan never ran. */
sfhk_status sfhk_plan_kernel_ms(sfhk_plan* plan, float ms[2]);

/* Release the plan, its graph and its events (host resources only). */
void sfhk_plan_destroy(sfhk_plan* plan);

/* ---------------------------------------------------------------- serving
 * Time-sliced propagation for continuous batching of spectrum requests.  A
 * request (one problem, its trajectory count and seed) owns a contiguous
 * device buffer (its share of the caller's serving pool) and one slot of a
 * device request table.  sfhk_serve_window advances any set of admitted
 * requests by a window of RK4 steps in one launch; the trajectory state stays
 * on the device between windows, so requests can be admitted and retired
 * between any two windows while others are in flight.  A request whose
 * windows have covered steps 0..N is finalised (dipole and spectrum).
 * Ownership: the caller owns the pool, the table and every request buffer;
 * the library keeps no pointer between calls except those it writes into the
 * device table.  Calls enqueue on `stream` and return at once; a buffer or
 * slot may be reused once the work that used it has completed on the stream.
 * Errors: a bad argument returns SFHK_E_INVALID, a buffer below the request's
 * footprint SFHK_E_NOMEM, a window of more than 2^32 work-items
 * SFHK_E_UNSUPPORTED, all before anything is enqueued; a launch failure
 * returns SFHK_E_DEVICE. */

/* Host only.  Device bytes of one request's buffer (its admission footprint). */
size_t sfhk_request_bytes(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega);

/* Host only.  Byte offsets, inside the request buffer, of its results:
 * v [N+1], V_re [n_omega], V_im [n_omega], yield [n_omega] (all double). */
sfhk_status sfhk_request_layout(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega,
                                size_t offsets[4]);

/* Host only.  Bytes of a device request table with max_requests slots. */
size_t sfhk_request_table_bytes(int32_t max_requests);

/* Admit a request into slot `slot` (< table_slots) of the device request table
 * `table` (sfhk_request_table_bytes(table_slots) bytes): lay out its buffers in `buffer`
 * (device, >= sfhk_request_bytes), and enqueue its field table, the sampling
 * of trajectories first_index .. first_index + n_traj - 1 under `seed`
 * (as sfhk_sample_initial), their packing and the zeroing of its dipole
 * accumulator.  Spectrum grid: w_m = m h_step w_laser, m < n_omega. */
sfhk_status sfhk_request_init(const sfhk_problem* p, uint64_t n_traj, uint64_t seed,
                              uint64_t first_index, double h_step, int32_t n_omega,
                              void* buffer, size_t buffer_bytes, void* table, int32_t table_slots,
                              int32_t slot, void* stream);

/* Advance n admitted requests by one window each: request slots[i] over its
 * steps [k_from[i], k_to[i]); n_traj[i] is its trajectory count (a larger
 * value only launches idle wavefronts, a smaller one drops packs).  The
 * launch covers pack group `group` of every request: its packs group,
 * group + n_groups, ... (0 <= group < n_groups <= 64).  Each pack group of a
 * request advances on its own: its windows must be launched in order, without
 * gaps, starting at 0, so different groups may be on different streams.  The
 * same physics as sfhk_propagate in FP64 (Sec. II.A; Eq. 4-6). */
sfhk_status sfhk_serve_window(void* table, int32_t table_slots, int32_t n, const int32_t* slots,
                              const uint64_t* n_traj, const int32_t* k_from, const int32_t* k_to,
                              int32_t group, int32_t n_groups, void* stream);

/* Advance one admitted request (slot `slot`, admitted by sfhk_request_init
 * with the same p, n_traj, n_omega and buffer) over its whole pulse, steps
 * 0..N, in one launch of the FP64 kernel of sfhk_propagate (one wavefront per
 * 64-lane pack): the same result as sfhk_serve_window over [0, N+1) for this
 * request, for a request that runs alone from its first step to its last.
 * The state kept between windows is not written, so no window may follow;
 * sfhk_request_finalize comes next.  Sec. II.A; Eq. 4-6. */
sfhk_status sfhk_request_run(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega,
                             void* buffer, size_t buffer_bytes, void* table, int32_t table_slots,
                             int32_t slot, void* stream);

/* Dipole (v = 2 accum / n_traj) and spectrum of a request whose windows have
 * covered steps 0..N; results at sfhk_request_layout's offsets. */
sfhk_status sfhk_request_finalize(const sfhk_problem* p, int32_t n_omega, void* table,
                                  int32_t table_slots, int32_t slot, void* stream);

#ifdef __cplusplus
}
#endif
#endif
