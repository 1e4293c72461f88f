// Internal declarations shared by the HIP translation units of libsfhk.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sfhk.h"

namespace sfhk {

constexpr int kWave = 64;
constexpr double kPi = 3.14159265358979323846;

// Coefficients of one RK4 step of length h: h/2, h/6 and the step matrix's
// h^2/6, h^3/12, h^4/24.  Computed on the host (FP64, and from the FP32 h in
// FP32) with the same operations a kernel would use: a division in a step
// loop costs about ten VALU instructions.
template <typename T>
struct RkCoef {
  T h, hh, h6, c2, c3, c4;
};

// Per-problem constants, derived once on the host and read by every kernel
// through wave-uniform (scalar) loads.
struct Desc {
  // laser and time grid (Sec. II.D pulse, grid t_k = t_first + k dt)
  double omega, E0, tau, cep, dt, t_first;
  int32_t N, align_kind, align_m, n_gto;
  int32_t screened, ionization;
  // target (Eq. 7) and coherent state
  double half_R, Ip, gamma, inv_gamma, inv_gamma2, half_inv_gamma;
  double Zinf[2], dZ[2], alpha[2], eps2[2];
  double adZ[2], a2dZ[2];  // alpha dZ and alpha^2 dZ
  float fZinf[2], fdZ[2], falpha[2], feps2[2];  // the same, rounded to FP32
  float fadZ[2], fa2dZ[2];
  // sampling (first-order tunnel exit and amplitude weight)
  double sigma, w_cut, kappa, wpow, kcube3, inv_E0;
  double nfix[3];
  uint64_t seed, first_index;
  // offsets into shared buffers
  uint64_t field_off;  // doubles: E(t_k) at 2k, E(t_k + dt/2) at 2k + 1
  uint64_t acc_off;    // accum / histogram bin of step 0
  uint64_t slot_off, n_slots;
  // GTO primitives (ionisation matrix element): l | centre << 1 (centre 0
  // at +R/2 n), 1/(2a) and c (2a)^{-3/2}
  double g_ion[SFHK_MAX_GTO], g_i2a[SFHK_MAX_GTO];
  int32_t g_l[SFHK_MAX_GTO];
  // Recombination shells: the primitives of one centre and one exponent a
  // share the Gaussian factor of the recombination element.  Shells of
  // centre 0 come first (n_shell0 of them).  Per shell: 1/(4 kappa2) with
  // kappa2 = 1/(4a) + 1/(2 gamma) (half of 1/(2 kappa2)), and the summed
  // normalisations of its s primitives and of its p primitives (the latter
  // times 1/(2a)); a normalisation is c (2a)^{-3/2} (pi gamma)^{-3/4}
  // (pi/kappa2)^{3/2}.
  int32_t n_shell, n_shell0;
  double sh_inv4k[SFHK_MAX_GTO];
  double sh_ns[SFHK_MAX_GTO], sh_np[SFHK_MAX_GTO];
  double g_inv4k_min;  // smallest 1/(4 kappa2) over the shells
  double c_max2;       // prefactor cap squared (0: none)
  RkCoef<double> rk;   // RK4 coefficients of h = dt
  RkCoef<float> frk;   // the same for the FP32 h = (float) dt
};

template <typename T> __host__ __device__ inline const RkCoef<T>& rk_coef(const Desc& d);
template <> __host__ __device__ inline const RkCoef<double>& rk_coef<double>(const Desc& d) {
  return d.rk;
}
template <> __host__ __device__ inline const RkCoef<float>& rk_coef<float>(const Desc& d) {
  return d.frk;
}

// True if any problem is born by the saddle-point step (it selects the
// sampler with that code).
inline bool any_saddle(const Desc* descs, int n) {
  for (int i = 0; i < n; ++i)
    if (descs[i].ionization != SFHK_ION_FIRST_ORDER) return true;
  return false;
}

// Device pointers of the ensemble, passed by value to kernels.
struct EnsPtrs {
  int32_t* k0;
  int32_t* prob;
  double *qx, *qy, *qz, *px, *py, *pz, *w, *nx, *ny, *nz, *dph;
  uint32_t *order, *live_start, *live_count, *pack_start;
};

// Device workspace carve-up (all offsets 256-byte aligned).
struct Workspace {
  Desc* descs;
  uint64_t* slot_off;   // [n_prob + 1]
  double* field;        // [sum 2 (N_P + 1)]
  uint32_t* hist;       // [n_bins + 1] counting-sort bins (then bin starts)
  uint32_t* cursor;     // [n_bins + 1]
  int32_t* redo;        // [capacity] mixed precision: FP64 re-run from this step (-1: none)
  uint32_t* order2;     // [capacity] packs of the FP64 re-run
  uint32_t* runs2;      // [3 n_prob + 1] live_start, live_count, pack_start of the re-run
  size_t bytes;
};

struct Layout {
  uint64_t n_bins = 0;        // sum (N_P + 1)
  uint64_t n_field = 0;       // sum 2 (N_P + 1)
  uint64_t n_slots = 0;       // sum n_per_prob (sampling) or capacity
  size_t bytes = 0;
  size_t off_descs = 0, off_slot = 0, off_field = 0, off_hist = 0, off_cursor = 0;
  size_t off_redo = 0, off_order2 = 0, off_runs2 = 0;
  // plans only: pack queues
  uint32_t max_packs = 0, n_len = 0;
  size_t off_qkeys = 0, off_qhist = 0, off_qcursor = 0, off_queue = 0, off_queue2 = 0;
  size_t off_counter = 0;
};

// Outputs of the counting sort into 64-lane packs.
struct PackOut {
  uint32_t *order, *live_start, *live_count, *pack_start;
};

// The mixed-precision kernel hands a trajectory to the FP64 kernel once an
// entry of its FP32 monodromy matrix exceeds this bound (FP32 rounding is
// then amplified past ~6e-4 relative).
constexpr float kMixedFlagNorm = 1.0e4f;
// With a prefactor cap set, it also hands a trajectory over once |C| (from
// the FP32 monodromy matrix) passes a quarter of the cap, so that the step at
// which the cap stops the trajectory is decided in FP64, as in the FP64 run.
constexpr double kMixedCapHandover2 = 1.0 / 16.0;

// launchers (setup_kernels.hip)
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_field(const Desc* descs, int n_prob, double* field, uint64_t n_field,
                        hipStream_t s);
hipError_t launch_sample(const Desc* descs, int n_prob, const uint64_t* slot_off,
                         uint64_t n_slots, const double* field, EnsPtrs e, uint32_t* hist,
                         bool saddle, hipStream_t s);
// Counts slot i (select ? select[i] >= 0 : w[i] > 0) into bin acc_off[prob] + k0.
hipError_t launch_count(const Desc* descs, uint64_t n_slots, EnsPtrs e, const int32_t* select,
                        uint32_t* hist, hipStream_t s);
// Counting sort of the selected slots by (problem, k0, slot) into packs.
hipError_t launch_sort(const Desc* descs, int n_prob, uint64_t n_slots, uint64_t n_bins,
                       uint32_t* hist, uint32_t* cursor, EnsPtrs e, const int32_t* select,
                       PackOut out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, uint64_t n, hipStream_t s);
// Stores one descriptor, passed as a kernel argument, at dst.
hipError_t launch_store_desc(const Desc& d, Desc* dst, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, uint64_t n, hipStream_t s);
hipError_t launch_scale(const double* in, double* out, double scale, uint64_t n, hipStream_t s);
hipError_t launch_returns(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                          uint32_t max_packs, double r_ret, int32_t* k_ret, double* e_ret,
                          hipStream_t s);
hipError_t launch_gabor(const double* v, int n_t, double t_first, double dt, double sigma,
                        const double* t_c, int n_c, const double* omega, int n_omega,
                        double* G_re, double* G_im, double* yield, hipStream_t s);
hipError_t launch_spectrum(const double* v, int n_t, double t_first, double dt, double tau_H,
                           const double* omega, int n_omega, double* V_re, double* V_im,
                           double* yield, hipStream_t s);
// Eq. 3 on the grid of a zero-padded transform of length 2^log2_len (work:
// 2^(log2_len + 1) complex doubles); outputs [2^(log2_len - 1) + 1], phase
// nullable.
hipError_t launch_spectrum_fft(const double* v, int n_t, double t_first, double dt, double tau_H,
                               int log2_len, double2* work, double* V_re, double* V_im,
                               double* yield, double* phase, hipStream_t s);
// The dipole acceleration on the step grid: the derivative of the windowed
// dipole through the same transform, back-transformed; a: [n_t].
hipError_t launch_acceleration_fft(const double* v, int n_t, double t_first, double dt,
                                   double tau_H, int log2_len, double2* work, double* a,
                                   hipStream_t s);
// propagate_f64.hip, propagate_mixed.hip
// Launch form of the trajectory kernels: one wavefront per pack (grid =
// max_packs), or a persistent grid pulling packs from queue[] through an
// atomic counter (zeroed before the launch); U = unroll steps per loop trip.
struct LaunchCfg {
  int persistent = 0;
  int unroll = 1;
  uint32_t grid = 0;
  const uint32_t* queue = nullptr;
  uint32_t* counter = nullptr;
  int pipe_mono = 1;  // latency form: monodromy wavefronts per unit (1 or 2)
};

// Optional per-slot records of a propagation (SFHK_FS_* layout, field-major,
// stride capacity): the final state, and the state at the grid steps
// k = s snap_every (s < n_snap) that the trajectory reaches.  Any record
// selects the one-pack-per-wavefront kernel that keeps them.
struct Records {
  double* final_state = nullptr;  // [SFHK_FS_COUNT][capacity]
  double* snap = nullptr;         // [n_snap][SFHK_FS_COUNT][capacity]
  int32_t n_snap = 0, snap_every = 1;
  uint64_t capacity = 0;
  bool any() const { return final_state != nullptr || snap != nullptr; }
};

// dep_from (nullable, per slot): deposit amplitudes only from that step on.
hipError_t launch_propagate_f64(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                                const int32_t* dep_from, uint32_t max_packs, double* accum,
                                const Records& rec, hipStream_t s, const LaunchCfg& cfg);
// The same FP64 propagation with one trajectory per 8-lane group (latency
// form, propagate_latency.hip): grid 8 max_packs, or with cfg.persistent a
// grid of cfg.grid wavefronts pulling 8-trajectory units of the packs in
// cfg.queue (records need the per-pack grid).
hipError_t launch_propagate_latency(const Desc* descs, int n_prob, const double* field,
                                    EnsPtrs e, const int32_t* dep_from, uint32_t max_packs,
                                    double* accum, const Records& rec, hipStream_t s,
                                    const LaunchCfg& cfg);
// Largest pack count an automatic choice runs in the latency form: eight
// wavefronts per pack, at most one per SIMD of a 256-CU device.
constexpr uint32_t kLatencyMaxPacks = 128;
// redo (per slot, preset to -1): set to the first step left to the FP64 re-run.
hipError_t launch_propagate_mixed(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                                  int32_t* redo, uint32_t max_packs, double* accum,
                                  const Records& rec, hipStream_t s, const LaunchCfg& cfg);
// Pack queue ordered by remaining steps (longest first), ties by pack id:
// queue[max_packs]; keys, hist, cursor: scratch of max_packs, n_len + 1, n_len + 1
// entries with n_len = max_P N_P + 1.
hipError_t launch_pack_queue(const Desc* descs, int n_prob, EnsPtrs e, uint32_t max_packs,
                             uint32_t n_len, uint32_t* keys, uint32_t* hist, uint32_t* cursor,
                             uint32_t* queue, hipStream_t s);
// Batched dipole: v = (2 / n_slots_P) accum over every problem's segment.
hipError_t launch_dipole_batched(const Desc* descs, int n_prob, uint32_t n_kmax,
                                 const double* accum, double* v, hipStream_t s);
// Batched spectrum on each problem's harmonic grid w_m = m h_step w_P,
// m < n_omega; outputs [n_prob][n_omega].
hipError_t launch_spectrum_batched(const Desc* descs, int n_prob, const double* v, double h_step,
                                   int n_omega, double* V_re, double* V_im, double* yield,
                                   hipStream_t s);

}  // namespace sfhk
