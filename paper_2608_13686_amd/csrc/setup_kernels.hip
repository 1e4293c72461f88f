// Field table, initial-condition sampling, counting sort into 64-lane packs,
// dipole normalisation and the windowed Fourier transform.
#include "sfa_step.h"
#include "sfhk_internal.h"

namespace sfhk {
namespace {

constexpr int kBlock = 256;

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_f64_kernel(double* __restrict__ p, double v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One problem descriptor, passed by value, stored to device memory: the
// upload reads no host memory after the launch call returns.
static_assert(sizeof(Desc) <= 3840, "Desc is passed by value as a kernel argument");
__global__ void store_desc_kernel(Desc d, Desc* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

// ---------------------------------------------------------------- field
// E(t) = -dA/dt of A(t) = -(E0/w) cos^2(pi t/tau) sin(w t + cep) for
// |t| <= tau/2, zero outside (sin^2 pulse of Sec. II.D / III.A, centred at
// t = 0).  Table entries 2k and 2k+1 hold E(t_k) and E(t_k + dt/2).
__device__ double field_at(const Desc& d, double t) {
  if (fabs(t) > 0.5 * d.tau) return 0.0;
  double env = cos(kPi * t / d.tau);
  double ph = d.omega * t + d.cep;
  return d.E0 * env * env * cos(ph) -
         (d.E0 * kPi / (d.omega * d.tau)) * sin(2.0 * kPi * t / d.tau) * sin(ph);
}

__global__ void field_kernel(const Desc* __restrict__ descs, double* __restrict__ field) {
  const Desc& d = descs[blockIdx.y];
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > d.N) return;
  double tk = d.t_first + (double)k * d.dt;
  field[d.field_off + 2 * (uint64_t)k] = field_at(d, tk);
  field[d.field_off + 2 * (uint64_t)k + 1] = field_at(d, tk + 0.5 * d.dt);
}

// -------------------------------------------------------------- Philox
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of two 32x32 -> 64-bit products and a word permutation, with
// the two key words advanced by Weyl increments between rounds.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ inline double open01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

__device__ inline int find_problem(const uint64_t* __restrict__ off, int n_prob, uint64_t i) {
  int lo = 0, hi = n_prob;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// One thread per ensemble slot.  Initial conditions at the tunnel exit for
// the first-order expansion of the SFA saddle-point equation (Eq. 2) about
// the birth time: p0 = (sigma g1, sigma g2, 0), q0 = -(Ip + p0^2/2)/E(t0) z,
// weight w = (F0/F)^{(2/kappa-1)/2} exp(-(kappa^3/3)(1/F - 1/F0)), F = |E(t0)|,
// dropped (w = 0) below w_cut; axis fixed or cos^(2m)-distributed (Eq. 6).
// Saddle = false is the sampler for first-order problems only: it carries no
// saddle-point code and so no per-lane stack, which every dispatch of a
// kernel with one would have to be given.
template <bool Saddle>
__global__ void sample_kernel(const Desc* __restrict__ descs, int n_prob,
                              const uint64_t* __restrict__ slot_off, uint64_t n_slots,
                              const double* __restrict__ field, EnsPtrs e,
                              uint32_t* __restrict__ hist) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  int P = find_problem(slot_off, n_prob, i);
  const Desc& d = descs[P];
  uint64_t j = d.first_index + (i - slot_off[P]);
  uint32_t klo = (uint32_t)d.seed, khi = (uint32_t)(d.seed >> 32);
  U4 x = philox4x32_10(U4{(uint32_t)j, (uint32_t)(j >> 32), 0u, 0u}, klo, khi);
  U4 y = philox4x32_10(U4{(uint32_t)j, (uint32_t)(j >> 32), 0u, 1u}, klo, khi);

  int32_t k0 = (int32_t)(((uint64_t)x.x * (uint64_t)d.N) >> 32);
  double r = sqrt(-2.0 * log(open01(x.y)));
  double u2 = open01(x.z);
  double px = d.sigma * r * cos(2.0 * kPi * u2);
  double py = d.sigma * r * sin(2.0 * kPi * u2);

  double nx, ny, nz;
  if (d.align_kind == SFHK_ALIGN_FIXED) {
    nx = d.nfix[0];
    ny = d.nfix[1];
    nz = d.nfix[2];
  } else {
    double c = 2.0 * open01(x.w) - 1.0;
    double cb = (c < 0.0 ? -1.0 : 1.0) * pow(fabs(c), 1.0 / (2.0 * d.align_m + 1.0));
    double sb = sqrt(1.0 - cb * cb);
    double al = 2.0 * kPi * open01(y.x);
    nx = sb * cos(al);
    ny = sb * sin(al);
    nz = cb;
  }

  double E = field[d.field_off + 2 * (uint64_t)k0];
  double F = fabs(E);
  double w = 0.0, qz = 0.0, pz = 0.0, dph = 0.0;
  if (Saddle && d.ionization != SFHK_ION_FIRST_ORDER) {
    const double nn[3] = {nx, ny, nz};
    SfaBirth b;
    if (sfa_birth(d, d.t_first + (double)k0 * d.dt, px, py, nn, b)) {
      w = b.w;
      qz = b.q0z;
      pz = b.kz;
      dph = b.dph;
    }
  } else if (F > 0.0) {
    w = pow(d.E0 / F, d.wpow) * exp(-d.kcube3 * (1.0 / F - d.inv_E0));
    qz = -(d.Ip + 0.5 * (px * px + py * py)) / E;
  }
  if (!(w >= d.w_cut)) {
    w = 0.0;
    dph = 0.0;
  }

  e.k0[i] = k0;
  e.prob[i] = P;
  e.qx[i] = 0.0;
  e.qy[i] = 0.0;
  e.qz[i] = qz;
  e.px[i] = px;
  e.py[i] = py;
  e.pz[i] = pz;
  e.dph[i] = dph;
  e.w[i] = w;
  e.nx[i] = nx;
  e.ny[i] = ny;
  e.nz[i] = nz;
  if (w > 0.0) atomicAdd(&hist[d.acc_off + (uint64_t)k0], 1u);
}

// ------------------------------------------------------ counting sort
// Exclusive scan of the bin counts in place (single block); entry n holds the
// total.  Each thread scans one contiguous chunk.
__global__ void __launch_bounds__(1024) scan_bins_kernel(uint32_t* __restrict__ h, uint64_t n) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  uint64_t chunk = (n + 1023) / 1024;
  uint64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
  uint32_t s = 0;
  for (uint64_t i = b; i < e; ++i) s += h[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive prefix of this chunk
  for (uint64_t i = b; i < e; ++i) {
    uint32_t c = h[i];
    h[i] = run;
    run += c;
  }
  if (t == 1023) h[n] = part[1023];
}

// Per-problem live runs and pack prefix (pack = 64 consecutive live slots).
__global__ void problem_runs_kernel(const Desc* __restrict__ descs, int n_prob,
                                    const uint32_t* __restrict__ start, PackOut o) {
  if (threadIdx.x != 0) return;
  uint32_t packs = 0;
  for (int P = 0; P < n_prob; ++P) {
    const Desc& d = descs[P];
    uint32_t s0 = start[d.acc_off], s1 = start[d.acc_off + (uint64_t)d.N + 1];
    o.live_start[P] = s0;
    o.live_count[P] = s1 - s0;
    o.pack_start[P] = packs;
    packs += (s1 - s0 + kWave - 1) / kWave;
  }
  o.pack_start[n_prob] = packs;
}

__device__ __forceinline__ bool selected(const EnsPtrs& e, const int32_t* select, uint64_t i) {
  return select ? select[i] >= 0 : e.w[i] > 0.0;
}

__global__ void count_kernel(const Desc* __restrict__ descs, uint64_t n_slots, EnsPtrs e,
                             const int32_t* __restrict__ select, uint32_t* __restrict__ hist) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots || !selected(e, select, i)) return;
  atomicAdd(&hist[descs[e.prob[i]].acc_off + (uint64_t)e.k0[i]], 1u);
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int32_t v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void copy_u32_kernel(const uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void scatter_kernel(const Desc* __restrict__ descs, uint64_t n_slots,
                               uint32_t* __restrict__ cursor, EnsPtrs e,
                               const int32_t* __restrict__ select, uint32_t* __restrict__ order) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots || !selected(e, select, i)) return;
  const Desc& d = descs[e.prob[i]];
  uint32_t pos = atomicAdd(&cursor[d.acc_off + (uint64_t)e.k0[i]], 1u);
  order[pos] = (uint32_t)i;
}

// Within each bin the scatter order is arbitrary; sort every bin's slots
// ascending so that the pack layout is deterministic.  The bitonic network in
// its all-ascending form (the first step of each merge compares mirror
// images) puts the smaller value at the lower index in every compare-exchange,
// so entries past a bin's end act as +infinity and their exchanges are
// skipped, with no padding: O(n log^2 n) work per bin at any occupancy.
// Each thread of a block owns one bin; the block's waves take its bins of
// 2..kSortWave entries one at a time, each sorted by one wave in its own LDS
// region (LDS operations of a wave complete in issue order, so a compiler
// fence between steps suffices); larger bins are then sorted one after the
// other by the whole block in place in global memory, a barrier between
// steps.
constexpr uint32_t kSortWave = 2048;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sorts a[0, n) by the threads t0, t0 + stride, ... of the group that calls
// it; sync() separates the steps.
template <typename Sync>
__device__ void bitonic_sort(uint32_t* a, uint64_t n, uint32_t t0, uint32_t stride, Sync sync) {
  uint64_t m = 1;
  while (m < n) m <<= 1;
  for (uint64_t k = 2; k <= m; k <<= 1) {
    for (uint64_t j = k >> 1; j > 0; j >>= 1) {
      for (uint64_t t = t0; t < m / 2; t += stride) {
        // the t-th index with bit j clear, and its partner above it
        const uint64_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const uint64_t l = j == k >> 1 ? i ^ (k - 1) : i + j;
        if (l < n) {
          const uint32_t x = a[i], y = a[l];
          if (x > y) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      sync();
    }
  }
}

__global__ void __launch_bounds__(kBlock) sort_bins_kernel(const uint32_t* __restrict__ start,
                                                           uint64_t n_bins, uint32_t* order) {
  __shared__ uint32_t buf[kBlock / kWave][kSortWave];
  __shared__ uint32_t big_lo[kBlock], big_n[kBlock];
  __shared__ uint32_t n_big;
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) n_big = 0;
  __syncthreads();
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t lo = 0, n = 0;
  if (b < n_bins) {
    lo = start[b];
    n = start[b + 1] - lo;
  }
  if (n > kSortWave) {
    const uint32_t at = atomicAdd(&n_big, 1u);
    big_lo[at] = lo;
    big_n[at] = n;
  }
  uint64_t todo = __ballot(n >= 2 && n <= kSortWave);
  uint32_t* a = buf[wave];
  while (todo) {
    const int src = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const uint32_t blo = __shfl(lo, src), bn = __shfl(n, src);
    for (uint32_t t = lane; t < bn; t += kWave) a[t] = order[blo + t];
    wave_fence();
    bitonic_sort(a, bn, lane, kWave, wave_fence);
    for (uint32_t t = lane; t < bn; t += kWave) order[blo + t] = a[t];
    wave_fence();
  }
  __syncthreads();
  const uint32_t nb = n_big;
  for (uint32_t k = 0; k < nb; ++k) {
    const uint32_t blo = big_lo[k], bn = big_n[k];
    bitonic_sort(order + blo, bn, threadIdx.x, kBlock, [] { __syncthreads(); });
  }
}

// ------------------------------------------------------------- dipole
__global__ void scale_kernel(const double* __restrict__ in, double* __restrict__ out, double s,
                             uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = s * in[i];
}

// ----------------------------------------------------------- spectrum
// One block per frequency; each thread sums a strided subset of the time
// grid, then a fixed-order tree reduction (deterministic).
__global__ void __launch_bounds__(kBlock) spectrum_kernel(const double* __restrict__ v, int n_t,
                                                          double t_first, double dt,
                                                          double tau_H,
                                                          const double* __restrict__ omega,
                                                          double* __restrict__ V_re,
                                                          double* __restrict__ V_im,
                                                          double* __restrict__ yield) {
  __shared__ double sr[kBlock], si[kBlock];
  const int m = blockIdx.x;
  const double w = omega[m];
  double ar = 0.0, ai = 0.0;
  for (int k = threadIdx.x; k < n_t; k += kBlock) {
    double t = t_first + (double)k * dt;
    double wh = fabs(t) <= tau_H ? 0.5 * (1.0 + cos(kPi * t / tau_H)) : 0.0;
    double s, c;
    sincos(w * t, &s, &c);
    double x = v[k] * wh;
    ar += x * c;
    ai += x * s;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sr[threadIdx.x] += sr[threadIdx.x + off];
      si[threadIdx.x] += si[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double re = dt * sr[0], im = dt * si[0];
    V_re[m] = re;
    V_im[m] = im;
    yield[m] = w * w * (re * re + im * im);
  }
}

// ------------------------------------------------------------ pack queue
// Key of a pack: (n_len - 1) - remaining steps of its first (earliest-born)
// lane, so that an ascending counting sort puts the longest packs first.
__global__ void pack_keys_kernel(const Desc* __restrict__ descs, int n_prob, EnsPtrs e,
                                 uint32_t max_packs, uint32_t n_len, uint32_t* __restrict__ keys,
                                 uint32_t* __restrict__ hist) {
  const uint32_t pack = blockIdx.x * blockDim.x + threadIdx.x;
  if (pack >= max_packs || pack >= e.pack_start[n_prob]) return;
  int lo = 0, hi = n_prob;  // pack_start[lo] <= pack < pack_start[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (e.pack_start[mid] <= pack) lo = mid; else hi = mid;
  }
  const uint32_t first = e.order[e.live_start[lo] + (pack - e.pack_start[lo]) * kWave];
  const uint32_t remaining = (uint32_t)(descs[lo].N - e.k0[first]);
  const uint32_t key = (n_len - 1) - remaining;
  keys[pack] = key;
  atomicAdd(&hist[key], 1u);
}

__global__ void pack_scatter_kernel(const EnsPtrs e, int n_prob, uint32_t max_packs,
                                    const uint32_t* __restrict__ keys,
                                    uint32_t* __restrict__ cursor, uint32_t* __restrict__ queue) {
  const uint32_t pack = blockIdx.x * blockDim.x + threadIdx.x;
  if (pack >= max_packs || pack >= e.pack_start[n_prob]) return;
  queue[atomicAdd(&cursor[keys[pack]], 1u)] = pack;
}

// ---------------------------------------------------- batched dipole
__global__ void dipole_batched_kernel(const Desc* __restrict__ descs,
                                      const double* __restrict__ accum, double* __restrict__ v) {
  const Desc& d = descs[blockIdx.y];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > d.N) return;
  const double sc = d.n_slots > 0 ? 2.0 / (double)d.n_slots : 0.0;
  v[d.acc_off + k] = sc * accum[d.acc_off + k];
}

// -------------------------------------------------- batched spectrum
// Problem blockIdx.y on its harmonic grid w_m = m h_step w, Hanning window
// over |t| <= tau/2; one block per (m, problem), fixed-order reduction.
__global__ void __launch_bounds__(kBlock) spectrum_batched_kernel(const Desc* __restrict__ descs,
                                                                  const double* __restrict__ v,
                                                                  double h_step, int n_omega,
                                                                  double* __restrict__ V_re,
                                                                  double* __restrict__ V_im,
                                                                  double* __restrict__ yield) {
  __shared__ double sr[kBlock], si[kBlock];
  const Desc& d = descs[blockIdx.y];
  const int m = blockIdx.x;
  const double w = (double)m * h_step * d.omega;
  const double tau_H = 0.5 * d.tau;
  const double* vp = v + d.acc_off;
  double ar = 0.0, ai = 0.0;
  for (int k = threadIdx.x; k <= d.N; k += kBlock) {
    const double t = d.t_first + (double)k * d.dt;
    const double wh = fabs(t) <= tau_H ? 0.5 * (1.0 + cos(kPi * t / tau_H)) : 0.0;
    double sn, cs;
    sincos(w * t, &sn, &cs);
    const double x = vp[k] * wh;
    ar += x * cs;
    ai += x * sn;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sr[threadIdx.x] += sr[threadIdx.x + off];
      si[threadIdx.x] += si[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double re = d.dt * sr[0], im = d.dt * si[0];
    const size_t o = (size_t)blockIdx.y * n_omega + m;
    V_re[o] = re;
    V_im[o] = im;
    yield[o] = w * w * (re * re + im * im);
  }
}

inline unsigned blocks_for(uint64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// --------------------------------------------------------------- Gabor
// One workgroup per window centre t_c.  The window-weighted signal
// u_k = v_k exp(-(t_k - t_c)^2 / (2 sigma^2)) over |t_k - t_c| <= 8 sigma
// (the rest is below 2e-14 of the peak weight) is staged through LDS in
// chunks; each thread sums u_k e^{i w t_k} for its frequencies, advancing
// e^{i w t_k} by the rotation e^{i w dt} and re-taking it exactly every 64
// steps (rounding growth below 64 ulp).
constexpr int kGaborChunk = 4096;

__global__ void __launch_bounds__(kBlock) gabor_kernel(const double* __restrict__ v, int n_t,
                                                       double t_first, double dt, double sigma,
                                                       const double* __restrict__ t_c,
                                                       const double* __restrict__ omega,
                                                       int n_omega, double* __restrict__ G_re,
                                                       double* __restrict__ G_im,
                                                       double* __restrict__ yield) {
  __shared__ double u[kGaborChunk];
  const int a = blockIdx.x;
  const double tc = t_c[a];
  const double half = 8.0 * sigma;
  // clamp in floating point first: a far-away centre must not overflow the cast
  const double flo = fmax(ceil((tc - half - t_first) / dt), 0.0);
  const double fhi = fmin(floor((tc + half - t_first) / dt), (double)(n_t - 1));
  const long long klo = (long long)fmin(flo, (double)n_t);
  const long long khi = (long long)fmax(fhi, -1.0);
  const double inv_s = 1.0 / sigma;
  // each thread keeps the partial sums of up to 8 frequencies
  constexpr int kPer = 8;
  for (int b0 = 0; b0 < n_omega; b0 += kBlock * kPer) {
    double sr[kPer], si[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) sr[j] = si[j] = 0.0;
    for (long long c0 = klo; c0 <= khi; c0 += kGaborChunk) {
      const int len = (int)((khi - c0 + 1) < kGaborChunk ? (khi - c0 + 1) : kGaborChunk);
      __syncthreads();
      for (int i = threadIdx.x; i < len; i += kBlock) {
        const double t = t_first + (double)(c0 + i) * dt;
        const double x = (t - tc) * inv_s;
        u[i] = v[c0 + i] * exp(-0.5 * x * x);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int b = b0 + j * kBlock + threadIdx.x;
        if (b >= n_omega || len <= 0) continue;
        const double w = omega[b];
        double rs, rc;
        sincos(w * dt, &rs, &rc);
        double zr = 0.0, zi = 0.0, ar = 0.0, ai = 0.0;
        for (int i = 0; i < len; ++i) {
          if ((i & 63) == 0) {
            sincos(w * (t_first + (double)(c0 + i) * dt), &zi, &zr);
          } else {
            const double nr = zr * rc - zi * rs;
            zi = zr * rs + zi * rc;
            zr = nr;
          }
          ar += u[i] * zr;
          ai += u[i] * zi;
        }
        sr[j] += ar;
        si[j] += ai;
      }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int b = b0 + j * kBlock + threadIdx.x;
      if (b >= n_omega) continue;
      const double gr = dt * sr[j], gi = dt * si[j], w = omega[b];
      const size_t o = (size_t)a * n_omega + b;
      G_re[o] = gr;
      G_im[o] = gi;
      yield[o] = w * w * (gr * gr + gi * gi);
    }
  }
}

}  // namespace

hipError_t launch_store_desc(const Desc& d, Desc* dst, hipStream_t s) {
  hipLaunchKernelGGL(store_desc_kernel, dim3(1), dim3(1), 0, s, d, dst);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_field(const Desc* descs, int n_prob, double* field, uint64_t n_kmax,
                        hipStream_t s) {
  // n_kmax: max_P (N_P + 1)
  hipLaunchKernelGGL(field_kernel, dim3(blocks_for(n_kmax, kBlock), n_prob), dim3(kBlock), 0, s,
                     descs, field);
  return hipGetLastError();
}

hipError_t launch_sample(const Desc* descs, int n_prob, const uint64_t* slot_off,
                         uint64_t n_slots, const double* field, EnsPtrs e, uint32_t* hist,
                         bool saddle, hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  if (saddle)
    hipLaunchKernelGGL(sample_kernel<true>, dim3(blocks_for(n_slots, kBlock)), dim3(kBlock), 0, s,
                       descs, n_prob, slot_off, n_slots, field, e, hist);
  else
    hipLaunchKernelGGL(sample_kernel<false>, dim3(blocks_for(n_slots, kBlock)), dim3(kBlock), 0,
                       s, descs, n_prob, slot_off, n_slots, field, e, hist);
  return hipGetLastError();
}

hipError_t launch_count(const Desc* descs, uint64_t n_slots, EnsPtrs e, const int32_t* select,
                        uint32_t* hist, hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(count_kernel, dim3(blocks_for(n_slots, kBlock)), dim3(kBlock), 0, s, descs,
                     n_slots, e, select, hist);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_sort(const Desc* descs, int n_prob, uint64_t n_slots, uint64_t n_bins,
                       uint32_t* hist, uint32_t* cursor, EnsPtrs e, const int32_t* select,
                       PackOut out, hipStream_t s) {
  hipLaunchKernelGGL(scan_bins_kernel, dim3(1), dim3(1024), 0, s, hist, n_bins);
  hipLaunchKernelGGL(problem_runs_kernel, dim3(1), dim3(64), 0, s, descs, n_prob, hist, out);
  hipLaunchKernelGGL(copy_u32_kernel, dim3(blocks_for(n_bins + 1, kBlock)), dim3(kBlock), 0, s,
                     hist, cursor, n_bins + 1);
  if (n_slots > 0)
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n_slots, kBlock)), dim3(kBlock), 0, s,
                       descs, n_slots, cursor, e, select, out.order);
  if (n_bins > 0)
    hipLaunchKernelGGL(sort_bins_kernel, dim3(blocks_for(n_bins, kBlock)), dim3(kBlock), 0, s, hist,
                     n_bins, out.order);
  return hipGetLastError();
}

hipError_t launch_pack_queue(const Desc* descs, int n_prob, EnsPtrs e, uint32_t max_packs,
                             uint32_t n_len, uint32_t* keys, uint32_t* hist, uint32_t* cursor,
                             uint32_t* queue, hipStream_t s) {
  hipError_t err = launch_fill_u32(hist, 0u, (uint64_t)n_len + 1, s);
  if (err != hipSuccess || max_packs == 0) return err;
  hipLaunchKernelGGL(pack_keys_kernel, dim3(blocks_for(max_packs, kBlock)), dim3(kBlock), 0, s,
                     descs, n_prob, e, max_packs, n_len, keys, hist);
  hipLaunchKernelGGL(scan_bins_kernel, dim3(1), dim3(1024), 0, s, hist, (uint64_t)n_len);
  hipLaunchKernelGGL(copy_u32_kernel, dim3(blocks_for((uint64_t)n_len + 1, kBlock)), dim3(kBlock),
                     0, s, hist, cursor, (uint64_t)n_len + 1);
  hipLaunchKernelGGL(pack_scatter_kernel, dim3(blocks_for(max_packs, kBlock)), dim3(kBlock), 0, s,
                     e, n_prob, max_packs, keys, cursor, queue);
  hipLaunchKernelGGL(sort_bins_kernel, dim3(blocks_for(n_len, kBlock)), dim3(kBlock), 0, s, hist,
                     (uint64_t)n_len, queue);
  return hipGetLastError();
}

hipError_t launch_dipole_batched(const Desc* descs, int n_prob, uint32_t n_kmax,
                                 const double* accum, double* v, hipStream_t s) {
  hipLaunchKernelGGL(dipole_batched_kernel, dim3(blocks_for(n_kmax, kBlock), n_prob), dim3(kBlock),
                     0, s, descs, accum, v);
  return hipGetLastError();
}

hipError_t launch_spectrum_batched(const Desc* descs, int n_prob, const double* v, double h_step,
                                   int n_omega, double* V_re, double* V_im, double* yield,
                                   hipStream_t s) {
  if (n_omega == 0) return hipSuccess;
  hipLaunchKernelGGL(spectrum_batched_kernel, dim3(n_omega, n_prob), dim3(kBlock), 0, s, descs, v,
                     h_step, n_omega, V_re, V_im, yield);
  return hipGetLastError();
}

hipError_t launch_scale(const double* in, double* out, double scale, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, in, out,
                     scale, n);
  return hipGetLastError();
}

hipError_t launch_spectrum(const double* v, int n_t, double t_first, double dt, double tau_H,
                           const double* omega, int n_omega, double* V_re, double* V_im,
                           double* yield, hipStream_t s) {
  if (n_omega == 0) return hipSuccess;
  hipLaunchKernelGGL(spectrum_kernel, dim3(n_omega), dim3(kBlock), 0, s, v, n_t, t_first, dt,
                     tau_H, omega, V_re, V_im, yield);
  return hipGetLastError();
}

// ------------------------------------------------ spectrum on an FFT grid
// Eq. 3 on the grid w_j = 2 pi j / (L dt) of a zero-padded transform of
// length L = 2^log2_len: the windowed dipole x_k = v_k W_H(t_k) is loaded
// into a complex array (zeros past n_t), transformed by log2_len radix-2
// Stockham passes with the positive exponent (X_j = sum_k x_k
// exp(2 pi i j k / L); out of place, so no bit reversal), and
// V_j = dt exp(i w_j t_first) X_j, A = -i w V, yield |A|^2 and phase arg A
// are formed for j = 0 .. L/2.  Twiddles come from sincospi of the exact
// rational k / Ns.
__global__ void fft_load_kernel(const double* __restrict__ v, int n_t, double t_first, double dt,
                                double tau_H, uint32_t L, double2* __restrict__ a) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  double x = 0.0;
  if ((int)k < n_t) {
    const double t = t_first + (double)k * dt;
    const double wh = fabs(t) <= tau_H ? 0.5 * (1.0 + cos(kPi * t / tau_H)) : 0.0;
    x = v[k] * wh;
  }
  a[k] = make_double2(x, 0.0);
}

__global__ void fft_stage_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                 uint32_t L, uint32_t Ns, double sign) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t half = L >> 1;
  if (j >= half) return;
  const uint32_t k = j & (Ns - 1);  // Ns is a power of two
  const double2 a0 = in[j], b = in[j + half];
  double sn, cs;
  sincospi((double)k / (double)Ns, &sn, &cs);
  sn *= sign;  // exp(sign i pi k / Ns)
  const double2 a1 = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
  const uint32_t o = ((j - k) << 1) + k;
  out[o] = make_double2(a0.x + a1.x, a0.y + a1.y);
  out[o + Ns] = make_double2(a0.x - a1.x, a0.y - a1.y);
}

__global__ void fft_post_kernel(const double2* __restrict__ X, uint32_t L, double t_first,
                                double dt, double* __restrict__ V_re, double* __restrict__ V_im,
                                double* __restrict__ yield, double* __restrict__ phase) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > (L >> 1)) return;
  const double w = 2.0 * kPi * (double)j / ((double)L * dt);
  double sn, cs;
  sincos(w * t_first, &sn, &cs);
  const double2 x = X[j];
  const double vr = dt * (cs * x.x - sn * x.y), vi = dt * (sn * x.x + cs * x.y);
  V_re[j] = vr;
  V_im[j] = vi;
  yield[j] = w * w * (vr * vr + vi * vi);
  if (phase) phase[j] = atan2(-w * vr, w * vi);  // arg of A = -i w V = w vi - i w vr
}

// The derivative in the spectrum: X_j <- -i w_j X_j with the two-sided
// frequencies (j > L/2 negative) and the Nyquist term dropped.
__global__ void fft_derivative_kernel(double2* __restrict__ X, uint32_t L, double dt) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  const double m = j < (L >> 1) ? (double)j : (j == (L >> 1) ? 0.0 : (double)j - (double)L);
  const double w = 2.0 * kPi * m / ((double)L * dt);
  const double2 x = X[j];
  X[j] = make_double2(w * x.y, -w * x.x);  // -i w (x.x + i x.y)
}

__global__ void fft_real_out_kernel(const double2* __restrict__ y, int n_t, double scale,
                                    double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_t) out[k] = scale * y[k].x;
}

// log2(L) radix-2 passes between a and b; returns the array holding the result
static double2* fft_passes(double2* a, double2* b, uint32_t L, double sign, hipStream_t s) {
  for (uint32_t Ns = 1; Ns < L; Ns <<= 1) {
    hipLaunchKernelGGL(fft_stage_kernel, dim3(blocks_for(L / 2, kBlock)), dim3(kBlock), 0, s, a,
                       b, L, Ns, sign);
    double2* t = a;
    a = b;
    b = t;
  }
  return a;
}

hipError_t launch_spectrum_fft(const double* v, int n_t, double t_first, double dt, double tau_H,
                               int log2_len, double2* work, double* V_re, double* V_im,
                               double* yield, double* phase, hipStream_t s) {
  const uint32_t L = 1u << log2_len;
  hipLaunchKernelGGL(fft_load_kernel, dim3(blocks_for(L, kBlock)), dim3(kBlock), 0, s, v, n_t,
                     t_first, dt, tau_H, L, work);
  double2* X = fft_passes(work, work + L, L, 1.0, s);
  hipLaunchKernelGGL(fft_post_kernel, dim3(blocks_for(L / 2 + 1, kBlock)), dim3(kBlock), 0, s, X,
                     L, t_first, dt, V_re, V_im, yield, phase);
  return hipGetLastError();
}

hipError_t launch_acceleration_fft(const double* v, int n_t, double t_first, double dt,
                                   double tau_H, int log2_len, double2* work, double* a,
                                   hipStream_t s) {
  const uint32_t L = 1u << log2_len;
  hipLaunchKernelGGL(fft_load_kernel, dim3(blocks_for(L, kBlock)), dim3(kBlock), 0, s, v, n_t,
                     t_first, dt, tau_H, L, work);
  double2* X = fft_passes(work, work + L, L, 1.0, s);
  hipLaunchKernelGGL(fft_derivative_kernel, dim3(blocks_for(L, kBlock)), dim3(kBlock), 0, s, X, L,
                     dt);
  double2* other = X == work ? work + L : work;
  double2* y = fft_passes(X, other, L, -1.0, s);
  hipLaunchKernelGGL(fft_real_out_kernel, dim3(blocks_for((uint64_t)n_t, kBlock)), dim3(kBlock), 0,
                     s, y, n_t, 1.0 / (double)L, a);
  return hipGetLastError();
}

}  // namespace sfhk

namespace sfhk {
hipError_t launch_gabor(const double* v, int n_t, double t_first, double dt, double sigma,
                        const double* t_c, int n_c, const double* omega, int n_omega,
                        double* G_re, double* G_im, double* yield, hipStream_t s) {
  if (n_c == 0 || n_omega == 0) return hipSuccess;
  hipLaunchKernelGGL(gabor_kernel, dim3(n_c), dim3(kBlock), 0, s, v, n_t, t_first, dt, sigma, t_c,
                     omega, n_omega, G_re, G_im, yield);
  return hipGetLastError();
}
}  // namespace sfhk
