// Time-sliced propagation for continuous batching: every launch advances a
// table of requests (each with its own ensemble, packs, per-trajectory state,
// dipole accumulator and spectrum buffers) by a window of RK4 steps.  The
// trajectory state is saved to and restored from HBM at the window edges, so
// requests can join and leave between windows.
#include "device_common.h"
#include "serve_internal.h"

namespace sfhk {
namespace {

constexpr int kMonoElems = 36;

// one wavefront per (request, pack of the launch's pack group); the window
// table is a kernel argument
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2, 2)))
serve_slice_f64(const ReqDev* __restrict__ reqs, SliceTable tab) {
  __shared__ double mono[kMonoElems][kWave];
  const int lane = threadIdx.x;
  const uint32_t w = blockIdx.x;
  int lo = 0, hi = tab.n;  // tab.e[lo].pack_begin <= w < tab.e[hi].pack_begin
  if (w >= tab.e[tab.n].pack_begin) return;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tab.e[mid].pack_begin <= w) lo = mid; else hi = mid;
  }
  const SliceEntry se = tab.e[lo];
  const ReqDev& R = reqs[se.slot];
  const Desc& d = R.desc;
  const uint32_t pack = tab.group + (w - se.pack_begin) * tab.n_groups;
  if (pack >= R.pack_start[1]) return;
  const int N = d.N;
  const uint32_t pos = pack * kWave + lane;
  const bool valid = pos < R.live_count[0];
  const uint32_t slot = valid ? R.order[R.live_start[0] + pos] : 0u;
  const int k0 = valid ? R.k0[slot] : N + 1;
  const int kmin = __builtin_amdgcn_readfirstlane(k0);
  const int k_from = se.k_from;
  const int k_to = se.k_to < N + 1 ? se.k_to : N + 1;
  if (kmin >= k_to) return;  // nobody in this pack is born before the window ends

  const double n[3] = {R.nx[slot], R.ny[slot], R.nz[slot]};
  const double w8 = R.w[slot];
  const double t0 = d.t_first + (double)k0 * d.dt;
  double q[3], p[3], S, Cre, Cim, flips;
  int kend;
  const uint64_t st = R.live_cap;
  double* __restrict__ sv = R.state + pos;
  if (k0 >= k_from) {  // born in this window (or later): start from the tunnel exit
    q[0] = R.qx[slot];
    q[1] = R.qy[slot];
    q[2] = R.qz[slot];
    p[0] = R.px[slot];
    p[1] = R.py[slot];
    p[2] = R.pz[slot];
    S = 0.0;
    Cre = 1.0;
    Cim = 0.0;
    flips = 0.0;
    kend = N + 1;
#pragma unroll
    for (int i = 0; i < kMonoElems; ++i) mono[i][lane] = (i % 7 == 0) ? 1.0 : 0.0;
  } else {  // resume from the state saved at the end of the previous window
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q[a] = sv[(SFHK_FS_Q + a) * st];
      p[a] = sv[(SFHK_FS_P + a) * st];
    }
#pragma unroll
    for (int i = 0; i < kMonoElems; ++i) mono[i][lane] = sv[(SFHK_FS_M + i) * st];
    S = sv[SFHK_FS_S * st];
    Cre = sv[SFHK_FS_CRE * st];
    Cim = sv[SFHK_FS_CIM * st];
    flips = sv[SFHK_FS_FLIPS * st];
    kend = (int)sv[kStateKend * st];
  }
  const double p0q0 =
      R.px[slot] * R.qx[slot] + R.py[slot] * R.qy[slot] + R.pz[slot] * R.qz[slot] + R.dph[slot];
  // R2 = 2R = Mqq + Mpp - i g Mqp + (i/g) Mpq of the restored M
  double Rr[3][3], Ri[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Rr[a][b] = mono[6 * a + b][lane] + mono[18 + 6 * a + 3 + b][lane];
      Ri[a][b] = d.inv_gamma * mono[18 + 6 * a + b][lane] - d.gamma * mono[6 * a + 3 + b][lane];
    }

  const double h = d.dt;
  const ExpK ekv = make_expk();  // the exponential's constants in VGPRs
  const ExpK* ek = &ekv;
  const double* __restrict__ fe = R.field;
  double* __restrict__ acc = R.accum;
  double acc_reg = 0.0;
  const int kstart = kmin > k_from ? kmin : k_from;
  int k = kstart;
  for (; k < k_to; ++k) {
    bool live = k >= k0 && k < kend;
    double re_a = 0.0;
    const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
    Geom<double> Gk;  // geometry at q_k: amplitude and first RK4 stage
    geometry(d, hRn, q, Gk);
    if (live) {
      prefactor_step(Rr, Ri, Cre, Cim, flips);
      if (d.c_max2 > 0.0 && Cre * Cre + Cim * Cim > d.c_max2) {
        kend = k;
        live = false;
      } else {
        bool near;
        re_a = amplitude_re(d, n, p, Gk, Cre, Cim, S, d.t_first + (double)k * h, t0, p0q0, w8,
                            near);
      }
    }
    deposit(re_a, k, N, lane, acc_reg, acc);
    if (k >= N || !live) continue;

    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
    double K1[6], K2[6], K3[6], K4[6];
    double V, g[3];
    double sq[3], sp3[3], sS, yq[3], yp[3];
    potential(d, Gk, V, g, K1, ek);
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
    potential(d, hRn, yq, V, g, K2, ek);
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
    potential(d, hRn, yq, V, g, K3, ek);
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
    potential(d, hRn, yq, V, g, K4, ek);
    {
      const double kp[3] = {-g[0], -g[1], -g[2] - E1};
      const double kS = 0.5 * (yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]) - V - yq[2] * E1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sq[a] += yp[a];
        sp3[a] += kp[a];
        q[a] = q[a] + d.rk.h6 * sq[a];
        p[a] = p[a] + d.rk.h6 * sp3[a];
      }
      sS += kS;
      S = S + d.rk.h6 * sS;
    }
    StepMatrix<double> P;
    rk4_step_matrix(K1, K2, K3, K4, d.rk, P);
    monodromy_step(P, mono, lane, d.gamma, d.inv_gamma, Rr, Ri);
  }
  // flush the partial 64-step block of dipole sums left at the window end
  if (acc_reg != 0.0) unsafeAtomicAdd(&acc[((k - 1) & ~(kWave - 1)) + lane], acc_reg);
  // save the state of every lane born before the window end
  if (valid && k0 < k_to) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sv[(SFHK_FS_Q + a) * st] = q[a];
      sv[(SFHK_FS_P + a) * st] = p[a];
    }
#pragma unroll
    for (int i = 0; i < kMonoElems; ++i) sv[(SFHK_FS_M + i) * st] = mono[i][lane];
    sv[SFHK_FS_S * st] = S;
    sv[SFHK_FS_CRE * st] = Cre;
    sv[SFHK_FS_CIM * st] = Cim;
    sv[SFHK_FS_FLIPS * st] = flips;
    sv[kStateKend * st] = (double)kend;
  }
}

__global__ void write_req_kernel(ReqDev r, ReqDev* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = r;
}

// dipole of a finished request: v = (2 / n_slots) accum
__global__ void req_dipole_kernel(const ReqDev* __restrict__ reqs, int slot) {
  const ReqDev& R = reqs[slot];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > R.desc.N) return;
  const double sc = R.desc.n_slots > 0 ? 2.0 / (double)R.desc.n_slots : 0.0;
  R.v[k] = sc * R.accum[k];
}

// spectrum of a finished request on its harmonic grid (fixed-order reduction)
__global__ void __launch_bounds__(256) req_spectrum_kernel(const ReqDev* __restrict__ reqs,
                                                           int slot) {
  __shared__ double sr[256], si[256];
  const ReqDev& R = reqs[slot];
  const Desc& d = R.desc;
  const int m = blockIdx.x;
  if (m >= R.n_omega) return;
  const double w = (double)m * R.h_step * d.omega;
  const double tau_H = 0.5 * d.tau;
  double ar = 0.0, ai = 0.0;
  for (int k = threadIdx.x; k <= d.N; k += 256) {
    const double t = d.t_first + (double)k * d.dt;
    const double wh = fabs(t) <= tau_H ? 0.5 * (1.0 + cos(kPi * t / tau_H)) : 0.0;
    double sn, cs;
    sincos(w * t, &sn, &cs);
    const double x = R.v[k] * wh;
    ar += x * cs;
    ai += x * sn;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sr[threadIdx.x] += sr[threadIdx.x + off];
      si[threadIdx.x] += si[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double re = d.dt * sr[0], im = d.dt * si[0];
    R.V_re[m] = re;
    R.V_im[m] = im;
    R.yield[m] = w * w * (re * re + im * im);
  }
}

}  // namespace

hipError_t launch_serve_slice(const ReqDev* reqs, const SliceTable& tab, hipStream_t s) {
  const uint32_t waves = tab.e[tab.n].pack_begin;
  if (tab.n == 0 || waves == 0) return hipSuccess;
  hipLaunchKernelGGL(serve_slice_f64, dim3(waves), dim3(kWave), 0, s, reqs, tab);
  return hipGetLastError();
}

hipError_t launch_request_finalize(const ReqDev* reqs, int slot, int n_kmax, int n_omega,
                                   hipStream_t s) {
  hipLaunchKernelGGL(req_dipole_kernel, dim3((n_kmax + 255) / 256), dim3(256), 0, s, reqs, slot);
  if (n_omega > 0)
    hipLaunchKernelGGL(req_spectrum_kernel, dim3(n_omega), dim3(256), 0, s, reqs, slot);
  return hipGetLastError();
}

hipError_t launch_write_req(const ReqDev& r, ReqDev* dst, hipStream_t s) {
  hipLaunchKernelGGL(write_req_kernel, dim3(1), dim3(1), 0, s, r, dst);
  return hipGetLastError();
}

}  // namespace sfhk
