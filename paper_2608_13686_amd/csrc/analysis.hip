// Classical return analysis for the long/short trajectory maps: for every
// live trajectory, the first step at which its orbit re-enters a sphere of
// radius r_ret around the molecular centre after leaving it, and its
// kinetic energy there.  Only (q, p) are stepped (the RK4 of the propagate
// kernels without monodromy, prefactor or amplitude), one trajectory per
// lane, one 64-lane pack per wavefront; a wavefront stops once every lane
// has returned.
#include "device_common.h"

namespace sfhk {
namespace {

__global__ void __launch_bounds__(kWave) returns_kernel(const Desc* __restrict__ descs,
                                                        int n_prob,
                                                        const double* __restrict__ field,
                                                        EnsPtrs e, double r2_ret,
                                                        int32_t* __restrict__ k_ret,
                                                        double* __restrict__ e_ret) {
  const int lane = threadIdx.x;
  Pack pk;
  if (!find_pack(e, n_prob, blockIdx.x, lane, pk)) return;
  const Desc& d = descs[pk.prob];
  const int N = d.N;
  const uint32_t slot = pk.slot;
  const int k0 = pk.valid ? e.k0[slot] : N + 1;
  double q[3] = {e.qx[slot], e.qy[slot], e.qz[slot]};
  double p[3] = {e.px[slot], e.py[slot], e.pz[slot]};
  const double n[3] = {e.nx[slot], e.ny[slot], e.nz[slot]};
  const double hRn[3] = {d.half_R * n[0], d.half_R * n[1], d.half_R * n[2]};
  const double h = d.dt;
  const double* __restrict__ fe = field + d.field_off;
  bool done = !pk.valid, outside = false;
  int kr = -1;
  double er = 0.0;
  for (int k = __builtin_amdgcn_readfirstlane(k0);; ++k) {
    bool live = !done && k >= k0;
    if (live) {
      const double r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
      if (r2 >= r2_ret) {
        outside = true;
      } else if (outside) {
        kr = k;
        er = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        done = true;
        live = false;
      }
    }
    if (k >= N || !__ballot(!done)) break;
    if (!live) continue;
    const double Ek = fe[2 * k], Eh = fe[2 * k + 1], E1 = fe[2 * k + 2];
    double V, g[3], K[6];
    double sq[3], sp[3], yq[3], yp[3];
    potential(d, hRn, q, V, g, K);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double kp = -g[a] - (a == 2 ? Ek : 0.0);
      sq[a] = p[a];
      sp[a] = kp;
      yq[a] = q[a] + 0.5 * h * p[a];
      yp[a] = p[a] + 0.5 * h * kp;
    }
    potential(d, hRn, yq, V, g, K);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double kq = yp[a], kp = -g[a] - (a == 2 ? Eh : 0.0);
      sq[a] += 2.0 * kq;
      sp[a] += 2.0 * kp;
      yq[a] = q[a] + 0.5 * h * kq;
      yp[a] = p[a] + 0.5 * h * kp;
    }
    potential(d, hRn, yq, V, g, K);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double kq = yp[a], kp = -g[a] - (a == 2 ? Eh : 0.0);
      sq[a] += 2.0 * kq;
      sp[a] += 2.0 * kp;
      yq[a] = q[a] + h * kq;
      yp[a] = p[a] + h * kp;
    }
    potential(d, hRn, yq, V, g, K);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sq[a] += yp[a];
      sp[a] += -g[a] - (a == 2 ? E1 : 0.0);
      q[a] = q[a] + d.rk.h6 * sq[a];
      p[a] = p[a] + d.rk.h6 * sp[a];
    }
  }
  if (pk.valid) {
    k_ret[slot] = kr;
    e_ret[slot] = er;
  }
}

}  // namespace

hipError_t launch_returns(const Desc* descs, int n_prob, const double* field, EnsPtrs e,
                          uint32_t max_packs, double r_ret, int32_t* k_ret, double* e_ret,
                          hipStream_t s) {
  if (max_packs == 0) return hipSuccess;
  hipLaunchKernelGGL(returns_kernel, dim3(max_packs), dim3(kWave), 0, s, descs, n_prob, field, e,
                     r_ret * r_ret, k_ret, e_ret);
  return hipGetLastError();
}

}  // namespace sfhk
