// C ABI of libsfhk: argument validation, per-problem constants, workspace
// carve-up and kernel launches.  No exception crosses the interface.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sfhk_internal.h"

using namespace sfhk;

namespace {

thread_local std::string g_err;

sfhk_status fail(sfhk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

sfhk_status ok() {
  g_err.clear();
  return SFHK_OK;
}

sfhk_status hip_fail(hipError_t e, const char* where) {
  return fail(SFHK_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// hc / E_h in hartree * nm and the atomic unit of intensity (W/cm^2)
constexpr double kHcHartreeNm = 45.56335252912;
constexpr double kIntensityAu = 3.50944552058977e16;

bool is_finite(double x) { return std::isfinite(x); }

// Laser constants of the sin^2 pulse: w, E0, tau, N (N = round(tau/dt) unless given).
void laser_consts(const sfhk_problem& p, double& omega, double& E0, double& tau, int64_t& N) {
  omega = kHcHartreeNm / p.las.lambda_nm;
  E0 = std::sqrt(p.las.intensity_wcm2 / kIntensityAu);
  tau = p.las.n_cycles * 2.0 * kPi / omega;
  N = p.n_steps > 0 ? (int64_t)p.n_steps : (int64_t)std::llround(tau / p.dt);
}

sfhk_status check_problem(const sfhk_problem* p, int idx) {
  if (!p) return fail(SFHK_E_INVALID, "problem %d: null", idx);
  const sfhk_laser& L = p->las;
  if (!(is_finite(L.lambda_nm) && L.lambda_nm > 0))
    return fail(SFHK_E_INVALID, "problem %d: lambda_nm must be > 0", idx);
  if (!(is_finite(L.intensity_wcm2) && L.intensity_wcm2 >= 0))
    return fail(SFHK_E_INVALID, "problem %d: intensity must be >= 0", idx);
  if (!(is_finite(L.n_cycles) && L.n_cycles > 0))
    return fail(SFHK_E_INVALID, "problem %d: n_cycles must be > 0", idx);
  if (!is_finite(L.cep)) return fail(SFHK_E_INVALID, "problem %d: cep not finite", idx);
  if (!(is_finite(p->dt) && p->dt > 0)) return fail(SFHK_E_INVALID, "problem %d: dt must be > 0", idx);
  if (!(is_finite(p->gamma_cs) && p->gamma_cs > 0))
    return fail(SFHK_E_INVALID, "problem %d: gamma_cs must be > 0", idx);
  if (!(is_finite(p->w_cut) && p->w_cut >= 0))
    return fail(SFHK_E_INVALID, "problem %d: w_cut must be >= 0", idx);
  if (!(is_finite(p->sigma_perp) && p->sigma_perp >= 0))
    return fail(SFHK_E_INVALID, "problem %d: sigma_perp must be >= 0", idx);
  if (p->n_steps < 0) return fail(SFHK_E_INVALID, "problem %d: n_steps must be >= 0", idx);
  const sfhk_target& T = p->tgt;
  if (!(is_finite(T.R) && T.R >= 0)) return fail(SFHK_E_INVALID, "problem %d: R must be >= 0", idx);
  if (!(is_finite(T.Ip) && T.Ip > 0)) return fail(SFHK_E_INVALID, "problem %d: Ip must be > 0", idx);
  for (int c = 0; c < 2; ++c) {
    const sfhk_center& C = T.ctr[c];
    if (!(is_finite(C.Zinf) && is_finite(C.dZ) && is_finite(C.alpha) && is_finite(C.eps2) && C.eps2 >= 0))
      return fail(SFHK_E_INVALID, "problem %d: centre %d parameters invalid", idx, c);
  }
  if (T.n_gto < 1 || T.n_gto > SFHK_MAX_GTO)
    return fail(SFHK_E_INVALID, "problem %d: n_gto must be in 1..%d", idx, SFHK_MAX_GTO);
  if (!T.gto) return fail(SFHK_E_INVALID, "problem %d: gto table is null", idx);
  for (int j = 0; j < T.n_gto; ++j) {
    const sfhk_gto& g = T.gto[j];
    if ((g.center != 0 && g.center != 1) || (g.l != 0 && g.l != 1) || !(is_finite(g.a) && g.a > 0) ||
        !is_finite(g.c))
      return fail(SFHK_E_INVALID, "problem %d: gto primitive %d invalid", idx, j);
  }
  const sfhk_align& A = p->al;
  if (A.kind != SFHK_ALIGN_FIXED && A.kind != SFHK_ALIGN_COS2M)
    return fail(SFHK_E_INVALID, "problem %d: unknown alignment kind %d", idx, A.kind);
  if (A.m < 0 || A.m > 64) return fail(SFHK_E_INVALID, "problem %d: alignment m out of range", idx);
  if (!(is_finite(A.theta) && is_finite(A.phi)))
    return fail(SFHK_E_INVALID, "problem %d: alignment angles not finite", idx);
  double omega, E0, tau;
  int64_t N;
  laser_consts(*p, omega, E0, tau, N);
  if (N < 1 || N > (1 << 24))
    return fail(SFHK_E_INVALID, "problem %d: step count %lld out of range 1..2^24", idx,
                (long long)N);
  return SFHK_OK;
}

sfhk_status check_problems(const sfhk_problem* probs, int32_t n_prob) {
  if (!probs) return fail(SFHK_E_INVALID, "probs is null");
  if (n_prob < 1 || n_prob > SFHK_MAX_PROBLEMS)
    return fail(SFHK_E_INVALID, "n_prob must be in 1..%d", SFHK_MAX_PROBLEMS);
  for (int i = 0; i < n_prob; ++i) {
    sfhk_status st = check_problem(&probs[i], i);
    if (st != SFHK_OK) return st;
  }
  return SFHK_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Per-problem constants; slot_off/seed/first are filled by the caller.
Desc make_desc(const sfhk_problem& p) {
  Desc d;
  std::memset(&d, 0, sizeof d);
  double omega, E0, tau;
  int64_t N;
  laser_consts(p, omega, E0, tau, N);
  d.omega = omega;
  d.E0 = E0;
  d.tau = tau;
  d.cep = p.las.cep;
  d.dt = p.dt;
  d.t_first = -0.5 * tau;
  d.N = (int32_t)N;
  d.align_kind = p.al.kind;
  d.align_m = p.al.m;
  d.n_gto = p.tgt.n_gto;
  d.screened = (p.tgt.ctr[0].dZ != 0.0 || p.tgt.ctr[1].dZ != 0.0) ? 1 : 0;
  d.half_R = 0.5 * p.tgt.R;
  d.Ip = p.tgt.Ip;
  d.gamma = p.gamma_cs;
  d.inv_gamma = 1.0 / p.gamma_cs;
  d.inv_gamma2 = 1.0 / (p.gamma_cs * p.gamma_cs);
  d.half_inv_gamma = 1.0 / (2.0 * p.gamma_cs);
  for (int c = 0; c < 2; ++c) {
    d.Zinf[c] = p.tgt.ctr[c].Zinf;
    d.dZ[c] = p.tgt.ctr[c].dZ;
    d.alpha[c] = p.tgt.ctr[c].alpha;
    d.eps2[c] = p.tgt.ctr[c].eps2;
    d.fZinf[c] = (float)d.Zinf[c];
    d.fdZ[c] = (float)d.dZ[c];
    d.falpha[c] = (float)d.alpha[c];
    d.feps2[c] = (float)d.eps2[c];
  }
  d.sigma = p.sigma_perp;
  d.w_cut = p.w_cut;
  d.kappa = std::sqrt(2.0 * p.tgt.Ip);
  d.wpow = 0.5 * (2.0 / d.kappa - 1.0);
  d.kcube3 = d.kappa * d.kappa * d.kappa / 3.0;
  d.inv_E0 = E0 > 0 ? 1.0 / E0 : 0.0;
  d.nfix[0] = std::sin(p.al.theta) * std::cos(p.al.phi);
  d.nfix[1] = std::sin(p.al.theta) * std::sin(p.al.phi);
  d.nfix[2] = std::cos(p.al.theta);
  const double g = p.gamma_cs;
  d.g_inv4k_min = 1e300;
  for (int j = 0; j < p.tgt.n_gto; ++j) {
    const sfhk_gto& G = p.tgt.gto[j];
    const double k2 = 1.0 / (4.0 * G.a) + 1.0 / (2.0 * g);
    d.g_sgn[j] = G.center == 0 ? 1.0 : -1.0;
    d.g_l[j] = G.l;
    d.g_inv4k[j] = 1.0 / (4.0 * k2);
    d.g_inv2k[j] = 1.0 / (2.0 * k2);
    d.g_norm[j] = G.c * std::pow(2.0 * G.a, -1.5) * std::pow(kPi * g, -0.75) *
                  std::pow(kPi / k2, 1.5);
    d.g_i2a[j] = 1.0 / (2.0 * G.a);
    d.g_inv4k_min = std::min(d.g_inv4k_min, d.g_inv4k[j]);
  }
  return d;
}

// Descriptors with field/accum offsets; returns the layout.
Layout build_layout(const sfhk_problem* probs, int32_t n_prob, uint64_t n_slots,
                    std::vector<Desc>* descs, int64_t* max_steps) {
  Layout L;
  uint64_t fo = 0, ao = 0;
  int64_t mx = 0;
  if (descs) descs->resize(n_prob);
  for (int i = 0; i < n_prob; ++i) {
    double omega, E0, tau;
    int64_t N;
    laser_consts(probs[i], omega, E0, tau, N);
    if (descs) {
      (*descs)[i] = make_desc(probs[i]);
      (*descs)[i].field_off = fo;
      (*descs)[i].acc_off = ao;
    }
    fo += 2 * (uint64_t)(N + 1);
    ao += (uint64_t)(N + 1);
    mx = std::max(mx, N);
  }
  L.n_field = fo;
  L.n_bins = ao;
  L.n_slots = n_slots;
  size_t off = 0;
  L.off_descs = off;
  off = align256(off + sizeof(Desc) * (size_t)n_prob);
  L.off_slot = off;
  off = align256(off + sizeof(uint64_t) * ((size_t)n_prob + 1));
  L.off_field = off;
  off = align256(off + sizeof(double) * (size_t)L.n_field);
  L.off_hist = off;
  off = align256(off + sizeof(uint32_t) * (size_t)(L.n_bins + 1));
  L.off_cursor = off;
  off = align256(off + sizeof(uint32_t) * (size_t)(L.n_bins + 1));
  L.off_redo = off;
  off = align256(off + sizeof(int32_t) * (size_t)n_slots);
  L.off_order2 = off;
  off = align256(off + sizeof(uint32_t) * (size_t)n_slots);
  L.off_runs2 = off;
  off = align256(off + sizeof(uint32_t) * (3 * (size_t)n_prob + 1));
  L.bytes = off;
  if (max_steps) *max_steps = mx;
  return L;
}

Workspace carve(void* base, const Layout& L) {
  char* b = static_cast<char*>(base);
  Workspace w;
  w.descs = reinterpret_cast<Desc*>(b + L.off_descs);
  w.slot_off = reinterpret_cast<uint64_t*>(b + L.off_slot);
  w.field = reinterpret_cast<double*>(b + L.off_field);
  w.hist = reinterpret_cast<uint32_t*>(b + L.off_hist);
  w.cursor = reinterpret_cast<uint32_t*>(b + L.off_cursor);
  w.redo = reinterpret_cast<int32_t*>(b + L.off_redo);
  w.order2 = reinterpret_cast<uint32_t*>(b + L.off_order2);
  w.runs2 = reinterpret_cast<uint32_t*>(b + L.off_runs2);
  w.bytes = L.bytes;
  return w;
}

sfhk_status check_ensemble(const sfhk_ensemble* e) {
  if (!e) return fail(SFHK_E_INVALID, "ensemble is null");
  if (e->capacity >= (uint64_t(1) << 32))
    return fail(SFHK_E_INVALID, "ensemble capacity must be < 2^32");
  if (e->capacity == 0) return SFHK_OK;
  const void* ptrs[] = {e->k0, e->prob, e->qx, e->qy, e->qz, e->px, e->py, e->pz,
                        e->w, e->nx, e->ny, e->nz, e->order, e->live_start,
                        e->live_count, e->pack_start};
  for (const void* q : ptrs)
    if (!q) return fail(SFHK_E_INVALID, "ensemble has a null device array");
  return SFHK_OK;
}

EnsPtrs ens_ptrs(const sfhk_ensemble* e) {
  EnsPtrs p;
  p.k0 = e->k0;
  p.prob = e->prob;
  p.qx = e->qx;
  p.qy = e->qy;
  p.qz = e->qz;
  p.px = e->px;
  p.py = e->py;
  p.pz = e->pz;
  p.w = e->w;
  p.nx = e->nx;
  p.ny = e->ny;
  p.nz = e->nz;
  p.order = e->order;
  p.live_start = e->live_start;
  p.live_count = e->live_count;
  p.pack_start = e->pack_start;
  return p;
}

// Upload descriptors and build the field tables.
sfhk_status stage_problems(const std::vector<Desc>& descs, const Workspace& ws,
                           const std::vector<uint64_t>* slot_off, int64_t max_steps,
                           hipStream_t s) {
  hipError_t e = hipMemcpyAsync(ws.descs, descs.data(), sizeof(Desc) * descs.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  if (slot_off) {
    e = hipMemcpyAsync(ws.slot_off, slot_off->data(), sizeof(uint64_t) * slot_off->size(),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "slot offset upload");
  }
  e = launch_field(ws.descs, (int)descs.size(), ws.field, (uint64_t)max_steps + 1, s);
  if (e != hipSuccess) return hip_fail(e, "field table");
  return SFHK_OK;
}

}  // namespace

extern "C" {

int32_t sfhk_abi_version(void) { return SFHK_ABI_VERSION; }

const char* sfhk_last_error(void) { return g_err.c_str(); }

sfhk_status sfhk_problem_steps(const sfhk_problem* p, int32_t* n_steps, double* t_first,
                               double* tau) {
  sfhk_status st = check_problem(p, 0);
  if (st != SFHK_OK) return st;
  double omega, E0, T;
  int64_t N;
  laser_consts(*p, omega, E0, T, N);
  if (n_steps) *n_steps = (int32_t)N;
  if (t_first) *t_first = -0.5 * T;
  if (tau) *tau = T;
  return ok();
}

size_t sfhk_workspace_bytes(const sfhk_problem* probs, int32_t n_prob, uint64_t capacity) {
  if (check_problems(probs, n_prob) != SFHK_OK) return 0;
  g_err.clear();
  return build_layout(probs, n_prob, capacity, nullptr, nullptr).bytes;
}

sfhk_status sfhk_sample_initial(const sfhk_problem* probs, int32_t n_prob,
                                const uint64_t* n_per_prob, const uint64_t* seeds,
                                const uint64_t* first_index, const sfhk_ensemble* ens,
                                void* workspace, size_t workspace_bytes, void* stream) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if (!n_per_prob || !seeds || !first_index)
    return fail(SFHK_E_INVALID, "n_per_prob, seeds and first_index must be non-null");
  if ((st = check_ensemble(ens)) != SFHK_OK) return st;
  std::vector<uint64_t> slot_off(n_prob + 1, 0);
  for (int i = 0; i < n_prob; ++i) {
    if (n_per_prob[i] > (uint64_t(1) << 32))
      return fail(SFHK_E_INVALID, "n_per_prob[%d] too large", i);
    slot_off[i + 1] = slot_off[i] + n_per_prob[i];
  }
  const uint64_t n_slots = slot_off[n_prob];
  if (n_slots > ens->capacity)
    return fail(SFHK_E_NOMEM, "sum(n_per_prob) = %llu exceeds ensemble capacity %llu",
                (unsigned long long)n_slots, (unsigned long long)ens->capacity);
  std::vector<Desc> descs;
  int64_t max_steps = 0;
  Layout L = build_layout(probs, n_prob, n_slots, &descs, &max_steps);
  if (L.n_bins + 1 >= (uint64_t(1) << 31))
    return fail(SFHK_E_UNSUPPORTED, "total step count of the problems too large");
  if (!workspace) return fail(SFHK_E_INVALID, "workspace is null");
  if (workspace_bytes < L.bytes)
    return fail(SFHK_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.bytes);
  for (int i = 0; i < n_prob; ++i) {
    descs[i].slot_off = slot_off[i];
    descs[i].n_slots = n_per_prob[i];
    descs[i].seed = seeds[i];
    descs[i].first_index = first_index[i];
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = carve(workspace, L);
  if ((st = stage_problems(descs, ws, &slot_off, max_steps, s)) != SFHK_OK) return st;
  EnsPtrs ep = ens_ptrs(ens);
  hipError_t e = launch_fill_u32(ws.hist, 0u, L.n_bins + 1, s);
  if (e == hipSuccess) e = launch_sample(ws.descs, n_prob, ws.slot_off, n_slots, ws.field, ep,
                                         ws.hist, s);
  PackOut po{ep.order, ep.live_start, ep.live_count, ep.pack_start};
  if (e == hipSuccess)
    e = launch_sort(ws.descs, n_prob, n_slots, L.n_bins, ws.hist, ws.cursor, ep, nullptr, po, s);
  if (e != hipSuccess) return hip_fail(e, "sample_initial");
  return ok();
}

sfhk_status sfhk_propagate(const sfhk_problem* probs, int32_t n_prob, const sfhk_ensemble* ens,
                           int32_t precision, double* accum, double* final_state,
                           void* workspace, size_t workspace_bytes, void* stream) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if ((st = check_ensemble(ens)) != SFHK_OK) return st;
  if (precision != SFHK_FP64 && precision != SFHK_MIXED)
    return fail(SFHK_E_INVALID, "unknown precision %d", precision);
  if (!accum) return fail(SFHK_E_INVALID, "accum is null");
  std::vector<Desc> descs;
  int64_t max_steps = 0;
  Layout L = build_layout(probs, n_prob, ens->capacity, &descs, &max_steps);
  if (!workspace) return fail(SFHK_E_INVALID, "workspace is null");
  if (workspace_bytes < L.bytes)
    return fail(SFHK_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.bytes);
  if (ens->capacity == 0) return ok();
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = carve(workspace, L);
  if ((st = stage_problems(descs, ws, nullptr, max_steps, s)) != SFHK_OK) return st;
  // one wavefront per 64-lane pack; packs never straddle problems
  const uint64_t max_packs = (ens->capacity + kWave - 1) / kWave + (uint64_t)n_prob;
  if (max_packs > 0x7fffffffull) return fail(SFHK_E_UNSUPPORTED, "ensemble too large");
  EnsPtrs ep = ens_ptrs(ens);
  hipError_t e;
  if (precision == SFHK_FP64) {
    e = launch_propagate_f64(ws.descs, n_prob, ws.field, ep, nullptr, (uint32_t)max_packs, accum,
                             final_state, ens->capacity, s);
  } else {
    // FP32 stepping for every trajectory; those whose monodromy matrix grows
    // past the FP32 bound are handed over, at that step, to an FP64 re-run
    // from their birth (sorted into packs of their own).
    e = launch_fill_i32(ws.redo, -1, ens->capacity, s);
    if (e == hipSuccess)
      e = launch_propagate_mixed(ws.descs, n_prob, ws.field, ep, ws.redo, (uint32_t)max_packs,
                                 accum, final_state, ens->capacity, s);
    if (e == hipSuccess) e = launch_fill_u32(ws.hist, 0u, L.n_bins + 1, s);
    if (e == hipSuccess) e = launch_count(ws.descs, ens->capacity, ep, ws.redo, ws.hist, s);
    PackOut po{ws.order2, ws.runs2, ws.runs2 + n_prob, ws.runs2 + 2 * n_prob};
    if (e == hipSuccess)
      e = launch_sort(ws.descs, n_prob, ens->capacity, L.n_bins, ws.hist, ws.cursor, ep, ws.redo,
                      po, s);
    if (e == hipSuccess) {
      EnsPtrs e2 = ep;
      e2.order = po.order;
      e2.live_start = po.live_start;
      e2.live_count = po.live_count;
      e2.pack_start = po.pack_start;
      e = launch_propagate_f64(ws.descs, n_prob, ws.field, e2, ws.redo, (uint32_t)max_packs,
                               accum, final_state, ens->capacity, s);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "propagate");
  return ok();
}

sfhk_status sfhk_dipole(const sfhk_problem* probs, int32_t n_prob, const double* accum,
                        const uint64_t* n_sampled, double* v_out, void* stream) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if (!accum || !v_out || !n_sampled)
    return fail(SFHK_E_INVALID, "accum, n_sampled and v_out must be non-null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t off = 0;
  for (int i = 0; i < n_prob; ++i) {
    double omega, E0, tau;
    int64_t N;
    laser_consts(probs[i], omega, E0, tau, N);
    const double sc = n_sampled[i] > 0 ? 2.0 / (double)n_sampled[i] : 0.0;
    hipError_t e = launch_scale(accum + off, v_out + off, sc, (uint64_t)(N + 1), s);
    if (e != hipSuccess) return hip_fail(e, "dipole");
    off += (uint64_t)(N + 1);
  }
  return ok();
}

sfhk_status sfhk_spectrum(const double* v, int32_t n_t, double t_first, double dt, double tau_H,
                          const double* omega, int32_t n_omega, double* V_re, double* V_im,
                          double* yield, void* stream) {
  if (n_t < 1) return fail(SFHK_E_INVALID, "n_t must be >= 1");
  if (n_omega < 0) return fail(SFHK_E_INVALID, "n_omega must be >= 0");
  if (!(is_finite(t_first) && is_finite(dt) && dt > 0 && is_finite(tau_H) && tau_H > 0))
    return fail(SFHK_E_INVALID, "t_first, dt > 0 and tau_H > 0 must be finite");
  if (n_omega == 0) return ok();
  if (!v || !omega || !V_re || !V_im || !yield)
    return fail(SFHK_E_INVALID, "spectrum pointers must be non-null");
  hipError_t e = launch_spectrum(v, n_t, t_first, dt, tau_H, omega, n_omega, V_re, V_im, yield,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "spectrum");
  return ok();
}

}  // extern "C"
