// C ABI of libsfhk: argument validation, per-problem constants, workspace
// carve-up and kernel launches.  No exception crosses the interface.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <memory>
#include <mutex>
#include <new>
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
  if (!is_finite(p->c_max)) return fail(SFHK_E_INVALID, "problem %d: c_max not finite", idx);
  if (p->n_steps < 0) return fail(SFHK_E_INVALID, "problem %d: n_steps must be >= 0", idx);
  if (p->ionization != SFHK_ION_FIRST_ORDER && p->ionization != SFHK_ION_SADDLE &&
      p->ionization != SFHK_ION_SADDLE_MODIFIED)
    return fail(SFHK_E_INVALID, "problem %d: unknown ionisation step %d", idx, p->ionization);
  // the saddle-point step writes the pulse as carriers w and w +- 2 pi/tau;
  // one cycle makes w - 2 pi/tau vanish
  if (p->ionization != SFHK_ION_FIRST_ORDER && !(p->las.n_cycles > 1.0))
    return fail(SFHK_E_INVALID, "problem %d: the saddle-point step needs n_cycles > 1", idx);
  const sfhk_target& T = p->tgt;
  if (!(is_finite(T.R) && T.R >= 0)) return fail(SFHK_E_INVALID, "problem %d: R must be >= 0", idx);
  if (!(is_finite(T.Ip) && T.Ip > 0)) return fail(SFHK_E_INVALID, "problem %d: Ip must be > 0", idx);
  for (int c = 0; c < 2; ++c) {
    const sfhk_center& C = T.ctr[c];
    if (!(is_finite(C.Zinf) && is_finite(C.dZ) && is_finite(C.alpha) && is_finite(C.eps2) && C.eps2 >= 0 &&
          C.alpha >= 0))
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
  d.ionization = p.ionization;
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
    d.adZ[c] = d.alpha[c] * d.dZ[c];
    d.a2dZ[c] = d.alpha[c] * d.adZ[c];
    d.fadZ[c] = (float)d.adZ[c];
    d.fa2dZ[c] = (float)d.a2dZ[c];
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
  d.c_max2 = p.c_max > 0.0 ? p.c_max * p.c_max : 0.0;
  {
    const double h = p.dt;
    d.rk = {h, 0.5 * h, h / 6.0, h * h / 6.0, h * h * h / 12.0, h * h * h * h / 24.0};
    const float f = (float)p.dt;
    d.frk = {f, 0.5f * f, f / 6.0f, f * f / 6.0f, f * f * f / 12.0f, f * f * f * f / 24.0f};
  }
  d.nfix[0] = std::sin(p.al.theta) * std::cos(p.al.phi);
  d.nfix[1] = std::sin(p.al.theta) * std::sin(p.al.phi);
  d.nfix[2] = std::cos(p.al.theta);
  const double g = p.gamma_cs;
  d.g_inv4k_min = 1e300;
  for (int j = 0; j < p.tgt.n_gto; ++j) {
    const sfhk_gto& G = p.tgt.gto[j];
    d.g_l[j] = G.l | (G.center << 1);
    d.g_ion[j] = G.c * std::pow(2.0 * G.a, -1.5);
    d.g_i2a[j] = 1.0 / (2.0 * G.a);
  }
  // recombination shells, centre 0 first
  d.n_shell = 0;
  for (int c = 0; c < 2; ++c) {
    const int first = d.n_shell;
    for (int j = 0; j < p.tgt.n_gto; ++j) {
      const sfhk_gto& G = p.tgt.gto[j];
      if (G.center != c) continue;
      const double k2 = 1.0 / (4.0 * G.a) + 1.0 / (2.0 * g);
      const double inv4k = 1.0 / (4.0 * k2);
      int s = first;
      while (s < d.n_shell && d.sh_inv4k[s] != inv4k) ++s;
      if (s == d.n_shell) {
        d.sh_inv4k[s] = inv4k;
        d.sh_ns[s] = d.sh_np[s] = 0.0;
        ++d.n_shell;
      }
      const double norm = G.c * std::pow(2.0 * G.a, -1.5) * std::pow(kPi * g, -0.75) *
                          std::pow(kPi / k2, 1.5);
      if (G.l == 0)
        d.sh_ns[s] += norm;
      else
        d.sh_np[s] += norm / (2.0 * G.a);
      d.g_inv4k_min = std::min(d.g_inv4k_min, inv4k);
    }
    if (c == 0) d.n_shell0 = d.n_shell;
  }
  return d;
}

// Descriptors with field/accum offsets; returns the layout.  The mixed
// precision's hand-over arrays (redo, order2, runs2) are laid out only for
// SFHK_MIXED (the default covers both precisions).
Layout build_layout(const sfhk_problem* probs, int32_t n_prob, uint64_t n_slots,
                    std::vector<Desc>* descs, int64_t* max_steps, bool with_queue = false,
                    int precision = SFHK_MIXED) {
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
  if (precision == SFHK_MIXED) {
    L.off_redo = off;
    off = align256(off + sizeof(int32_t) * (size_t)n_slots);
    L.off_order2 = off;
    off = align256(off + sizeof(uint32_t) * (size_t)n_slots);
    L.off_runs2 = off;
    off = align256(off + sizeof(uint32_t) * (3 * (size_t)n_prob + 1));
  }
  if (with_queue) {
    L.max_packs = (uint32_t)((n_slots + kWave - 1) / kWave + (uint64_t)n_prob);
    L.n_len = (uint32_t)(mx + 1);
    L.off_qkeys = off;
    off = align256(off + sizeof(uint32_t) * (size_t)L.max_packs);
    L.off_qhist = off;
    off = align256(off + sizeof(uint32_t) * ((size_t)L.n_len + 1));
    L.off_qcursor = off;
    off = align256(off + sizeof(uint32_t) * ((size_t)L.n_len + 1));
    L.off_queue = off;
    off = align256(off + sizeof(uint32_t) * (size_t)L.max_packs);
    L.off_queue2 = off;
    off = align256(off + sizeof(uint32_t) * (size_t)L.max_packs);
    L.off_counter = off;
    off = align256(off + 2 * sizeof(uint32_t));
  }
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
  w.redo = L.off_redo ? reinterpret_cast<int32_t*>(b + L.off_redo) : nullptr;
  w.order2 = L.off_order2 ? reinterpret_cast<uint32_t*>(b + L.off_order2) : nullptr;
  w.runs2 = L.off_runs2 ? reinterpret_cast<uint32_t*>(b + L.off_runs2) : nullptr;
  w.bytes = L.bytes;
  return w;
}

sfhk_status check_ensemble(const sfhk_ensemble* e) {
  if (!e) return fail(SFHK_E_INVALID, "ensemble is null");
  if (e->capacity >= (uint64_t(1) << 32))
    return fail(SFHK_E_INVALID, "ensemble capacity must be < 2^32");
  if (e->capacity == 0) return SFHK_OK;
  const void* ptrs[] = {e->k0, e->prob, e->qx, e->qy, e->qz, e->px, e->py, e->pz,
                        e->w, e->nx, e->ny, e->nz, e->dph, e->order, e->live_start,
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
  p.dph = e->dph;
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

// The same staging with the descriptors passed as kernel arguments (one
// small kernel per problem), so that no host memory is read after the call.
sfhk_status stage_problems_by_args(const std::vector<Desc>& descs, const Workspace& ws,
                                   int64_t max_steps, hipStream_t s) {
  for (size_t i = 0; i < descs.size(); ++i) {
    hipError_t e = launch_store_desc(descs[i], ws.descs + i, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  }
  hipError_t e = launch_field(ws.descs, (int)descs.size(), ws.field, (uint64_t)max_steps + 1, s);
  if (e != hipSuccess) return hip_fail(e, "field table");
  return SFHK_OK;
}

// Workspace of sfhk_propagate_static: a device array of the library, one
// copy per GPU, that lives until the process ends.  Host code never uses its
// name as an address: the device address of each GPU's copy is looked up
// once, with that GPU current, and kept.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kStaticMaxProblems = 1024;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

sfhk_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(SFHK_E_UNSUPPORTED, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "static workspace address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SFHK_OK;
}

// Argument checks, descriptors and workspace layout of a propagation.
sfhk_status propagate_prepare(const sfhk_problem* probs, int32_t n_prob, const sfhk_ensemble* ens,
                              int32_t precision, double* accum, double* snapshots,
                              int32_t n_snap, int32_t snap_every, std::vector<Desc>& descs,
                              int64_t& max_steps, Layout& L) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if ((st = check_ensemble(ens)) != SFHK_OK) return st;
  if (precision != SFHK_FP64 && precision != SFHK_MIXED)
    return fail(SFHK_E_INVALID, "unknown precision %d", precision);
  if (!accum) return fail(SFHK_E_INVALID, "accum is null");
  if (snapshots && (n_snap < 1 || snap_every < 1))
    return fail(SFHK_E_INVALID, "snapshots need n_snap >= 1 and snap_every >= 1");
  L = build_layout(probs, n_prob, ens->capacity, &descs, &max_steps, false, precision);
  return SFHK_OK;
}

Records make_records(const sfhk_ensemble* ens, double* final_state, double* snapshots,
                     int32_t n_snap, int32_t snap_every) {
  Records rec;
  rec.final_state = final_state;
  rec.snap = snapshots;
  rec.n_snap = snapshots ? n_snap : 0;
  rec.snap_every = snapshots ? snap_every : 1;
  rec.capacity = ens->capacity;
  return rec;
}

// Propagation of a sampled ensemble whose problems are staged in ws: FP64,
// or FP32 stepping for every trajectory with the ones whose monodromy matrix
// grows past the FP32 bound handed over, at that step, to an FP64 re-run from
// their birth (sorted into packs of their own).
sfhk_status propagate_enqueue(int n_prob, const sfhk_ensemble* ens, int precision, double* accum,
                              const Records& rec, const Workspace& ws, const Layout& L,
                              hipStream_t s) {
  // one wavefront per 64-lane pack; packs never straddle problems
  const uint64_t max_packs = (ens->capacity + kWave - 1) / kWave + (uint64_t)n_prob;
  if (max_packs > 0x7fffffffull) return fail(SFHK_E_UNSUPPORTED, "ensemble too large");
  EnsPtrs ep = ens_ptrs(ens);
  hipError_t e;
  if (precision == SFHK_FP64) {
    // far below device fill a trajectory's step latency sets the time: the
    // latency form (one trajectory per 8 lanes)
    if (max_packs <= kLatencyMaxPacks)
      e = launch_propagate_latency(ws.descs, n_prob, ws.field, ep, nullptr, (uint32_t)max_packs,
                                   accum, rec, s, LaunchCfg{});
    else
      e = launch_propagate_f64(ws.descs, n_prob, ws.field, ep, nullptr, (uint32_t)max_packs,
                               accum, rec, s, LaunchCfg{});
  } else {
    e = launch_fill_i32(ws.redo, -1, ens->capacity, s);
    if (e == hipSuccess)
      e = launch_propagate_mixed(ws.descs, n_prob, ws.field, ep, ws.redo, (uint32_t)max_packs,
                                 accum, rec, s, LaunchCfg{});
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
      // the handed-over trajectories are few: latency form (units of two
      // monodromy wavefronts when the launch is above the latency threshold:
      // hundreds of units share the SIMDs)
      LaunchCfg lc;
      lc.pipe_mono = max_packs > kLatencyMaxPacks ? 2 : 1;
      e = launch_propagate_latency(ws.descs, n_prob, ws.field, e2, ws.redo, (uint32_t)max_packs,
                                   accum, rec, s, lc);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "propagate");
  return ok();
}

// Bytes of the ensemble arrays of sfhk_ensemble for `capacity` slots and
// n_prob problems, each array 256-byte aligned.
size_t ensemble_bytes(uint64_t capacity, int n_prob) {
  const size_t c = (size_t)std::max<uint64_t>(capacity, 1);
  return 2 * align256(sizeof(int32_t) * c) + 11 * align256(sizeof(double) * c) +
         align256(sizeof(uint32_t) * c) + 2 * align256(sizeof(uint32_t) * (size_t)n_prob) +
         align256(sizeof(uint32_t) * ((size_t)n_prob + 1));
}

}  // namespace

// entry points of this file used by the serving ABI (serve_abi.hip)
namespace sfhk_abi_detail {
sfhk_status check_problem_ext(const sfhk_problem* p, int idx) { return check_problem(p, idx); }
Desc make_desc_ext(const sfhk_problem& p) { return make_desc(p); }
sfhk_status fail_ext(sfhk_status st, const char* msg) { return fail(st, "%s", msg); }
sfhk_status hip_fail_ext(hipError_t e, const char* where) { return hip_fail(e, where); }
sfhk_status ok_ext() { return ok(); }
}  // namespace sfhk_abi_detail

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

size_t sfhk_footprint_bytes(const sfhk_problem* p, uint64_t n_traj, int32_t precision) {
  if (check_problems(p, 1) != SFHK_OK) return 0;
  if (precision != SFHK_FP64 && precision != SFHK_MIXED) {
    fail(SFHK_E_INVALID, "unknown precision %d", precision);
    return 0;
  }
  if (n_traj >= (uint64_t(1) << 32)) {
    fail(SFHK_E_INVALID, "n_traj must be < 2^32");
    return 0;
  }
  double omega, E0, tau;
  int64_t N;
  laser_consts(*p, omega, E0, tau, N);
  g_err.clear();
  return ensemble_bytes(n_traj, 1) +
         build_layout(p, 1, n_traj, nullptr, nullptr, false, precision).bytes +
         2 * align256(sizeof(double) * (size_t)(N + 1));
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
  // sampling uses no hand-over arrays: the FP64 layout (a prefix of both)
  Layout L = build_layout(probs, n_prob, n_slots, &descs, &max_steps, false, SFHK_FP64);
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
                                         ws.hist, any_saddle(descs.data(), n_prob), s);
  PackOut po{ep.order, ep.live_start, ep.live_count, ep.pack_start};
  if (e == hipSuccess)
    e = launch_sort(ws.descs, n_prob, n_slots, L.n_bins, ws.hist, ws.cursor, ep, nullptr, po, s);
  if (e != hipSuccess) return hip_fail(e, "sample_initial");
  return ok();
}

sfhk_status sfhk_propagate(const sfhk_problem* probs, int32_t n_prob, const sfhk_ensemble* ens,
                           int32_t precision, double* accum, double* final_state,
                           double* snapshots, int32_t n_snap, int32_t snap_every,
                           void* workspace, size_t workspace_bytes, void* stream) {
  std::vector<Desc> descs;
  int64_t max_steps = 0;
  Layout L;
  sfhk_status st = propagate_prepare(probs, n_prob, ens, precision, accum, snapshots, n_snap,
                                     snap_every, descs, max_steps, L);
  if (st != SFHK_OK) return st;
  if (!workspace) return fail(SFHK_E_INVALID, "workspace is null");
  if (workspace_bytes < L.bytes)
    return fail(SFHK_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.bytes);
  if (ens->capacity == 0) return ok();
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = carve(workspace, L);
  if ((st = stage_problems(descs, ws, nullptr, max_steps, s)) != SFHK_OK) return st;
  return propagate_enqueue(n_prob, ens, precision, accum,
                           make_records(ens, final_state, snapshots, n_snap, snap_every), ws, L,
                           s);
}

sfhk_status sfhk_propagate_static(const sfhk_problem* probs, int32_t n_prob,
                                  const sfhk_ensemble* ens, int32_t precision, double* accum,
                                  double* final_state, double* snapshots, int32_t n_snap,
                                  int32_t snap_every, void* stream) {
  std::vector<Desc> descs;
  int64_t max_steps = 0;
  Layout L;
  sfhk_status st = propagate_prepare(probs, n_prob, ens, precision, accum, snapshots, n_snap,
                                     snap_every, descs, max_steps, L);
  if (st != SFHK_OK) return st;
  if (n_prob > kStaticMaxProblems)
    return fail(SFHK_E_NOMEM, "sfhk_propagate_static takes at most %d problems, got %d",
                kStaticMaxProblems, n_prob);
  if (L.bytes > kStaticScratchBytes)
    return fail(SFHK_E_NOMEM,
                "sfhk_propagate_static: these problems and %llu slots need %zu bytes of "
                "workspace, the static workspace holds %zu",
                (unsigned long long)ens->capacity, L.bytes, kStaticScratchBytes);
  if (ens->capacity == 0) return ok();
  void* base = nullptr;
  if ((st = static_scratch(&base)) != SFHK_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = carve(base, L);
  if ((st = stage_problems_by_args(descs, ws, max_steps, s)) != SFHK_OK) return st;
  return propagate_enqueue(n_prob, ens, precision, accum,
                           make_records(ens, final_state, snapshots, n_snap, snap_every), ws, L,
                           s);
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

int32_t sfhk_fft_log2_len(int32_t n_t) {
  if (n_t < 1 || n_t > (1 << 25)) return 0;
  int32_t b = 0;
  while ((int64_t(1) << b) < 8 * (int64_t)n_t) ++b;
  return b;
}

size_t sfhk_spectrum_fft_work_bytes(int32_t log2_len) {
  if (log2_len < 1 || log2_len > 28) return 0;
  return sizeof(double) * 4 * ((size_t)1 << log2_len);  // two complex arrays of L
}

sfhk_status sfhk_spectrum_fft(const double* v, int32_t n_t, double t_first, double dt,
                              double tau_H, int32_t log2_len, void* work, size_t work_bytes,
                              double* V_re, double* V_im, double* yield, double* phase,
                              void* stream) {
  if (n_t < 1) return fail(SFHK_E_INVALID, "n_t must be >= 1");
  if (log2_len < 1 || log2_len > 28 || (int64_t(1) << log2_len) < (int64_t)n_t)
    return fail(SFHK_E_INVALID, "log2_len must be in 1..28 with 2^log2_len >= n_t");
  if (!(is_finite(t_first) && is_finite(dt) && dt > 0 && is_finite(tau_H) && tau_H > 0))
    return fail(SFHK_E_INVALID, "t_first, dt > 0 and tau_H > 0 must be finite");
  if (!v || !work || !V_re || !V_im || !yield)
    return fail(SFHK_E_INVALID, "spectrum pointers must be non-null (phase may be)");
  const size_t need = sfhk_spectrum_fft_work_bytes(log2_len);
  if (work_bytes < need)
    return fail(SFHK_E_NOMEM, "work has %zu bytes, needs %zu", work_bytes, need);
  hipError_t e = launch_spectrum_fft(v, n_t, t_first, dt, tau_H, log2_len,
                                     static_cast<double2*>(work), V_re, V_im, yield, phase,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "spectrum fft");
  return ok();
}

sfhk_status sfhk_acceleration(const double* v, int32_t n_t, double t_first, double dt,
                              double tau_H, int32_t log2_len, void* work, size_t work_bytes,
                              double* a, void* stream) {
  if (n_t < 1) return fail(SFHK_E_INVALID, "n_t must be >= 1");
  if (log2_len < 1 || log2_len > 28 || (int64_t(1) << log2_len) < (int64_t)n_t)
    return fail(SFHK_E_INVALID, "log2_len must be in 1..28 with 2^log2_len >= n_t");
  if (!(is_finite(t_first) && is_finite(dt) && dt > 0 && is_finite(tau_H) && tau_H > 0))
    return fail(SFHK_E_INVALID, "t_first, dt > 0 and tau_H > 0 must be finite");
  if (!v || !work || !a) return fail(SFHK_E_INVALID, "v, work and a must be non-null");
  const size_t need = sfhk_spectrum_fft_work_bytes(log2_len);
  if (work_bytes < need)
    return fail(SFHK_E_NOMEM, "work has %zu bytes, needs %zu", work_bytes, need);
  hipError_t e = launch_acceleration_fft(v, n_t, t_first, dt, tau_H, log2_len,
                                         static_cast<double2*>(work), a,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "acceleration");
  return ok();
}

sfhk_status sfhk_return_steps(const sfhk_problem* probs, int32_t n_prob,
                              const sfhk_ensemble* ens, double r_return, int32_t* k_ret,
                              double* e_ret, void* workspace, size_t workspace_bytes,
                              void* stream) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if ((st = check_ensemble(ens)) != SFHK_OK) return st;
  if (!(is_finite(r_return) && r_return > 0)) return fail(SFHK_E_INVALID, "r_return must be > 0");
  if (ens->capacity > 0 && (!k_ret || !e_ret)) return fail(SFHK_E_INVALID, "outputs are null");
  std::vector<Desc> descs;
  int64_t max_steps = 0;
  Layout L = build_layout(probs, n_prob, ens->capacity, &descs, &max_steps, false, SFHK_FP64);
  if (!workspace) return fail(SFHK_E_INVALID, "workspace is null");
  if (workspace_bytes < L.bytes)
    return fail(SFHK_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.bytes);
  if (ens->capacity == 0) return ok();
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = carve(workspace, L);
  if ((st = stage_problems(descs, ws, nullptr, max_steps, s)) != SFHK_OK) return st;
  const uint64_t max_packs = (ens->capacity + kWave - 1) / kWave + (uint64_t)n_prob;
  if (max_packs > 0x7fffffffull) return fail(SFHK_E_UNSUPPORTED, "ensemble too large");
  hipError_t e = launch_fill_i32(k_ret, -1, ens->capacity, s);
  if (e == hipSuccess) e = launch_fill_f64(e_ret, 0.0, ens->capacity, s);
  if (e == hipSuccess)
    e = launch_returns(ws.descs, n_prob, ws.field, ens_ptrs(ens), (uint32_t)max_packs, r_return,
                       k_ret, e_ret, s);
  if (e != hipSuccess) return hip_fail(e, "return steps");
  return ok();
}

sfhk_status sfhk_gabor(const double* v, int32_t n_t, double t_first, double dt, double sigma,
                       const double* t_c, int32_t n_c, const double* omega, int32_t n_omega,
                       double* G_re, double* G_im, double* yield, void* stream) {
  if (n_t < 1) return fail(SFHK_E_INVALID, "n_t must be >= 1");
  if (n_c < 0 || n_omega < 0) return fail(SFHK_E_INVALID, "n_c and n_omega must be >= 0");
  if (n_c > 0 && (size_t)n_c * (size_t)n_omega > (size_t(1) << 31))
    return fail(SFHK_E_INVALID, "n_c * n_omega must be <= 2^31");
  if (!(is_finite(t_first) && is_finite(dt) && dt > 0 && is_finite(sigma) && sigma > 0))
    return fail(SFHK_E_INVALID, "t_first, dt > 0 and sigma > 0 must be finite");
  if (n_c == 0 || n_omega == 0) return ok();
  if (!v || !t_c || !omega || !G_re || !G_im || !yield)
    return fail(SFHK_E_INVALID, "gabor pointers must be non-null");
  hipError_t e = launch_gabor(v, n_t, t_first, dt, sigma, t_c, n_c, omega, n_omega, G_re, G_im,
                              yield, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "gabor");
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ plans

struct sfhk_plan {
  int n_prob = 0;
  int precision = SFHK_FP64;
  sfhk_tuning tune{};
  std::vector<Desc> descs;
  Layout L;
  Workspace ws{};
  EnsPtrs ens{};
  uint64_t capacity = 0, n_slots = 0;
  int64_t max_steps = 0;
  uint32_t grid = 0;
  uint32_t grid_latency = 0;  // persistent grid of the latency-form re-run
  double *accum = nullptr, *v = nullptr, *Vre = nullptr, *Vim = nullptr, *Y = nullptr;
  double h_step = 0.0;
  int n_omega = 0;
  uint32_t *qkeys = nullptr, *qhist = nullptr, *qcursor = nullptr, *queue = nullptr,
           *queue2 = nullptr, *counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // measurement: events around the trajectory kernel (0, 1) and the FP64
  // re-run (2, 3), recorded by sfhk_plan_run only
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ran_timed = false;
};

namespace {

// timed: record the plan's measurement events (not in a graph recording).
sfhk_status plan_enqueue(sfhk_plan* P, hipStream_t s, bool timed) {
  const int n_prob = P->n_prob;
  const Workspace& ws = P->ws;
  EnsPtrs ep = P->ens;
  LaunchCfg cfg;
  cfg.persistent = P->tune.persistent;
  cfg.unroll = P->tune.step_unroll;
  cfg.grid = P->grid;
  cfg.queue = P->queue;
  cfg.counter = P->counter;
  const uint32_t mp = P->L.max_packs;
  hipError_t e = launch_fill_u32(ws.hist, 0u, P->L.n_bins + 1, s);
  if (e == hipSuccess)
    e = launch_sample(ws.descs, n_prob, ws.slot_off, P->n_slots, ws.field, ep, ws.hist,
                      any_saddle(P->descs.data(), n_prob), s);
  PackOut po{ep.order, ep.live_start, ep.live_count, ep.pack_start};
  if (e == hipSuccess)
    e = launch_sort(ws.descs, n_prob, P->n_slots, P->L.n_bins, ws.hist, ws.cursor, ep, nullptr,
                    po, s);
  if (e == hipSuccess) e = launch_fill_f64(P->accum, 0.0, P->L.n_bins, s);
  if (e == hipSuccess && cfg.persistent) {
    e = launch_pack_queue(ws.descs, n_prob, ep, mp, P->L.n_len, P->qkeys, P->qhist, P->qcursor,
                          P->queue, s);
    if (e == hipSuccess) e = launch_fill_u32(P->counter, 0u, 2, s);
  }
  auto mark = [&](int i) {
    if (timed && e == hipSuccess) e = hipEventRecord(P->ev[i], s);
  };
  if (e == hipSuccess) {
    if (P->precision == SFHK_FP64) {
      // the same choice of form as sfhk_propagate: latency form far below fill
      mark(0);
      if (e == hipSuccess)
        e = mp <= kLatencyMaxPacks
                ? launch_propagate_latency(ws.descs, n_prob, ws.field, ep, nullptr, mp, P->accum,
                                           Records{}, s, cfg)
                : launch_propagate_f64(ws.descs, n_prob, ws.field, ep, nullptr, mp, P->accum,
                                       Records{}, s, cfg);
      mark(1);
    } else {
      e = launch_fill_i32(ws.redo, -1, P->capacity, s);
      mark(0);
      if (e == hipSuccess)
        e = launch_propagate_mixed(ws.descs, n_prob, ws.field, ep, ws.redo, mp, P->accum,
                                   Records{}, s, cfg);
      mark(1);
      if (e == hipSuccess) e = launch_fill_u32(ws.hist, 0u, P->L.n_bins + 1, s);
      if (e == hipSuccess) e = launch_count(ws.descs, P->n_slots, ep, ws.redo, ws.hist, s);
      PackOut p2{ws.order2, ws.runs2, ws.runs2 + n_prob, ws.runs2 + 2 * n_prob};
      if (e == hipSuccess)
        e = launch_sort(ws.descs, n_prob, P->n_slots, P->L.n_bins, ws.hist, ws.cursor, ep,
                        ws.redo, p2, s);
      EnsPtrs e2 = ep;
      e2.order = p2.order;
      e2.live_start = p2.live_start;
      e2.live_count = p2.live_count;
      e2.pack_start = p2.pack_start;
      LaunchCfg cfg2 = cfg;
      cfg2.queue = P->queue2;
      cfg2.counter = P->counter + 1;
      const bool lat = P->tune.lanes_per_traj == 8;
      if (lat && cfg.persistent) cfg2.grid = P->grid_latency;
      // the re-run of a launch above the latency threshold puts hundreds of
      // units on the SIMDs at once: units of two monodromy wavefronts
      cfg2.pipe_mono = mp > kLatencyMaxPacks ? 2 : 1;
      if (e == hipSuccess && cfg.persistent)
        e = launch_pack_queue(ws.descs, n_prob, e2, mp, P->L.n_len, P->qkeys, P->qhist,
                              P->qcursor, P->queue2, s);
      mark(2);
      if (e == hipSuccess)
        e = lat ? launch_propagate_latency(ws.descs, n_prob, ws.field, e2, ws.redo, mp, P->accum,
                                           Records{}, s, cfg2)
                : launch_propagate_f64(ws.descs, n_prob, ws.field, e2, ws.redo, mp, P->accum,
                                       Records{}, s, cfg2);
      mark(3);
    }
  }
  if (e == hipSuccess)
    e = launch_dipole_batched(ws.descs, n_prob, (uint32_t)(P->max_steps + 1), P->accum, P->v, s);
  if (e == hipSuccess)
    e = launch_spectrum_batched(ws.descs, n_prob, P->v, P->h_step, P->n_omega, P->Vre, P->Vim,
                                P->Y, s);
  if (e != hipSuccess) return hip_fail(e, "plan run");
  return SFHK_OK;
}

}  // namespace

extern "C" {

size_t sfhk_plan_workspace_bytes(const sfhk_problem* probs, int32_t n_prob,
                                 const uint64_t* n_per_prob) {
  if (check_problems(probs, n_prob) != SFHK_OK || !n_per_prob) return 0;
  uint64_t n = 0;
  for (int i = 0; i < n_prob; ++i) n += n_per_prob[i];
  g_err.clear();
  return build_layout(probs, n_prob, n, nullptr, nullptr, true).bytes;
}

sfhk_status sfhk_plan_create(const sfhk_problem* probs, int32_t n_prob,
                             const uint64_t* n_per_prob, const uint64_t* seeds,
                             const uint64_t* first_index, int32_t precision,
                             const sfhk_tuning* tuning, double h_step, int32_t n_omega,
                             const sfhk_ensemble* ens, void* workspace, size_t workspace_bytes,
                             double* accum, double* v, double* V_re, double* V_im, double* yield,
                             void* stream, sfhk_plan** plan) {
  sfhk_status st = check_problems(probs, n_prob);
  if (st != SFHK_OK) return st;
  if (!plan) return fail(SFHK_E_INVALID, "plan is null");
  *plan = nullptr;
  if (!n_per_prob || !seeds || !first_index)
    return fail(SFHK_E_INVALID, "n_per_prob, seeds and first_index must be non-null");
  if (precision != SFHK_FP64 && precision != SFHK_MIXED)
    return fail(SFHK_E_INVALID, "unknown precision %d", precision);
  if ((st = check_ensemble(ens)) != SFHK_OK) return st;
  if (!accum || !v) return fail(SFHK_E_INVALID, "accum and v must be non-null");
  if (n_omega < 0 || (n_omega > 0 && (!V_re || !V_im || !yield || !(h_step >= 0.0))))
    return fail(SFHK_E_INVALID, "spectrum outputs invalid");
  sfhk_tuning t{0, 8, 1, 1, 8};
  if (tuning) {
    t = *tuning;
    if (t.waves_per_cu == 0) t.waves_per_cu = 8;
    if (t.step_unroll == 0) t.step_unroll = 1;
    if (t.traj_per_lane == 0) t.traj_per_lane = 1;
    if (t.lanes_per_traj == 0) t.lanes_per_traj = 8;
  }
  if ((t.persistent != 0 && t.persistent != 1) || t.waves_per_cu < 1 || t.waves_per_cu > 32 ||
      (t.step_unroll != 1 && t.step_unroll != 2 && t.step_unroll != 4) ||
      (t.lanes_per_traj != 1 && t.lanes_per_traj != 8))
    return fail(SFHK_E_INVALID, "tuning out of range");
  if (t.traj_per_lane != 1)
    return fail(SFHK_E_UNSUPPORTED, "traj_per_lane %d: only 1 fits the register budget",
                t.traj_per_lane);
  std::vector<uint64_t> slot_off(n_prob + 1, 0);
  for (int i = 0; i < n_prob; ++i) {
    if (n_per_prob[i] > (uint64_t(1) << 32))
      return fail(SFHK_E_INVALID, "n_per_prob[%d] too large", i);
    slot_off[i + 1] = slot_off[i] + n_per_prob[i];
  }
  const uint64_t n_slots = slot_off[n_prob];
  if (n_slots > ens->capacity)
    return fail(SFHK_E_NOMEM, "sum(n_per_prob) exceeds ensemble capacity");
  std::unique_ptr<sfhk_plan> P(new (std::nothrow) sfhk_plan());
  if (!P) return fail(SFHK_E_NOMEM, "host allocation of the plan failed");
  P->L = build_layout(probs, n_prob, n_slots, &P->descs, &P->max_steps, true);
  if (P->L.n_bins + 1 >= (uint64_t(1) << 31))
    return fail(SFHK_E_UNSUPPORTED, "total step count of the problems too large");
  if (!workspace) return fail(SFHK_E_INVALID, "workspace is null");
  if (workspace_bytes < P->L.bytes)
    return fail(SFHK_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, P->L.bytes);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  for (int i = 0; i < n_prob; ++i) {
    P->descs[i].slot_off = slot_off[i];
    P->descs[i].n_slots = n_per_prob[i];
    P->descs[i].seed = seeds[i];
    P->descs[i].first_index = first_index[i];
  }
  P->n_prob = n_prob;
  P->precision = precision;
  P->tune = t;
  P->ws = carve(workspace, P->L);
  P->ens = ens_ptrs(ens);
  P->capacity = ens->capacity;
  P->n_slots = n_slots;
  P->grid = (uint32_t)cus * (uint32_t)t.waves_per_cu;
  P->grid_latency = (uint32_t)cus * 8;  // two wavefronts per SIMD
  P->accum = accum;
  P->v = v;
  P->Vre = V_re;
  P->Vim = V_im;
  P->Y = yield;
  P->h_step = h_step;
  P->n_omega = n_omega;
  char* b = static_cast<char*>(workspace);
  P->qkeys = reinterpret_cast<uint32_t*>(b + P->L.off_qkeys);
  P->qhist = reinterpret_cast<uint32_t*>(b + P->L.off_qhist);
  P->qcursor = reinterpret_cast<uint32_t*>(b + P->L.off_qcursor);
  P->queue = reinterpret_cast<uint32_t*>(b + P->L.off_queue);
  P->queue2 = reinterpret_cast<uint32_t*>(b + P->L.off_queue2);
  P->counter = reinterpret_cast<uint32_t*>(b + P->L.off_counter);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (hipEvent_t& ev : P->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      for (hipEvent_t& x : P->ev)
        if (x) hipEventDestroy(x);
      return hip_fail(e, "plan events");
    }
  }
  if ((st = stage_problems(P->descs, P->ws, &slot_off, P->max_steps, s)) != SFHK_OK) return st;
  // the host copy of the descriptors must outlive the asynchronous upload
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "plan set-up");
  *plan = P.release();
  return ok();
}

sfhk_status sfhk_plan_run(sfhk_plan* plan, void* stream) {
  if (!plan) return fail(SFHK_E_INVALID, "plan is null");
  sfhk_status st = plan_enqueue(plan, static_cast<hipStream_t>(stream), true);
  if (st == SFHK_OK) plan->ran_timed = true;
  return st == SFHK_OK ? ok() : st;
}

sfhk_status sfhk_plan_capture(sfhk_plan* plan, void* stream) {
  if (!plan) return fail(SFHK_E_INVALID, "plan is null");
  if (!stream) return fail(SFHK_E_INVALID, "graph capture needs a non-null stream");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->exec) {
    hipGraphExecDestroy(plan->exec);
    plan->exec = nullptr;
  }
  if (plan->graph) {
    hipGraphDestroy(plan->graph);
    plan->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "begin capture");
  sfhk_status st = plan_enqueue(plan, s, false);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (st != SFHK_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return hip_fail(e, "graph instantiate");
  }
  plan->graph = g;
  return ok();
}

sfhk_status sfhk_plan_replay(sfhk_plan* plan, void* stream) {
  if (!plan) return fail(SFHK_E_INVALID, "plan is null");
  if (!plan->exec) return fail(SFHK_E_INVALID, "plan has no recorded graph");
  hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return ok();
}

sfhk_status sfhk_plan_kernel_ms(sfhk_plan* plan, float ms[2]) {
  if (!plan || !ms) return fail(SFHK_E_INVALID, "plan and ms must be non-null");
  if (!plan->ran_timed) return fail(SFHK_E_INVALID, "the plan has not been run with sfhk_plan_run");
  ms[0] = ms[1] = 0.0f;
  hipError_t e = hipEventElapsedTime(&ms[0], plan->ev[0], plan->ev[1]);
  if (e == hipSuccess && plan->precision == SFHK_MIXED)
    e = hipEventElapsedTime(&ms[1], plan->ev[2], plan->ev[3]);
  if (e != hipSuccess) return hip_fail(e, "plan kernel times");
  return ok();
}

void sfhk_plan_destroy(sfhk_plan* plan) {
  if (!plan) return;
  if (plan->exec) hipGraphExecDestroy(plan->exec);
  if (plan->graph) hipGraphDestroy(plan->graph);
  for (hipEvent_t ev : plan->ev)
    if (ev) hipEventDestroy(ev);
  delete plan;
}

}  // extern "C"
