// C ABI of the time-sliced serving path: per-request buffer layout, admission
// (field table, sampling and packing of one request into its own buffers),
// one window launch over many requests, and per-request finalisation.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "serve_internal.h"

using namespace sfhk;

// shared with abi.hip (same library)
namespace sfhk_abi_detail {
sfhk_status check_problem_ext(const sfhk_problem* p, int idx);
Desc make_desc_ext(const sfhk_problem& p);
sfhk_status fail_ext(sfhk_status st, const char* msg);
sfhk_status hip_fail_ext(hipError_t e, const char* where);
sfhk_status ok_ext();
}  // namespace sfhk_abi_detail

using namespace sfhk_abi_detail;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ReqLayout {
  size_t field, accum, v, vre, vim, yield, k0, prob, f64[11], order, runs, hist, cursor, state,
      slot_off, bytes;
};

ReqLayout req_layout(int64_t N, uint64_t n, int32_t n_omega) {
  ReqLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.field = take(sizeof(double) * 2 * (size_t)(N + 1));
  L.accum = take(sizeof(double) * (size_t)(N + 1));
  L.v = take(sizeof(double) * (size_t)(N + 1));
  L.vre = take(sizeof(double) * (size_t)n_omega);
  L.vim = take(sizeof(double) * (size_t)n_omega);
  L.yield = take(sizeof(double) * (size_t)n_omega);
  L.k0 = take(sizeof(int32_t) * n);
  L.prob = take(sizeof(int32_t) * n);
  for (int i = 0; i < 11; ++i) L.f64[i] = take(sizeof(double) * n);
  L.order = take(sizeof(uint32_t) * n);
  L.runs = take(sizeof(uint32_t) * 4);
  L.hist = take(sizeof(uint32_t) * (size_t)(N + 2));
  L.cursor = take(sizeof(uint32_t) * (size_t)(N + 2));
  L.state = take(sizeof(double) * (size_t)kStateFields * n);
  L.slot_off = take(sizeof(uint64_t) * 2);
  L.bytes = o;
  return L;
}

int64_t steps_of(const sfhk_problem* p) {
  Desc d = make_desc_ext(*p);
  return d.N;
}

// The request's device view: its problem constants and its buffers carved
// from `buffer` by req_layout.
ReqDev carve_request(const sfhk_problem* p, uint64_t n_traj, uint64_t seed, uint64_t first_index,
                     double h_step, int32_t n_omega, void* buffer, const ReqLayout& L) {
  char* b = static_cast<char*>(buffer);
  ReqDev r;
  std::memset(&r, 0, sizeof r);
  r.desc = make_desc_ext(*p);
  r.desc.field_off = 0;
  r.desc.acc_off = 0;
  r.desc.slot_off = 0;
  r.desc.n_slots = n_traj;
  r.desc.seed = seed;
  r.desc.first_index = first_index;
  r.field = reinterpret_cast<double*>(b + L.field);
  r.accum = reinterpret_cast<double*>(b + L.accum);
  r.v = reinterpret_cast<double*>(b + L.v);
  r.V_re = reinterpret_cast<double*>(b + L.vre);
  r.V_im = reinterpret_cast<double*>(b + L.vim);
  r.yield = reinterpret_cast<double*>(b + L.yield);
  r.k0 = reinterpret_cast<int32_t*>(b + L.k0);
  r.prob = reinterpret_cast<int32_t*>(b + L.prob);
  double** f64[11] = {&r.qx, &r.qy, &r.qz, &r.px, &r.py, &r.pz, &r.w,
                      &r.nx, &r.ny, &r.nz, &r.dph};
  for (int i = 0; i < 11; ++i) *f64[i] = reinterpret_cast<double*>(b + L.f64[i]);
  r.order = reinterpret_cast<uint32_t*>(b + L.order);
  uint32_t* runs = reinterpret_cast<uint32_t*>(b + L.runs);
  r.live_start = runs;
  r.live_count = runs + 1;
  r.pack_start = runs + 2;
  r.state = reinterpret_cast<double*>(b + L.state);
  r.live_cap = n_traj;
  r.h_step = h_step;
  r.n_omega = n_omega;
  return r;
}

EnsPtrs ens_of(const ReqDev& r) {
  return EnsPtrs{r.k0, r.prob, r.qx, r.qy, r.qz, r.px, r.py, r.pz, r.w, r.nx, r.ny, r.nz,
                 r.dph, r.order, r.live_start, r.live_count, r.pack_start};
}

}  // namespace

extern "C" {

size_t sfhk_request_bytes(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega) {
  if (check_problem_ext(p, 0) != SFHK_OK || n_omega < 0) return 0;
  return req_layout(steps_of(p), n_traj, n_omega).bytes;
}

sfhk_status sfhk_request_layout(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega,
                                size_t offsets[4]) {
  sfhk_status st = check_problem_ext(p, 0);
  if (st != SFHK_OK) return st;
  if (!offsets || n_omega < 0) return fail_ext(SFHK_E_INVALID, "offsets null or n_omega < 0");
  ReqLayout L = req_layout(steps_of(p), n_traj, n_omega);
  offsets[0] = L.v;
  offsets[1] = L.vre;
  offsets[2] = L.vim;
  offsets[3] = L.yield;
  return ok_ext();
}

size_t sfhk_request_table_bytes(int32_t max_requests) {
  if (max_requests < 1) return 0;
  return sizeof(ReqDev) * (size_t)max_requests;
}

sfhk_status sfhk_request_init(const sfhk_problem* p, uint64_t n_traj, uint64_t seed,
                              uint64_t first_index, double h_step, int32_t n_omega,
                              void* buffer, size_t buffer_bytes, void* table, int32_t table_slots,
                              int32_t slot, void* stream) {
  sfhk_status st = check_problem_ext(p, 0);
  if (st != SFHK_OK) return st;
  if (!buffer || !table || slot < 0 || slot >= table_slots)
    return fail_ext(SFHK_E_INVALID, "buffer/table/slot invalid");
  if (n_traj == 0 || n_traj >= (uint64_t(1) << 31))
    return fail_ext(SFHK_E_INVALID, "n_traj must be in 1..2^31-1");
  if (n_omega < 0 || !(h_step >= 0.0)) return fail_ext(SFHK_E_INVALID, "spectrum grid invalid");
  const int64_t N = steps_of(p);
  ReqLayout L = req_layout(N, n_traj, n_omega);
  if (buffer_bytes < L.bytes) return fail_ext(SFHK_E_NOMEM, "request buffer too small");
  char* b = static_cast<char*>(buffer);
  ReqDev r = carve_request(p, n_traj, seed, first_index, h_step, n_omega, buffer, L);
  ReqDev* dst = static_cast<ReqDev*>(table) + slot;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* hist = reinterpret_cast<uint32_t*>(b + L.hist);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(b + L.cursor);
  uint64_t* slot_off = reinterpret_cast<uint64_t*>(b + L.slot_off);
  EnsPtrs ep = ens_of(r);
  const Desc* ddev = &dst->desc;
  hipError_t e = launch_write_req(r, dst, s);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(slot_off), 0u, 4, s);
  double* field = reinterpret_cast<double*>(b + L.field);
  if (e == hipSuccess) e = launch_field(ddev, 1, field, (uint64_t)N + 1, s);
  if (e == hipSuccess) e = launch_fill_u32(hist, 0u, (uint64_t)N + 2, s);
  if (e == hipSuccess)
    e = launch_sample(ddev, 1, slot_off, n_traj, r.field, ep, hist, any_saddle(&r.desc, 1), s);
  PackOut po{r.order, r.live_start, r.live_count, r.pack_start};
  if (e == hipSuccess)
    e = launch_sort(ddev, 1, n_traj, (uint64_t)N + 1, hist, cursor, ep, nullptr, po, s);
  if (e == hipSuccess) e = launch_fill_f64(r.accum, 0.0, (uint64_t)N + 1, s);
  if (e != hipSuccess) return hip_fail_ext(e, "request init");
  return ok_ext();
}

sfhk_status sfhk_serve_window(void* table, int32_t table_slots, int32_t n, const int32_t* slots,
                              const uint64_t* n_traj, const int32_t* k_from, const int32_t* k_to,
                              int32_t group, int32_t n_groups, void* stream) {
  if (!table || n < 0 || (n > 0 && (!slots || !n_traj || !k_from || !k_to)))
    return fail_ext(SFHK_E_INVALID, "window arguments invalid");
  if (n_groups < 1 || n_groups > 64 || group < 0 || group >= n_groups)
    return fail_ext(SFHK_E_INVALID, "pack group must satisfy 0 <= group < n_groups <= 64");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int i = 0;
  while (i < n) {  // at most kMaxSlice requests per launch
    SliceTable tab;
    std::memset(&tab, 0, sizeof tab);
    tab.group = (uint16_t)group;
    tab.n_groups = (uint16_t)n_groups;
    uint32_t waves = 0;
    int m = 0;
    for (; i < n && m < kMaxSlice; ++i, ++m) {
      if (slots[i] < 0 || slots[i] >= table_slots || k_from[i] < 0 || k_to[i] <= k_from[i])
        return fail_ext(SFHK_E_INVALID, "window entry invalid");
      const uint64_t all = (n_traj[i] + kWave - 1) / kWave;  // packs of the request
      const uint64_t packs = all > (uint64_t)group ? (all - group + n_groups - 1) / n_groups : 0;
      // the launch holds waves * 64 work-items, which must stay below 2^32
      if ((uint64_t)waves + packs > 0xffffffffull / kWave)
        return fail_ext(SFHK_E_UNSUPPORTED, "window too large");
      tab.e[m].slot = (uint32_t)slots[i];
      tab.e[m].pack_begin = waves;
      tab.e[m].k_from = k_from[i];
      tab.e[m].k_to = k_to[i];
      waves += (uint32_t)packs;
    }
    tab.n = m;
    tab.e[m].pack_begin = waves;
    hipError_t e = launch_serve_slice(static_cast<const ReqDev*>(table), tab, s);
    if (e != hipSuccess) return hip_fail_ext(e, "serve window");
  }
  return ok_ext();
}

sfhk_status sfhk_request_run(const sfhk_problem* p, uint64_t n_traj, int32_t n_omega,
                             void* buffer, size_t buffer_bytes, void* table, int32_t table_slots,
                             int32_t slot, void* stream) {
  sfhk_status st = check_problem_ext(p, 0);
  if (st != SFHK_OK) return st;
  if (!buffer || !table || slot < 0 || slot >= table_slots || n_omega < 0)
    return fail_ext(SFHK_E_INVALID, "buffer/table/slot/n_omega invalid");
  if (n_traj == 0 || n_traj >= (uint64_t(1) << 31))
    return fail_ext(SFHK_E_INVALID, "n_traj must be in 1..2^31-1");
  const ReqLayout L = req_layout(steps_of(p), n_traj, n_omega);
  if (buffer_bytes < L.bytes) return fail_ext(SFHK_E_NOMEM, "request buffer too small");
  // host-side pointers into the request's buffer; seed and grid do not enter
  // the propagation
  const ReqDev r = carve_request(p, n_traj, 0, 0, 0.0, n_omega, buffer, L);
  const Desc* ddev = &(static_cast<const ReqDev*>(table) + slot)->desc;
  const uint32_t max_packs = (uint32_t)((n_traj + kWave - 1) / kWave + 1);
  hipError_t e = launch_propagate_f64(ddev, 1, r.field, ens_of(r), nullptr, max_packs, r.accum,
                                      Records{}, static_cast<hipStream_t>(stream), LaunchCfg{});
  if (e != hipSuccess) return hip_fail_ext(e, "request run");
  return ok_ext();
}

sfhk_status sfhk_request_finalize(const sfhk_problem* p, int32_t n_omega, void* table,
                                  int32_t table_slots, int32_t slot, void* stream) {
  sfhk_status st = check_problem_ext(p, 0);
  if (st != SFHK_OK) return st;
  if (!table || slot < 0 || slot >= table_slots || n_omega < 0)
    return fail_ext(SFHK_E_INVALID, "finalize arguments");
  hipError_t e = launch_request_finalize(static_cast<const ReqDev*>(table), slot,
                                         (int)steps_of(p) + 1, n_omega,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail_ext(e, "request finalize");
  return ok_ext();
}

}  // extern "C"
