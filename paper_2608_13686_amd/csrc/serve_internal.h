// Internal types of the time-sliced serving path.
#pragma once

#include "sfhk_internal.h"

namespace sfhk {

// Per-trajectory state saved between windows: the SFHK_FS_* fields up to the
// branch-flip count, plus the step at which the prefactor cap stopped the
// trajectory.
constexpr int kStateKend = SFHK_FS_FLIPS + 1;
constexpr int kStateFields = kStateKend + 1;

// One request's device view: its problem constants and the device buffers
// carved from its slice of the pool (one problem, so offsets are 0).
struct ReqDev {
  Desc desc;
  const double* field;
  double *accum, *v, *V_re, *V_im, *yield;
  int32_t *k0, *prob;
  double *qx, *qy, *qz, *px, *py, *pz, *w, *nx, *ny, *nz, *dph;
  uint32_t *order, *live_start, *live_count, *pack_start;
  double* state;     // [kStateFields][live_cap], indexed by pack position
  uint64_t live_cap;
  double h_step;
  int32_t n_omega, pad;
};
static_assert(sizeof(ReqDev) <= 3840, "ReqDev is passed by value as a kernel argument");

constexpr int kMaxSlice = 112;  // requests per window launch (kernel-argument table)

struct SliceEntry {
  uint32_t slot;        // request table index
  uint32_t pack_begin;  // first wavefront of this request in the launch
  int32_t k_from, k_to; // window of steps [k_from, k_to)
};

// A launch covers one pack group of every listed request: the packs
// group, group + n_groups, group + 2 n_groups, ... of each request.
struct SliceTable {
  int32_t n;
  uint16_t group, n_groups;
  SliceEntry e[kMaxSlice + 1];  // e[n].pack_begin = total wavefronts
};
static_assert(sizeof(SliceTable) <= 2048, "SliceTable is a kernel argument");

hipError_t launch_serve_slice(const ReqDev* reqs, const SliceTable& tab, hipStream_t s);
hipError_t launch_write_req(const ReqDev& r, ReqDev* dst, hipStream_t s);
hipError_t launch_request_finalize(const ReqDev* reqs, int slot, int n_kmax, int n_omega,
                                   hipStream_t s);

}  // namespace sfhk
