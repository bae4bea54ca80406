// Backward pass entry (pf_backward.hip) and the forward state it consumes.
#pragma once

#include "pf_internal.hpp"

namespace pf {

struct BwdState {
  RecBuf rec;                 // contribution records of all views
  int64_t nrec = 0;           // records written
  int64_t nseg = 0;           // segments written
  int64_t npix = 0;           // pixels of all views
  int32_t ncam = 0;           // views
  int64_t ntiles = 0;         // 16x16 tiles the records cover (grid of the per-pixel pass)
  int64_t tile0 = 0;          // global index of the first of them (over the tiles of all views)
  pf_camera* cams_dev = nullptr;
};

// Options of the backward: normal-loss weight and the statistic outputs
// (device pointers, may be null).
struct BwdOpts {
  float lambda_normal = 0.0f;
  float* contribution = nullptr;   // [n] += sum of T a per cell
  double* normal_loss = nullptr;   // [1] += sum of T a max(n.d, 0)^2
  const float* pixel_error = nullptr;   // [pixels] per-pixel error e
  float* error = nullptr;          // [n] += sum of T a e per cell
};

pf_status backward_impl(const Scene& sc, const BwdState& st, const float* d_rgba, const pf_grads& g,
                        const BwdOpts& o, hipStream_t s);
// Bytes backward_impl allocates at most for a state of record capacity cap
// (every buffer, all live at once at most).
int64_t backward_bytes(int64_t n, int64_t cap, bool want_err);

}  // namespace pf
