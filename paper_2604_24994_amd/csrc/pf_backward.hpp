// Backward pass entry (pf_backward.hip) and the forward state it consumes.
#pragma once

#include "pf_internal.hpp"

namespace pf {

struct BwdState {
  RecBuf rec;                 // contribution records of all views
  int64_t nrec = 0;           // records written
  int64_t nseg = 0;           // segments written
  int64_t npix = 0;           // pixels of all views
  pf_camera* cams_dev = nullptr;
};

pf_status backward_impl(const Scene& sc, const BwdState& st, const float* d_rgba, const pf_grads& g,
                        hipStream_t s);

}  // namespace pf
