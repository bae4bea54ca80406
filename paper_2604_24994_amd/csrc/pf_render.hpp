// Host entry points of the render translation unit.
#pragma once

#include <string>

#include "pf_internal.hpp"

namespace pf {

bool camera_ok(const pf_camera& c, std::string* why);
// All cameras of a call in one batch; images back to back in rgba.
// rec: store-mode records (null: plain forward).
pf_status raster_views(Scene& sc, const pf_camera* cams, int ncam, float t_min, float* rgba, hipStream_t s,
                       const RecBuf* rec = nullptr);
// Sum of the segments' record counts into *total_dev (device).
pf_status seg_record_total(const int4* seg, int64_t nseg, unsigned long long* total_dev, hipStream_t s);
// rec: store-mode records (null: plain walk); the records' view index and
// the offset of this view's pixels in the per-pixel arrays.
pf_status trace_view(const Scene& sc, const pf_camera& cam, float t_min, int max_steps, float* rgba,
                     unsigned long long* trunc_dev, hipStream_t s, const RecBuf* rec = nullptr, int view = 0,
                     int64_t pix_base = 0);

}  // namespace pf
