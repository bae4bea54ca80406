// Host entry points of the render translation unit.
#pragma once

#include <functional>
#include <string>

#include "pf_internal.hpp"

namespace pf {

bool camera_ok(const pf_camera& c, std::string* why);

// Composite of a binned group's tiles [first, first + count) (indices within
// the group), with records into r (null: plain).  The wave segment tails of
// the launch go to r->wtail[0 .. 4 count).
using GroupComposite = std::function<pf_status(int64_t first, int64_t count, const RecBuf* r)>;
// Called once per group of views after its binning: tiles_before = tiles of
// the earlier groups, ntiles = the group's tiles.
using GroupFn = std::function<pf_status(int64_t tiles_before, int64_t ntiles, const GroupComposite& run)>;

// All cameras of a call in groups of views; images back to back in rgba.
// Without fn: each group is composited whole, with records into rec (null:
// plain forward), wave segment tails indexed by the call's tile index.
// With fn: fn decides how each group is composited.
// counters (device, may be null): RASTER_COUNTERS work counters of the
// composite, accumulated.
constexpr int RASTER_COUNTERS = 6;
pf_status raster_views(Scene& sc, const pf_camera* cams, int ncam, float t_min, float* rgba, hipStream_t s,
                       const RecBuf* rec = nullptr, const GroupFn* fn = nullptr,
                       unsigned long long* counters = nullptr);
// Views per binning group, 16x16 tiles of a camera.
int raster_group_size(int64_t n, int ncam);
int64_t view_tiles(const pf_camera& c);
// Bytes raster_views allocates for one group (every buffer, all live at once
// at most), given its pair count.
int64_t raster_group_bytes(int64_t n, int nv, int64_t ntiles, int64_t np);
// Runs the cull-and-count pass of every group (no pairs emitted) and returns
// the largest group's raster_group_bytes.  Synchronises the stream.
pf_status raster_workspace(Scene& sc, const pf_camera* cams, int ncam, hipStream_t s, int64_t* bytes);
// Sum of the segments' record counts into *total_dev (device).
pf_status seg_record_total(const int4* seg, int64_t nseg, unsigned long long* total_dev, hipStream_t s);
// rec: store-mode records (null: plain walk); the records' view index and
// the offset of this view's pixels in the per-pixel arrays; the tiles
// [tile_first, tile_first + tile_count) of the view (tile_count < 0: to the end).
// scratch: device memory of the start-cell search given by the caller (null:
// taken from the library's allocator for the call).
struct TraceScratch {
  double* pk;        // [TRACE_START_BLOCKS] per-block least power distance
  long long* pi;     // [TRACE_START_BLOCKS] its cell
  int32_t* start;    // [1] the start cell
};
constexpr int TRACE_START_BLOCKS = 1024;
// counters (device, may be null): TRACE_COUNTERS work counters of the walk,
// accumulated.
constexpr int TRACE_COUNTERS = 6;
pf_status trace_view(const Scene& sc, const pf_camera& cam, float t_min, int max_steps, float* rgba,
                     unsigned long long* trunc_dev, hipStream_t s, const RecBuf* rec = nullptr, int view = 0,
                     int64_t pix_base = 0, int64_t tile_first = 0, int64_t tile_count = -1,
                     const TraceScratch* scratch = nullptr, unsigned long long* counters = nullptr);

}  // namespace pf
