// Internal declarations shared by the HIP translation units of libpowerfoam.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "powerfoam.h"

#define PF_HD __host__ __device__
#include "pf_record.hpp"

namespace pf {

constexpr int KD = 8;              // detail sites per face (built variant)
constexpr int MA = 8;              // Spherical-Voronoi axes per detail site
constexpr int TEXW = 3 + 6 * MA;   // floats per (cell, detail site)
constexpr int TILE = 16;           // raster tile edge in pixels
constexpr int FACE_CAP = 64;       // planes / faces per cell in the main build pass (larger cells take a second pass)
constexpr int LEAF = 64;           // sites per leaf of the build tree

// Per-cell flags written by the build.
constexpr int FLAG_EMPTY_POWER = 1;   // the power cell itself is empty
constexpr int FLAG_OVERFLOW = 2;      // build capacity exceeded (reason below)
constexpr int FLAG_OVER_VERTS = 4;    //   vertex slots
constexpr int FLAG_OVER_PLANES = 8;   //   live planes
constexpr int FLAG_OVER_WORK = 16;    //   work limit
constexpr int FLAG_OVER_STACK = 32;   //   traversal stack

// Implicit 64-ary tree over the Morton-sorted sites: level 0 = sites,
// level L >= 1 = nodes (box of their sites; lo.w = largest weight, hi.w =
// largest sphere radius).
constexpr int MAXLVL = 8;
struct Levels {
  int n;                          // number of node levels (>= 1)
  long long off[MAXLVL];          // offset of level L (1-based) in the node arrays
  long long cnt[MAXLVL + 1];      // cnt[0] = sites, cnt[L] = nodes at level L
};

struct Scene {
  int64_t n = 0;
  pf_params prm{};                 // caller arrays (device) and constants
  float box_min[3]{}, box_max[3]{};
  // packed per-cell records
  float4* geo = nullptr;           // (p, r)
  float4* nrm = nullptr;           // (unit normal, sigma)
  float* cull = nullptr;           // radius of a ball at p bounding the
                                   // non-empty bounded cell; < 0: hidden
  int32_t* flags = nullptr;
  int32_t* wit = nullptr;          // [n][8] per empty cell: sites that emptied it (next build's seeds)
  // adjacency, CSR; per cell: raster faces, other neighbour faces, box faces
  int32_t* row = nullptr;          // [n+1]
  int32_t* nrast = nullptr;        // [n] faces that can cut the sphere
  int32_t* col = nullptr;          // [E] neighbour, or -1-f for box face f
  float4* plane = nullptr;         // [E] (m, h): (x - p_i).m <= h
  int64_t n_faces = 0, n_hidden = 0, n_overflow = 0, n_big = 0, n_dropped = 0;
  double rec_per_pixel = 0.0;      // record-pool sizing hint for store mode (0: none yet)
  double seg_per_pixel = 0.0;      // segment-list sizing hint for store mode
  double pairs_per_cell = 0.0;     // tile pairs per (view, cell) of the last raster
  // the build's site tree, kept for the sphere-overlap (Cech) queries
  float4* t_sp = nullptr;          // [n] sorted (p, w)
  int32_t* t_sidx = nullptr;       // [n] original index
  float* t_srad = nullptr;         // [n] sorted radius
  float4* t_lo = nullptr;          // node boxes
  float4* t_hi = nullptr;
  Levels t_lv{};
};

// Contribution records written by the store-mode forward: one per (pixel,
// cell) with alpha > 0, chained per pixel back to front through `prev`.
//   ri = (cell, pixel within its view, prev record or -1,
//         pack_view_bind(view, bind0, bind1), see pf_record.hpp)
//   rf = (alpha, c.r, c.g, c.b); after the per-pixel pass (dL/dalpha, dL/dc)
//   rt = transmittance in front of the contribution
// bind: -1 sphere, -2 ray start, f >= 0 raster face index of the cell.
// Every wave-wide append of one cell's records is also listed as a segment
// (cell, first record, lane mask low 32 bits, high 32 bits): the records of
// a segment are contiguous, belong to one cell and, in lane order, to the
// lanes of the mask (count = popcount of the mask), which lets the backward
// group records by cell with one atomic per segment.  A wave reserves its
// segment slots in blocks; the first slot of a block is a header
// (-1, previous block of the wave or -1, 0, 0) with an empty mask, and the
// raster records each wave's last block, so that the backward can walk a
// wave's segments in reverse append order (back to front for every pixel of
// the wave).  The walk lists one-record segments (mask 1), without headers.
// Segment slots a raster wave reserves at a time (header included).
constexpr int SEG_BLOCK = 32;

// Records listed by a segment (0 for headers and unused slots).
__device__ inline int seg_count(const int4& g) { return __popc((uint32_t)g.z) + __popc((uint32_t)g.w); }

struct RecBuf {
  int4* ri = nullptr;
  float4* rf = nullptr;
  float* rt = nullptr;
  int32_t* head = nullptr;            // [pixels of all views] last record or -1
  unsigned long long* counter = nullptr;   // [2]: records, segments appended
  int4* seg = nullptr;
  int2* wtail = nullptr;              // raster: [4 x tiles] (last segment block or -1, slots used in it)
  int64_t cap = 0;                    // record capacity
  int64_t seg_cap = 0;                // segment capacity
};

// Thread-local error text.
void set_error(const std::string& msg);

// Device allocation helpers (stream-ordered); return false on failure with
// the error text set.
bool dmalloc(void** p, size_t bytes, hipStream_t s, const char* what);
void dfree(void* p, hipStream_t s);

// Library device memory: blocks cached by the library and reused
// stream-ordered.  pool_alloc returns a block usable on stream s; pool_free
// gives it back once the work queued on s so far has finished with it.
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
// The caller's allocator (NULL: the library's cache); the cache's limit;
// requested bytes in use, their high-water mark and the cached bytes.
void set_allocator(const pf_allocator* a);
void set_cache_limit(size_t bytes);
void memory_stats(int64_t* live, int64_t* peak, int64_t* cached, bool reset_peak);

// --- scan / sort utilities (pf_util.hip) ---------------------------------
// Exclusive prefix sum of n uint32 values; out may alias in.  Returns the
// total through *total_dev (device, may be null).  Scratch is allocated on
// the stream: scan_scratch_bytes(n) bytes at most, all live at once.
int64_t scan_scratch_bytes(int64_t n);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n,
                              uint32_t* total_dev, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bits,
                          hipStream_t s);

// --- build (pf_build.hip) -------------------------------------------------
// prev (may be null): a built scene of the same cells whose adjacency seeds
// each cell's first candidates (the result does not depend on it).
pf_status build_scene_impl(const pf_params& prm, const pf_build_opts& opt,
                           hipStream_t s, Scene* sc, const Scene* prev = nullptr);
// Frees the scene's arrays: stream-ordered on s (async), or synchronously.
void free_scene(Scene* sc, hipStream_t s = nullptr, bool async = false);
// lambda * sum_i sum_{j overlapping i} max(r_i + r_j - |p_i - p_j|, 0)^2 and
// its gradient (adds into g.p and g.radius; the value into *loss_dev).
pf_status connect_loss_impl(const Scene& sc, float lambda, const pf_grads& g, double* loss_dev, hipStream_t s);

// --- Steiner cells (pf_steiner.hip) --------------------------------------
pf_status steiner_impl(const pf_params& prm, const float* z, const pf_steiner_opts& opt, int64_t cap, float* out_p,
                       float* out_power, float* out_radius, int32_t* out_near, int64_t* round_counts,
                       int64_t* n_out, hipStream_t s);

// --- densify / prune (pf_densify.hip) ------------------------------------
pf_status ema_impl(float* ema, const float* value, int64_t n, float beta, hipStream_t s);
pf_status densify_impl(const pf_params& in, const float* err_ema, const float* contrib_ema, const float* u,
                       const float* delta, const pf_densify_opts& o, const pf_cell_arrays& out, float* out_err,
                       float* out_contrib, int32_t* out_parent, int64_t* n_kept, int64_t* n_drawn, hipStream_t s);

// --- kernel timing (pf_api.hip) ----------------------------------------
bool profiling();
// Records an event pair around a launch; call prof_begin before and
// prof_end after the launch on the same stream.
int prof_begin(const char* name, hipStream_t s);
void prof_end(int token, hipStream_t s);

struct ProfScope {
  int tok;
  hipStream_t s;
  ProfScope(const char* name, hipStream_t st) : tok(profiling() ? prof_begin(name, st) : -1), s(st) {}
  ~ProfScope() { if (tok >= 0) prof_end(tok, s); }
};

}  // namespace pf

#define PF_HIP_TRY(expr)                                                    \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) {                                                 \
      pf::set_error(std::string("HIP error ") + hipGetErrorString(_e) +    \
                    " at " + __FILE__ + ":" + std::to_string(__LINE__));    \
      return _e == hipErrorOutOfMemory ? PF_ERR_OOM : PF_ERR_HIP;           \
    }                                                                       \
  } while (0)
