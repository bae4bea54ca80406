// C ABI entry points: argument checks, error text, handle lifetime.
#include <algorithm>
#include <atomic>
#include <functional>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pf_backward.hpp"
#include "pf_internal.hpp"
#include "pf_render.hpp"

struct pf_scene {
  pf::Scene s;
  pf_build_opts opts;   // kept for pf_update_scene
};

namespace {
// process-wide record-pool sizing hints (records / segment slots per pixel)
std::atomic<double> g_rec_hint{16.0};
std::atomic<double> g_seg_hint{4.0};
}  // namespace

struct pf_fwd_state {
  pf_scene* scene = nullptr;
  pf::BwdState st;
  std::vector<pf_camera> cams;
  int kind = 0;          // 0 raster, 1 ray walk
  int mode = 0;          // 0 records stored, 1 recomputed by pf_backward
  bool consumed = false; // store mode: pf_backward has overwritten the records
  float t_min = 1e-6f;
  int max_steps = 4096;
  int64_t limit = 0;     // workspace limit of the render options (0: none)
  hipStream_t stream = nullptr;   // the stream it was rendered on: its memory is freed there
};

namespace {
void free_records(pf::RecBuf& r, hipStream_t s) {
  void* ptrs[] = {r.ri, r.rf, r.rt, r.head, r.counter, r.seg, r.wtail};
  for (void* q : ptrs)
    if (q) pf::pool_free(q, s);
  r = pf::RecBuf{};
}

void free_state_mem(pf_fwd_state* s) {
  free_records(s->st.rec, s->stream);
  if (s->st.cams_dev) pf::pool_free(s->st.cams_dev, s->stream);
  s->st.cams_dev = nullptr;
}

// Device bytes of a record pool of cap record slots and seg_cap segment slots.
constexpr int64_t REC_BYTES = sizeof(int4) + sizeof(float4) + sizeof(float);   // 36
constexpr int64_t SEG_BYTES = sizeof(int4);                                    // 16
// recompute window without a limit: at 1M cells and 8 views of 1600x1066 a
// 1 GiB window replays the step in 18 windows (218 ms, 1.9 GiB peak), 2 GiB in
// 8 (182 ms, 3.0 GiB), 4 GiB in 5 (178 ms, 5.1 GiB)
constexpr int64_t DEFAULT_WINDOW = int64_t(2) << 30;

struct Caps {
  int64_t cap = 0, seg_cap = 0;
};

// Segment slots per record slot: one per record for the walk, else the
// scene's ratio of its last raster (at least 1/16).
double seg_ratio(const pf::Scene& sc, int kind) {
  if (kind == 1) return 1.0;
  const double rpp = sc.rec_per_pixel > 0.0 ? sc.rec_per_pixel : g_rec_hint.load();
  const double spp = sc.rec_per_pixel > 0.0 ? sc.seg_per_pixel : g_seg_hint.load();
  return std::min(1.0, std::max(1.0 / 16.0, spp / std::max(rpp, 1e-9)));
}

// The largest pool of at most `bytes`.
Caps caps_within(int64_t bytes, double ratio) {
  Caps c;
  c.cap = std::max<int64_t>(1, (int64_t)((double)bytes / ((double)REC_BYTES + SEG_BYTES * ratio)));
  c.cap = std::min<int64_t>(c.cap, INT32_MAX - 1);
  c.seg_cap = std::max<int64_t>(1, std::min<int64_t>((int64_t)(ratio * (double)c.cap), INT32_MAX - 1));
  while (c.cap * REC_BYTES + c.seg_cap * SEG_BYTES > bytes && c.cap > 1) {
    c.cap -= 1 + c.cap / 64;
    c.seg_cap = std::max<int64_t>(1, (int64_t)(ratio * (double)c.cap));
  }
  return c;
}

int64_t pool_bytes(const Caps& c) { return c.cap * REC_BYTES + c.seg_cap * SEG_BYTES; }
}  // namespace

namespace pf {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

namespace {
struct ProfRec {
  std::string name;
  hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::vector<ProfRec> g_prof;
}  // namespace

bool profiling() { return g_prof_on.load(std::memory_order_relaxed); }

int prof_begin(const char* name, hipStream_t s) {
  ProfRec r{name, nullptr, nullptr};
  if (hipEventCreate(&r.e0) != hipSuccess) return -1;
  if (hipEventCreate(&r.e1) != hipSuccess) {
    (void)hipEventDestroy(r.e0);
    return -1;
  }
  (void)hipEventRecord(r.e0, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

void prof_end(int token, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (token >= 0 && token < (int)g_prof.size()) (void)hipEventRecord(g_prof[token].e1, s);
}

}  // namespace pf

namespace {

pf_status invalid(const std::string& msg) {
  pf::set_error(msg);
  return PF_ERR_INVALID;
}

int64_t image_floats(const pf_camera* cams, int32_t ncam) {
  int64_t t = 0;
  for (int c = 0; c < ncam; ++c) t += 4ll * cams[c].width * cams[c].height;
  return t;
}

}  // namespace


extern "C" {

const char* pf_last_error(void) { return pf::g_error.c_str(); }

static pf_status check_params(const pf_params* params, const char* who) {
  const std::string w(who);
  if (!params) return invalid(w + ": params is NULL");
  const pf_params& p = *params;
  if (p.n < 1) return invalid(w + ": n must be >= 1");
  if (p.n >= (1ll << 30)) return invalid(w + ": n must be < 2^30");
  if (!p.p || !p.power || !p.radius || !p.normal || !p.occ_logit || !p.rgb || !p.tex)
    return invalid(w + ": a parameter array is NULL");
  if (p.k_detail < 1 || p.m_axes < 1) return invalid(w + ": k_detail and m_axes must be >= 1");
  if (p.k_detail != pf::KD || p.m_axes != pf::MA) {
    pf::set_error(w + ": only k_detail = 8 and m_axes = 8 are built");
    return PF_ERR_UNSUPPORTED;
  }
  if (!std::isfinite(p.sigma_scale) || !(p.sigma_scale >= 0) || !std::isfinite(p.tau))
    return invalid(w + ": sigma_scale and tau must be finite, sigma_scale >= 0");
  return PF_OK;
}

pf_status pf_build_scene(const pf_params* params, const pf_build_opts* opts, void* stream, pf_scene** out) {
  if (!out) return invalid("pf_build_scene: out is NULL");
  *out = nullptr;
  {
    const pf_status st = check_params(params, "pf_build_scene");
    if (st != PF_OK) return st;
  }
  const pf_params& p = *params;
  pf_build_opts o{};
  o.box_min[0] = 1.0f;
  o.box_max[0] = -1.0f;
  o.box_pad = 0.01f;
  if (opts) o = *opts;
  pf_scene* sc = new (std::nothrow) pf_scene();
  if (!sc) {
    pf::set_error("pf_build_scene: host allocation failed");
    return PF_ERR_OOM;
  }
  sc->opts = o;
  pf_status st = pf::build_scene_impl(p, o, (hipStream_t)stream, &sc->s);
  if (st != PF_OK) {
    pf::free_scene(&sc->s);
    delete sc;
    return st;
  }
  *out = sc;
  return PF_OK;
}

pf_status pf_update_scene(pf_scene* scene, const pf_params* params, void* stream) {
  if (!scene) return invalid("pf_update_scene: scene is NULL");
  {
    const pf_status st = check_params(params, "pf_update_scene");
    if (st != PF_OK) return st;
  }
  pf::Scene fresh;
  const pf_status st = pf::build_scene_impl(*params, scene->opts, (hipStream_t)stream, &fresh, &scene->s);
  if (st != PF_OK) {
    pf::free_scene(&fresh, (hipStream_t)stream, true);
    return st;
  }
  fresh.rec_per_pixel = scene->s.rec_per_pixel;
  fresh.seg_per_pixel = scene->s.seg_per_pixel;
  fresh.pairs_per_cell = scene->s.pairs_per_cell;
  pf::free_scene(&scene->s, (hipStream_t)stream, true);
  scene->s = fresh;
  return PF_OK;
}

pf_status pf_scene_info_get(const pf_scene* scene, pf_scene_info* info) {
  if (!scene || !info) return invalid("pf_scene_info_get: NULL argument");
  info->n = scene->s.n;
  info->n_faces = scene->s.n_faces;
  info->n_hidden = scene->s.n_hidden;
  info->n_overflow = scene->s.n_overflow;
  info->n_high_degree = scene->s.n_big;
  info->n_dropped = scene->s.n_dropped;
  for (int a = 0; a < 3; ++a) {
    info->box_min[a] = scene->s.box_min[a];
    info->box_max[a] = scene->s.box_max[a];
  }
  return PF_OK;
}

pf_status pf_scene_adjacency(const pf_scene* scene, int32_t* row, int32_t* col, void* stream) {
  if (!scene || !row || !col) return invalid("pf_scene_adjacency: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  PF_HIP_TRY(hipMemcpyAsync(row, scene->s.row, sizeof(int32_t) * (scene->s.n + 1), hipMemcpyDeviceToDevice, s));
  if (scene->s.n_faces)
    PF_HIP_TRY(hipMemcpyAsync(col, scene->s.col, sizeof(int32_t) * scene->s.n_faces, hipMemcpyDeviceToDevice, s));
  return PF_OK;
}

void pf_scene_destroy(pf_scene* scene) {
  if (!scene) return;
  pf::free_scene(&scene->s);
  delete scene;
}

static pf_status check_render(pf_scene* scene, const pf_camera* cams, int32_t ncam, const float* rgba,
                              const char* who) {
  if (!scene) return invalid(std::string(who) + ": scene is NULL");
  if (!cams || ncam < 1) return invalid(std::string(who) + ": need ncam >= 1 cameras");
  if (!rgba) return invalid(std::string(who) + ": rgba is NULL");
  for (int c = 0; c < ncam; ++c) {
    std::string why;
    if (!pf::camera_ok(cams[c], &why)) return invalid(std::string(who) + ": camera " + std::to_string(c) + ": " + why);
  }
  return PF_OK;
}

namespace {

// The pass that produces a forward state's records: kind 0 tile raster,
// kind 1 ray walk (one view after the other).
pf_status run_pass(pf_scene* scene, const std::vector<pf_camera>& cams, int kind, float t_min, int max_steps,
                   float* rgba, unsigned long long* trunc_dev, hipStream_t s, const pf::RecBuf* rec,
                   unsigned long long* counters = nullptr) {
  const int ncam = (int)cams.size();
  if (kind == 0) return pf::raster_views(scene->s, cams.data(), ncam, t_min, rgba, s, rec, nullptr, counters);
  int64_t off = 0;
  for (int c = 0; c < ncam; ++c) {
    const pf_status st = pf::trace_view(scene->s, cams[c], t_min, max_steps, rgba + 4 * off, trunc_dev, s, rec, c, off,
                                        0, -1, nullptr, counters);
    if (st != PF_OK) return st;
    off += (int64_t)cams[c].width * cams[c].height;
  }
  return PF_OK;
}

// New state with the cameras on the device (no records yet).
pf_status new_state(pf_scene* scene, const pf_camera* cams, int32_t ncam, int kind, int mode, float t_min,
                    int max_steps, int64_t limit, hipStream_t s, pf_fwd_state** out, const char* who) {
  *out = nullptr;
  // the records store the view in 12 bits (pf_record.hpp)
  if (ncam > pf::REC_MAX_VIEWS) return invalid(std::string(who) + ": at most 4096 cameras per call with a forward state");
  pf_fwd_state* fs = new (std::nothrow) pf_fwd_state();
  if (!fs) {
    pf::set_error(std::string(who) + ": host allocation failed");
    return PF_ERR_OOM;
  }
  fs->scene = scene;
  fs->cams.assign(cams, cams + ncam);
  fs->kind = kind;
  fs->mode = mode;
  fs->t_min = t_min;
  fs->max_steps = max_steps;
  fs->limit = limit;
  fs->stream = s;
  int64_t npix = 0, ntiles = 0;
  for (int c = 0; c < ncam; ++c) {
    npix += (int64_t)cams[c].width * cams[c].height;
    ntiles += pf::view_tiles(cams[c]);
  }
  fs->st.npix = npix;
  fs->st.ncam = ncam;
  fs->st.ntiles = ntiles;
  hipError_t e = pf::pool_alloc((void**)&fs->st.cams_dev, sizeof(pf_camera) * ncam, s);
  if (e == hipSuccess) e = hipMemcpyAsync(fs->st.cams_dev, cams, sizeof(pf_camera) * ncam, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    pf::set_error(std::string(who) + ": " + hipGetErrorString(e));
    free_state_mem(fs);
    delete fs;
    return e == hipErrorOutOfMemory ? PF_ERR_OOM : PF_ERR_HIP;
  }
  *out = fs;
  return PF_OK;
}

pf_status hip_status(hipError_t e, const char* who) {
  pf::set_error(std::string(who) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? PF_ERR_OOM : PF_ERR_HIP;
}

// Per-pixel heads and counters of a record buffer; wtail_tiles raster tiles
// of segment tails (0: none, the walk).
pf_status alloc_record_meta(pf::RecBuf& r, int64_t npix, int64_t wtail_tiles, hipStream_t s, const char* who) {
  hipError_t e = pf::pool_alloc((void**)&r.head, sizeof(int32_t) * npix, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&r.counter, 3 * sizeof(unsigned long long), s);
  if (e == hipSuccess && wtail_tiles > 0) e = pf::pool_alloc((void**)&r.wtail, sizeof(int2) * 4 * wtail_tiles, s);
  return e == hipSuccess ? PF_OK : hip_status(e, who);
}

pf_status alloc_pool(pf::RecBuf& r, const Caps& c, hipStream_t s, const char* who) {
  r.cap = c.cap;
  r.seg_cap = c.seg_cap;
  hipError_t e = pf::pool_alloc((void**)&r.ri, sizeof(int4) * c.cap, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&r.rf, sizeof(float4) * c.cap, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&r.rt, sizeof(float) * c.cap, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&r.seg, sizeof(int4) * c.seg_cap, s);
  return e == hipSuccess ? PF_OK : hip_status(e, who);
}

void free_pool(pf::RecBuf& r, hipStream_t s) {
  void* pool[] = {r.ri, r.rf, r.rt, r.seg};
  for (void* q : pool)
    if (q) pf::pool_free(q, s);
  r.ri = nullptr;
  r.rf = nullptr;
  r.rt = nullptr;
  r.seg = nullptr;
}

// Clears the pool's counters (and, for the walk, its segment slots: unused
// slots of a wave's blocks must read as empty) before a pass.
pf_status reset_pool(pf::RecBuf& r, bool walk, hipStream_t s, const char* who) {
  hipError_t e = hipMemsetAsync(r.counter, 0, 3 * sizeof(unsigned long long), s);
  if (e == hipSuccess && walk) e = hipMemsetAsync(r.seg, 0, sizeof(int4) * r.seg_cap, s);
  return e == hipSuccess ? PF_OK : hip_status(e, who);
}

// After a pass: slots reserved (records, segments) and, if they fit, the
// records the segments list.  Synchronises the stream.
pf_status pool_usage(pf::RecBuf& r, hipStream_t s, unsigned long long used[3], const char* who) {
  used[0] = used[1] = used[2] = 0;
  hipError_t e = hipMemcpyAsync(used, r.counter, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_status(e, who);
  if ((int64_t)used[0] <= r.cap && (int64_t)used[1] <= r.seg_cap) {
    const pf_status st = pf::seg_record_total(r.seg, (int64_t)used[1], r.counter + 2, s);
    if (st != PF_OK) return st;
    e = hipMemcpyAsync(used + 2, r.counter + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, who);
  }
  return PF_OK;
}

// Record and segment slots for a store-mode pass, from the scene's last
// raster (else any scene's), in coarse steps so that steps of similar size
// ask for the same block sizes; within `limit` bytes when one is set.
Caps store_caps(const pf_fwd_state* fs, int64_t need_rec, int64_t need_seg) {
  const pf::Scene& sc = fs->scene->s;
  const double npix = (double)fs->st.npix;
  const bool seen = sc.rec_per_pixel > 0.0;
  const double rpp = seen ? sc.rec_per_pixel : g_rec_hint.load();
  const double spp = seen ? sc.seg_per_pixel : g_seg_hint.load();
  auto coarse = [](int64_t x, int64_t step) { return (x + step - 1) / step * step; };
  Caps c;
  c.cap = coarse(std::max<int64_t>((int64_t)(rpp * npix), need_rec) + 4096, 1 << 22);
  c.seg_cap = coarse(std::max<int64_t>((int64_t)(spp * npix), need_seg) + 4096, 1 << 20);
  if (fs->kind == 1) c.seg_cap = std::max(c.seg_cap, c.cap);   // one segment per record on the walk
  // record and segment indices are stored as 32-bit integers
  c.cap = std::min<int64_t>(c.cap, INT32_MAX - 1);
  c.seg_cap = std::min<int64_t>(c.seg_cap, INT32_MAX - 1);
  if (fs->limit > 0 && pool_bytes(c) > fs->limit) c = caps_within(fs->limit, seg_ratio(sc, fs->kind));
  return c;
}

// Runs the state's pass with records (store mode).  A pass that runs out of
// room is repeated once with the exact sizes; when the records do not fit
// the state's workspace limit, the state becomes a recompute-mode state
// (*demoted = true; the image of the pass is complete either way).  rgba
// receives the image; trunc_dev (walk only) is zeroed before each attempt.
pf_status fill_records(pf_fwd_state* fs, float* rgba, unsigned long long* trunc_dev, hipStream_t s,
                       const char* who, bool* demoted, unsigned long long* counters = nullptr) {
  *demoted = false;
  pf_scene* scene = fs->scene;
  const int64_t npix = fs->st.npix;
  pf_status st = alloc_record_meta(fs->st.rec, npix, fs->kind == 0 ? fs->st.ntiles : 0, s, who);
  if (st != PF_OK) return st;
  Caps c = store_caps(fs, 0, 0);
  for (int attempt = 0; attempt < 2; ++attempt) {
    st = alloc_pool(fs->st.rec, c, s, who);
    if (st == PF_OK) st = reset_pool(fs->st.rec, fs->kind == 1, s, who);
    if (st == PF_OK && trunc_dev) {
      const hipError_t e = hipMemsetAsync(trunc_dev, 0, sizeof(unsigned long long), s);
      if (e != hipSuccess) st = hip_status(e, who);
    }
    if (st == PF_OK)
      st = run_pass(scene, fs->cams, fs->kind, fs->t_min, fs->max_steps, rgba, trunc_dev, s, &fs->st.rec, counters);
    unsigned long long used[3];
    if (st == PF_OK) st = pool_usage(fs->st.rec, s, used, who);
    if (st != PF_OK) return st;
    if (used[0] >= (unsigned long long)INT32_MAX || used[1] >= (unsigned long long)INT32_MAX) {
      if (fs->limit > 0) break;   // recompute in windows instead
      return invalid(std::string(who) + ": more than 2^31 - 2 contributions or segments in one call; render fewer "
                                        "views or set a workspace limit");
    }
    if (fs->kind == 0) {
      scene->s.rec_per_pixel = 1.05 * (double)used[0] / (double)npix;
      scene->s.seg_per_pixel = 1.05 * (double)used[1] / (double)npix;
      g_rec_hint.store(scene->s.rec_per_pixel);
      g_seg_hint.store(scene->s.seg_per_pixel);
    }
    if ((int64_t)used[0] <= c.cap && (int64_t)used[1] <= c.seg_cap) {
      fs->st.nrec = (int64_t)used[2];
      fs->st.nseg = (int64_t)used[1];
      return PF_OK;
    }
    free_pool(fs->st.rec, s);
    const Caps exact = store_caps(fs, (int64_t)used[0], (int64_t)used[1]);
    if (exact.cap < (int64_t)used[0] || exact.seg_cap < (int64_t)used[1]) break;   // over the limit
    c = exact;
  }
  if (fs->limit > 0) {
    // the records do not fit the limit: keep the cameras only and replay
    // the pass in windows inside pf_backward
    free_records(fs->st.rec, s);
    fs->mode = 1;
    fs->st.nrec = fs->st.nseg = 0;
    *demoted = true;
    return PF_OK;
  }
  pf::set_error(std::string(who) + ": record pool sizing failed");
  return PF_ERR_HIP;
}

// Record window of a recompute-mode backward: the state's workspace limit,
// else DEFAULT_WINDOW.
Caps window_caps(const pf_fwd_state* fs) {
  return caps_within(fs->limit > 0 ? fs->limit : DEFAULT_WINDOW, seg_ratio(fs->scene->s, fs->kind));
}

// Recompute-mode backward: the state's pass is replayed over windows of
// consecutive tiles whose records fit one bounded pool, and each window's
// records are differentiated and released before the next window is
// replayed.  A window whose records overflow the pool is split in two and
// replayed.  Peak memory: the binned lists of one group of views, the
// window's pool and the backward's workspace for it, one scratch image and
// the per-pixel heads.
pf_status backward_windows(pf_fwd_state* fs, const float* d_rgba, const pf_grads& g, const pf::BwdOpts& bo,
                           hipStream_t s) {
  const char* who = "pf_backward";
  pf::Scene& sc = fs->scene->s;
  const int64_t npix = fs->st.npix;
  const Caps c = window_caps(fs);
  // a window's tiles from the expected records per tile
  const double rpp = sc.rec_per_pixel > 0.0 ? sc.rec_per_pixel : g_rec_hint.load();
  const int64_t est_tiles = std::max<int64_t>(1, (int64_t)((double)c.cap / (1.25 * rpp * pf::TILE * pf::TILE)));
  const bool walk = fs->kind == 1;
  int64_t max_tiles = 0;   // tiles of the largest launch (wave segment tails)
  for (const pf_camera& cam : fs->cams) max_tiles = std::max(max_tiles, pf::view_tiles(cam));
  max_tiles = std::min<int64_t>(walk ? max_tiles : fs->st.ntiles, 4 * est_tiles);

  pf::BwdState w;
  w.npix = npix;
  w.ncam = fs->st.ncam;
  w.cams_dev = fs->st.cams_dev;
  float* scratch = nullptr;
  unsigned long long* trunc = nullptr;
  hipError_t e = pf::pool_alloc((void**)&scratch, sizeof(float) * 4 * npix, s);
  if (e == hipSuccess && walk) e = pf::pool_alloc((void**)&trunc, sizeof(unsigned long long), s);
  pf_status st = e == hipSuccess ? PF_OK : hip_status(e, who);
  if (st == PF_OK) st = alloc_record_meta(w.rec, npix, walk ? 0 : max_tiles, s, who);
  if (st == PF_OK) st = alloc_pool(w.rec, c, s, who);

  // one window [first, first + count) of a launch over a group's (or a
  // view's) tiles; global_first: its first tile among all views' tiles
  using Launch = std::function<pf_status(int64_t first, int64_t count)>;
  // windows are sized from the records per tile seen so far (first: the
  // scene's records per pixel); a window that overflows is halved
  double per_window = (double)std::min(max_tiles, est_tiles);
  auto windows = [&](int64_t ntiles, int64_t global_first, const Launch& launch) -> pf_status {
    int64_t first = 0;
    while (first < ntiles) {
      const int64_t count = std::min<int64_t>(ntiles - first, std::max<int64_t>(1, (int64_t)per_window));
      pf_status r = reset_pool(w.rec, walk, s, who);
      if (r == PF_OK) r = launch(first, count);
      unsigned long long used[3];
      if (r == PF_OK) r = pool_usage(w.rec, s, used, who);
      if (r != PF_OK) return r;
      if ((int64_t)used[0] > w.rec.cap || (int64_t)used[1] > w.rec.seg_cap) {
        if (count == 1) {
          pf::set_error(std::string(who) + ": the records of one 16x16 tile exceed the workspace limit");
          return PF_ERR_OOM;
        }
        per_window = (double)(count / 2);
        continue;
      }
      w.nrec = (int64_t)used[2];
      w.nseg = (int64_t)used[1];
      w.ntiles = count;
      w.tile0 = global_first + first;
      r = pf::backward_impl(sc, w, d_rgba, g, bo, s);
      if (r != PF_OK) return r;
      first += count;
      // the next window from this one's fill (slots of records and segments)
      const double fill = std::max((double)used[0] / (double)w.rec.cap, (double)used[1] / (double)w.rec.seg_cap);
      per_window = std::min((double)max_tiles, std::max(1.0, (double)count / std::max(fill, 1e-3) / 1.15));
    }
    return PF_OK;
  };

  if (st == PF_OK && !walk) {
    const pf::GroupFn fn = [&](int64_t tiles_before, int64_t ntiles, const pf::GroupComposite& run) {
      return windows(ntiles, tiles_before, [&](int64_t first, int64_t count) { return run(first, count, &w.rec); });
    };
    st = pf::raster_views(sc, fs->cams.data(), (int)fs->cams.size(), fs->t_min, scratch, s, nullptr, &fn);
  } else if (st == PF_OK) {
    int64_t pix = 0, tiles = 0;
    for (int v = 0; v < (int)fs->cams.size() && st == PF_OK; ++v) {
      const pf_camera& cam = fs->cams[v];
      const int64_t nt = pf::view_tiles(cam);
      st = windows(nt, tiles, [&](int64_t first, int64_t count) {
        return pf::trace_view(sc, cam, fs->t_min, fs->max_steps, scratch + 4 * pix, trunc, s, &w.rec, v, pix, first,
                              count);
      });
      pix += (int64_t)cam.width * cam.height;
      tiles += nt;
    }
  }
  if (st == PF_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_status(e, who);
  }
  free_records(w.rec, s);
  if (scratch) pf::pool_free(scratch, s);
  if (trunc) pf::pool_free(trunc, s);
  return st;
}

}  // namespace

pf_status pf_render_raster(pf_scene* scene, const pf_camera* cams, int32_t ncam, const pf_render_opts* opts,
                           float* rgba, pf_fwd_state** state, void* stream) {
  if (state) *state = nullptr;
  pf_status st = check_render(scene, cams, ncam, rgba, "pf_render_raster");
  if (st != PF_OK) return st;
  const float t_min = (opts && opts->t_min > 0) ? opts->t_min : 1e-6f;
  const int mode = opts ? opts->state_mode : 0;
  const int64_t limit = opts ? opts->workspace_limit : 0;
  if (mode != 0 && mode != 1) return invalid("pf_render_raster: state_mode must be 0 (store) or 1 (recompute)");
  if (limit < 0) return invalid("pf_render_raster: workspace_limit must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* counters = opts ? opts->counters : nullptr;
  if (!state || mode == 1) {
    st = pf::raster_views(scene->s, cams, ncam, t_min, rgba, s, nullptr, nullptr, counters);
    if (st != PF_OK || !state) return st;
    return new_state(scene, cams, ncam, 0, 1, t_min, 0, limit, s, state, "pf_render_raster");
  }
  pf_fwd_state* fs = nullptr;
  st = new_state(scene, cams, ncam, 0, 0, t_min, 0, limit, s, &fs, "pf_render_raster");
  if (st != PF_OK) return st;
  bool demoted = false;
  st = fill_records(fs, rgba, nullptr, s, "pf_render_raster", &demoted, counters);
  if (st != PF_OK) {
    free_state_mem(fs);
    delete fs;
    return st;
  }
  *state = fs;
  return PF_OK;
}

pf_status pf_render_trace(pf_scene* scene, const pf_camera* cams, int32_t ncam, const pf_render_opts* opts,
                          float* rgba, int64_t* truncated, pf_fwd_state** state, void* stream) {
  if (state) *state = nullptr;
  pf_status st = check_render(scene, cams, ncam, rgba, "pf_render_trace");
  if (st != PF_OK) return st;
  for (int c = 0; c < ncam; ++c) {
    const float* m = cams[c].c2w;
    const float o[3] = {m[3], m[7], m[11]};
    for (int a = 0; a < 3; ++a)
      if (!(o[a] >= scene->s.box_min[a] && o[a] <= scene->s.box_max[a]))
        return invalid("pf_render_trace: camera " + std::to_string(c) +
                       " centre lies outside the domain box; rebuild the scene with a box containing it");
  }
  const float t_min = (opts && opts->t_min > 0) ? opts->t_min : 1e-6f;
  const int max_steps = (opts && opts->max_steps > 0) ? opts->max_steps : 4096;
  const int mode = opts ? opts->state_mode : 0;
  const int64_t limit = opts ? opts->workspace_limit : 0;
  if (mode != 0 && mode != 1) return invalid("pf_render_trace: state_mode must be 0 (store) or 1 (recompute)");
  if (limit < 0) return invalid("pf_render_trace: workspace_limit must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* trunc = nullptr;
  PF_HIP_TRY(pf::pool_alloc((void**)&trunc, sizeof(unsigned long long), s));
  hipError_t e = hipMemsetAsync(trunc, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) {
    pf::pool_free(trunc, s);
    PF_HIP_TRY(e);
  }
  pf_fwd_state* fs = nullptr;
  const std::vector<pf_camera> cv(cams, cams + ncam);
  unsigned long long* counters = opts ? opts->counters : nullptr;
  if (!state || mode == 1) {
    st = run_pass(scene, cv, 1, t_min, max_steps, rgba, trunc, s, nullptr, counters);
    if (st == PF_OK && state)
      st = new_state(scene, cams, ncam, 1, 1, t_min, max_steps, limit, s, &fs, "pf_render_trace");
  } else {
    st = new_state(scene, cams, ncam, 1, 0, t_min, max_steps, limit, s, &fs, "pf_render_trace");
    bool demoted = false;
    if (st == PF_OK) st = fill_records(fs, rgba, trunc, s, "pf_render_trace", &demoted, counters);
  }
  if (st == PF_OK && truncated) {
    unsigned long long h = 0;
    e = hipMemcpyAsync(&h, trunc, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      pf::set_error(std::string("pf_render_trace: ") + hipGetErrorString(e));
      st = PF_ERR_HIP;
    } else {
      *truncated = (int64_t)h;
    }
  }
  pf::pool_free(trunc, s);
  if (st != PF_OK) {
    if (fs) {
      free_state_mem(fs);
      delete fs;
    }
    return st;
  }
  if (state) *state = fs;
  return PF_OK;
}

namespace {

// Scratch of pf_render_trace_noalloc: a device array in the library's code
// object, one copy per device, shared by every call on that device (calls
// that overlap on one device race on it).  Layout (bytes):
//   [0, 8192)        start-cell search, least power distance per block
//   [8192, 16384)    its cell per block
//   [16384, 16388)   the start cell
//   [16640, 16648)   rays cut by max_steps
constexpr size_t NOALLOC_PK = 0;
constexpr size_t NOALLOC_PI = NOALLOC_PK + sizeof(double) * pf::TRACE_START_BLOCKS;
constexpr size_t NOALLOC_START = NOALLOC_PI + sizeof(long long) * pf::TRACE_START_BLOCKS;
constexpr size_t NOALLOC_TRUNC = (NOALLOC_START + sizeof(int32_t) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_TRUNC + 256;
static_assert(NOALLOC_BYTES == PF_NOALLOC_SCRATCH_BYTES, "scratch layout and the documented size differ");

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};   // device address of scratch per device

// Device address of the current device's scratch (looked up once per device).
pf_status noalloc_scratch(unsigned char** out, const char* who) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    pf::set_error(std::string(who) + ": " + hipGetErrorString(e));
    return PF_ERR_HIP;
  }
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return invalid(std::string(who) + ": device index above 63");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      pf::set_error(std::string(who) + ": hipGetSymbolAddress of the scratch array failed: " +
                    hipGetErrorString(e));
      return PF_ERR_HIP;
    }
    g_noalloc_ptr[dev] = ptr;
  }
  *out = (unsigned char*)g_noalloc_ptr[dev];
  return PF_OK;
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

}  // namespace

pf_status pf_render_trace_noalloc(pf_scene* scene, const pf_camera* cams, int32_t ncam,
                                  const pf_render_opts* opts, float* rgba, int64_t* truncated, void* stream) {
  const char* who = "pf_render_trace_noalloc";
  pf_status st = check_render(scene, cams, ncam, rgba, who);
  if (st != PF_OK) return st;
  for (int c = 0; c < ncam; ++c) {
    const float* m = cams[c].c2w;
    const float o[3] = {m[3], m[7], m[11]};
    for (int a = 0; a < 3; ++a)
      if (!(o[a] >= scene->s.box_min[a] && o[a] <= scene->s.box_max[a]))
        return invalid(std::string(who) + ": camera " + std::to_string(c) +
                       " centre lies outside the domain box; rebuild the scene with a box containing it");
  }
  if (opts && opts->state_mode != 0) return invalid(std::string(who) + ": no forward state (state_mode must be 0)");
  // the start-cell search takes one partial per block of 256 cells, at most
  // TRACE_START_BLOCKS of them, so its scratch need never exceeds the array
  const int64_t nb = std::min<int64_t>(pf::TRACE_START_BLOCKS, (scene->s.n + 255) / 256);
  if ((size_t)nb * (sizeof(double) + sizeof(long long)) + sizeof(int32_t) > NOALLOC_TRUNC)
    return invalid(std::string(who) + ": start-cell search larger than the scratch array");
  const float t_min = (opts && opts->t_min > 0) ? opts->t_min : 1e-6f;
  const int max_steps = (opts && opts->max_steps > 0) ? opts->max_steps : 4096;
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = nullptr;
  st = noalloc_scratch(&base, who);
  if (st != PF_OK) return st;
  pf::TraceScratch ts;
  ts.pk = (double*)(base + NOALLOC_PK);
  ts.pi = (long long*)(base + NOALLOC_PI);
  ts.start = (int32_t*)(base + NOALLOC_START);
  unsigned long long* trunc = (unsigned long long*)(base + NOALLOC_TRUNC);
  // cleared by a kernel, not a memset node, so that the call can be captured
  k_zero_u64<<<1, 1, 0, s>>>(trunc);
  PF_HIP_TRY(hipGetLastError());
  int64_t off = 0;
  for (int c = 0; c < ncam; ++c) {
    st = pf::trace_view(scene->s, cams[c], t_min, max_steps, rgba + 4 * off, trunc, s, nullptr, c, off, 0, -1, &ts,
                        opts ? opts->counters : nullptr);
    if (st != PF_OK) return st;
    off += (int64_t)cams[c].width * cams[c].height;
  }
  if (truncated) {
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, trunc, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      pf::set_error(std::string(who) + ": " + hipGetErrorString(e));
      return PF_ERR_HIP;
    }
    *truncated = (int64_t)h;
  }
  return PF_OK;
}

pf_status pf_backward(pf_scene* scene, pf_fwd_state* state, const float* d_rgba, const pf_grads* grads,
                      const pf_backward_opts* opts, void* stream) {
  if (!scene || !state || !d_rgba || !grads) return invalid("pf_backward: NULL argument");
  if (state->scene != scene) return invalid("pf_backward: the state belongs to another scene");
  if (state->consumed)
    return invalid("pf_backward: this store-mode state was already used by pf_backward (its records are "
                   "overwritten); render again");
  pf::BwdOpts bo;
  if (opts) {
    if (!std::isfinite(opts->lambda_normal)) return invalid("pf_backward: lambda_normal must be finite");
    bo.lambda_normal = opts->lambda_normal;
    bo.contribution = opts->contribution;
    bo.normal_loss = opts->normal_loss;
    bo.pixel_error = opts->pixel_error;
    bo.error = opts->error;
  }
  hipStream_t s = (hipStream_t)stream;
  if (state->mode == 0) {
    state->consumed = true;
    return pf::backward_impl(scene->s, state->st, d_rgba, *grads, bo, s);
  }
  return backward_windows(state, d_rgba, *grads, bo, s);
}

pf_status pf_connect_loss(const pf_scene* scene, float lambda, const pf_grads* grads, double* loss, void* stream) {
  if (!scene || !grads) return invalid("pf_connect_loss: NULL argument");
  if (!std::isfinite(lambda)) return invalid("pf_connect_loss: lambda must be finite");
  return pf::connect_loss_impl(scene->s, lambda, *grads, loss, (hipStream_t)stream);
}

pf_status pf_steiner(const pf_params* params, const float* z, const pf_steiner_opts* opts, int64_t cap,
                     float* out_p, float* out_power, float* out_radius, int32_t* out_near, int64_t* round_counts,
                     int64_t* n_out, void* stream) {
  if (!params || !z || !opts || !n_out) return invalid("pf_steiner: NULL argument");
  const pf_params& p = *params;
  if (p.n < 1 || p.n >= (1ll << 30)) return invalid("pf_steiner: n must be in 1 .. 2^30 - 1");
  if (!p.p || !p.power || !p.radius) return invalid("pf_steiner: p, power and radius must not be NULL");
  const pf_steiner_opts& o = *opts;
  if (o.rounds < 1 || o.rounds > 64) return invalid("pf_steiner: rounds must be in 1 .. 64");
  if (o.n_cand < 1 || o.n_cand >= (1ll << 31)) return invalid("pf_steiner: n_cand must be in 1 .. 2^31 - 1");
  if (!std::isfinite(o.lo_ratio) || !std::isfinite(o.hi_ratio) || o.lo_ratio > o.hi_ratio)
    return invalid("pf_steiner: lo_ratio and hi_ratio must be finite, lo_ratio <= hi_ratio");
  if (cap < 0 || p.n + cap >= (1ll << 31)) return invalid("pf_steiner: cap must be >= 0 and n + cap < 2^31");
  if (cap > 0 && (!out_p || !out_power || !out_radius)) return invalid("pf_steiner: an output array is NULL");
  *n_out = 0;
  return pf::steiner_impl(p, z, o, cap, out_p, out_power, out_radius, out_near, round_counts, n_out,
                          (hipStream_t)stream);
}

pf_status pf_ema_update(float* ema, const float* value, int64_t n, float beta, void* stream) {
  if (!ema || !value || n < 0) return invalid("pf_ema_update: NULL argument or n < 0");
  if (!(beta >= 0.0f && beta <= 1.0f)) return invalid("pf_ema_update: beta must be in [0, 1]");
  if (n == 0) return PF_OK;
  return pf::ema_impl(ema, value, n, beta, (hipStream_t)stream);
}

pf_status pf_densify_prune(const pf_params* params, const float* err_ema, const float* contrib_ema, const float* u,
                           const float* delta, const pf_densify_opts* opts, const pf_cell_arrays* out, float* out_err,
                           float* out_contrib, int32_t* out_parent, int64_t* n_kept, int64_t* n_drawn,
                           void* stream) {
  if (!opts || !out || !err_ema || !contrib_ema || !out_err || !out_contrib || !n_kept || !n_drawn)
    return invalid("pf_densify_prune: NULL argument");
  {
    const pf_status st = check_params(params, "pf_densify_prune");
    if (st != PF_OK) return st;
  }
  const pf_cell_arrays& o = *out;
  if (!o.p || !o.power || !o.radius || !o.normal || !o.occ_logit || !o.rgb || !o.tex)
    return invalid("pf_densify_prune: an output array is NULL");
  if (opts->n_new < 0 || params->n + opts->n_new >= (1ll << 30))
    return invalid("pf_densify_prune: n_new must be >= 0 and n + n_new < 2^30");
  if (opts->n_new > 0 && (!u || !delta)) return invalid("pf_densify_prune: u and delta are needed for n_new > 0");
  if (!std::isfinite(opts->prune_below) || !std::isfinite(opts->spread))
    return invalid("pf_densify_prune: prune_below and spread must be finite");
  *n_kept = *n_drawn = 0;
  return pf::densify_impl(*params, err_ema, contrib_ema, u, delta, *opts, o, out_err, out_contrib, out_parent, n_kept,
                          n_drawn, (hipStream_t)stream);
}

pf_status pf_query_workspace(pf_scene* scene, const pf_camera* cams, int32_t ncam, int32_t what,
                             const pf_render_opts* opts, void* stream, int64_t* bytes) {
  if (!scene || !cams || ncam < 1 || !bytes) return invalid("pf_query_workspace: NULL argument or ncam < 1");
  if (what < 0 || what > 2) return invalid("pf_query_workspace: what must be 0, 1 or 2");
  for (int c = 0; c < ncam; ++c) {
    std::string why;
    if (!pf::camera_ok(cams[c], &why)) return invalid("pf_query_workspace: camera " + std::to_string(c) + ": " + why);
  }
  const int mode = opts ? opts->state_mode : 0;
  const int64_t limit = opts ? opts->workspace_limit : 0;
  if (mode != 0 && mode != 1) return invalid("pf_query_workspace: state_mode must be 0 or 1");
  if (limit < 0) return invalid("pf_query_workspace: workspace_limit must be >= 0");
  if (what > 0 && ncam > pf::REC_MAX_VIEWS) return invalid("pf_query_workspace: at most 4096 cameras with a state");
  const pf::Scene& sc = scene->s;
  const int64_t n = sc.n;
  int64_t group = 0;   // binned lists of the largest group of views
  {
    const pf_status st = pf::raster_workspace(scene->s, cams, ncam, (hipStream_t)stream, &group);
    if (st != PF_OK) return st;
  }
  if (what == 0) {
    *bytes = group;
    return PF_OK;
  }
  int64_t npix = 0, ntiles = 0;
  for (int c = 0; c < ncam; ++c) {
    npix += (int64_t)cams[c].width * cams[c].height;
    ntiles += pf::view_tiles(cams[c]);
  }
  const int64_t state = (int64_t)sizeof(pf_camera) * ncam;
  const int64_t meta = 4 * npix + 3 * 8 + 8 * 4 * ntiles;   // heads, counters, wave segment tails
  // recompute: the render keeps the cameras; the backward replays windows
  pf_fwd_state probe;
  probe.scene = scene;
  probe.kind = 0;
  probe.limit = limit;
  probe.st.npix = npix;
  const Caps wc = window_caps(&probe);
  const int64_t recompute_render = group + state;
  const int64_t recompute_bwd = state + 16 * npix + meta + pool_bytes(wc) + group + pf::backward_bytes(n, wc.cap, true);
  if (mode == 1) {
    *bytes = what == 1 ? recompute_render : std::max(recompute_render, recompute_bwd);
    return PF_OK;
  }
  // store: records for the whole call (within the limit, else demoted to
  // recompute, whose backward is then the bound)
  // (with a limit every pool the render asks for, the first one sized from
  // the hints or the exact one of a repeated pass, is within it)
  const Caps c = store_caps(&probe, 0, 0);
  const int64_t pool = limit > 0 ? limit : pool_bytes(c);
  const int64_t cap = limit > 0 ? limit / REC_BYTES : c.cap;
  const int64_t render = state + meta + pool + group;
  int64_t b = render;
  if (what == 2) {
    b = std::max(b, state + meta + pool + pf::backward_bytes(n, cap, true));
    if (limit > 0) b = std::max(b, recompute_bwd);
  }
  *bytes = b;
  return PF_OK;
}

pf_status pf_set_allocator(const pf_allocator* alloc) {
  if (alloc && (!alloc->alloc || !alloc->free)) return invalid("pf_set_allocator: alloc and free must both be set");
  pf::set_allocator(alloc);
  return PF_OK;
}

pf_status pf_set_cache_limit(int64_t bytes) {
  if (bytes < 0) return invalid("pf_set_cache_limit: bytes must be >= 0");
  pf::set_cache_limit((size_t)bytes);
  return PF_OK;
}

pf_status pf_memory_stats(int64_t* live, int64_t* peak, int64_t* cached, int32_t reset_peak) {
  pf::memory_stats(live, peak, cached, reset_peak != 0);
  return PF_OK;
}

void pf_state_release(pf_fwd_state* state) {
  if (!state) return;
  free_state_mem(state);
  delete state;
}

pf_status pf_state_info(const pf_fwd_state* state, int64_t* n_records, int64_t* n_pixels, int32_t* mode) {
  if (!state || !n_records || !n_pixels) return invalid("pf_state_info: NULL argument");
  *n_records = state->st.nrec;
  *n_pixels = state->st.npix;
  if (mode) *mode = state->mode;
  return PF_OK;
}

pf_status pf_profile_enable(int32_t on) {
  pf::g_prof_on.store(on != 0);
  return PF_OK;
}

pf_status pf_profile_read(pf_profile_entry* out, int32_t max_entries, int32_t* n_out) {
  if (!n_out || (max_entries > 0 && !out)) return invalid("pf_profile_read: NULL argument");
  std::vector<pf::ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(pf::g_prof_mu);
    recs.swap(pf::g_prof);
  }
  std::map<std::string, std::pair<int64_t, double>> acc;
  hipError_t first = hipSuccess;
  for (auto& r : recs) {
    hipError_t e = hipEventSynchronize(r.e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.e0, r.e1);
    if (e != hipSuccess && first == hipSuccess) first = e;
    auto& a = acc[r.name];
    a.first += 1;
    a.second += ms;
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  int32_t k = 0;
  for (auto& kv : acc) {
    if (k >= max_entries) break;
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
    out[k].launches = kv.second.first;
    out[k].total_ms = kv.second.second;
    ++k;
  }
  *n_out = k;
  PF_HIP_TRY(first);
  return PF_OK;
}

}  // extern "C"
