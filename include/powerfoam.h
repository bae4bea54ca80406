/*
 * powerfoam.h -- C ABI of the bounded-power-diagram renderer for gfx950.
 *
 * The library renders a scene of N cells.  Cell i is a site p_i with a power
 * weight w_i and a sphere radius r_i; the rendered cell is the power cell
 *   Pi_i = { x : |x-p_i|^2 - w_i <= |x-p_j|^2 - w_j  for all j }
 * intersected with the sphere B(p_i, r_i) (Sec. 3.2 of the paper, power cell
 * and bounded power diagram; appendix B, power distance).  Each cell is split
 * by an oriented dipole face through p_i with normal n_i; the side the normal
 * points away from is dense with density sigma_scale*softplus(lambda_i), the
 * other side is empty (Sec. 3.3).  The face carries K detail sites with a
 * soft-Voronoi displacement and Spherical-Voronoi radiance (Sec. 3.4,
 * Eq. svdisp and Eq. svrad; Sec. 3.6).  A pixel's colour is the exact
 * segment sum C = sum_k T_k alpha_k c_k over the cells its ray crosses, with
 * A = 1 - T_end and a black background (Sec. 3.1).
 *
 * The same image is produced two ways: tile rasterisation with cells taken
 * in increasing power distance from the camera centre, a valid painter's
 * order for every ray through that centre (appendix B, theorem), and a
 * cell-to-cell ray walk over the power-diagram adjacency clipped by the
 * spheres (Sec. 3.2, ray tracing; appendix C).
 *
 * Conventions
 *  - All array pointers are DEVICE pointers (gfx950 HBM) unless marked
 *    "(host)".  float arrays are IEEE binary32, C-contiguous, row-major.
 *  - Every call is stream-ordered on the caller's hipStream_t, passed as
 *    void* (NULL = the null stream).  Calls that must size buffers from
 *    device results synchronise that stream; this is stated per call.
 *  - Every call returns a pf_status.  On a non-OK status, pf_last_error()
 *    returns a thread-local message; outputs are unspecified and no handle
 *    is created.  The library never aborts or exits.
 *  - Parameters, images and gradients are caller-owned; the library keeps
 *    pointers to the parameter arrays inside a scene, so they must stay
 *    allocated and unchanged until pf_scene_destroy (re-build after changing
 *    them).  Library-owned memory (adjacency, per-view lists, forward state)
 *    is released by pf_scene_destroy / pf_state_release.
 *  - Device memory of the library comes from the caller's allocator when one
 *    is set (pf_set_allocator), e.g. the framework's caching allocator, so
 *    that one allocator owns all memory.  Without one, the library keeps
 *    released device blocks in a cache of its own and reuses them
 *    stream-ordered (a reuse waits for an event recorded where the block was
 *    released); blocks go back to the runtime when the cache passes its
 *    limit (48 GiB, pf_set_cache_limit) or a device allocation fails.
 *    pf_query_workspace bounds what a call will request.
 *  - Images: a call with ncam cameras writes ncam images back to back into
 *    rgba, image c at float offset 4*sum_{c'<c} W_c'*H_c', each [H][W][4]
 *    (R, G, B, A), pixel (x, y) at row y, column x, sampled at its centre.
 */
#ifndef POWERFOAM_H
#define POWERFOAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PF_OK = 0,
  PF_ERR_INVALID = 1,      /* bad argument: nothing was launched            */
  PF_ERR_OOM = 2,          /* device allocation failed; the scene is intact */
  PF_ERR_HIP = 3,          /* HIP runtime error (incl. earlier async faults) */
  PF_ERR_UNSUPPORTED = 4,  /* valid but not built (e.g. K, M other than 8)  */
  PF_ERR_OVERFLOW = 5      /* a fixed per-cell capacity was exceeded        */
} pf_status;

typedef struct pf_scene pf_scene;          /* opaque, library-owned */
typedef struct pf_fwd_state pf_fwd_state;  /* opaque, library-owned */

/* Cell parameters, structure of arrays (Sec. 3.2-3.4, 3.6).
   tex[i][k] = (s.x, s.y, d, a_0.xyz .. a_{M-1}.xyz, c_0.rgb .. c_{M-1}.rgb):
   detail-site position in the face frame, displacement along the normal,
   M Spherical-Voronoi axes and their colours. */
typedef struct {
  int64_t n;                 /* number of cells, >= 1                         */
  int32_t k_detail;          /* K detail sites per face (must be 8)           */
  int32_t m_axes;            /* M SV axes per detail site (must be 8)         */
  const float* p;            /* [n][3] sites                                  */
  const float* power;        /* [n]    power weights w_i                      */
  const float* radius;       /* [n]    sphere radii r_i (> 0)                 */
  const float* normal;       /* [n][3] dipole normals (normalised on use)     */
  const float* occ_logit;    /* [n]    density logits lambda_i                */
  const float* rgb;          /* [n][3] base colours                           */
  const float* tex;          /* [n][K][3+6M] detail-site texture              */
  float sigma_scale;         /* density per world unit at softplus = 1        */
  float tau;                 /* soft-Voronoi temperature per world unit       */
} pf_params;

/* A central camera.  c2w is row-major 3x4 camera-to-world (OpenCV axes: x
   right, y down, z forward); column 3 is the centre every ray starts from
   (t >= 0).  model 0 = pinhole (fx, fy, cx, cy in pixels); model 1 =
   equidistant fisheye: polar angle = image radius / f_fish, pixels with angle
   > theta_max render as 0. */
typedef struct {
  int32_t model;
  int32_t width, height;
  float c2w[12];
  float fx, fy, cx, cy;
  float f_fish, theta_max;
} pf_camera;

typedef struct {
  /* Domain box for the ray walk.  If box_min[0] > box_max[0], the box is the
     bounding box of all spheres grown by box_pad of its extent; otherwise the
     given box is grown to contain the spheres.  Trace cameras must lie
     inside it. */
  float box_min[3], box_max[3];
  float box_pad;             /* relative padding, default 0.01                */
} pf_build_opts;

typedef struct {
  float t_min;               /* stop a ray once T < t_min (default 1e-6)      */
  int32_t max_steps;         /* ray-walk step cap (default 4096)              */
  int32_t state_mode;        /* forward state: 0 store the contribution
                                records (default), 1 keep only the cameras and
                                replay the forward inside pf_backward         */
  int64_t workspace_limit;   /* bytes the contribution records may occupy at
                                once (0: no limit).  Store mode: a forward
                                whose records exceed it keeps only the cameras
                                (the state becomes a recompute-mode state).
                                Recompute mode: the backward's replay window
                                (0: 2 GiB).                                   */
  unsigned long long* counters; /* device, may be NULL: work counters of the
                                call's kernels, accumulated (+=) over every
                                composite / walk launch of the call (a store
                                pass repeated after the record pool was
                                resized counts twice).  Raster, 6 entries:
                                pixel-cell tests, sphere hits, contributions,
                                (wave, cell) steps that tested, that computed
                                a piece, that shaded.  Walk, 6 entries: rays,
                                cells walked, pieces computed (sphere hits),
                                contributions, exit faces scanned, the most
                                cells one ray walked (maximum).             */
} pf_render_opts;

/* Caller allocator.  alloc returns a device block of at least `bytes` bytes
   usable in stream order on `stream` (a hipStream_t), or NULL on failure;
   free takes back a block from alloc (with the size asked for), after all
   work the library queued on `stream` so far that uses it: an allocator
   that reuses blocks in stream order (as a caching allocator does per
   stream) may hand it out at once on that stream.  Both are called from the
   thread that makes the library call. */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, size_t bytes, void* stream);
  void* ctx;
} pf_allocator;

typedef struct {
  int64_t n;
  int64_t n_faces;           /* total directed faces in the adjacency         */
  int64_t n_hidden;          /* cells never rasterised: empty bounded cell or zero density */
  int64_t n_overflow;        /* cells whose build exceeded a capacity (0)     */
  int64_t n_high_degree;     /* cells that took the high-degree build pass    */
  int64_t n_dropped;         /* zero-density cells dropped for exceeding the
                                build's face capacity (see pf_build_scene)    */
  float box_min[3], box_max[3];
} pf_scene_info;

/* Gradient outputs, same shapes as pf_params; the library ADDS into them
   (the caller zeroes them).  Any pointer may be NULL to skip it. */
typedef struct {
  float *p, *power, *radius, *normal, *occ_logit, *rgb, *tex;
} pf_grads;

/* Builds the face adjacency of the power diagram clipped to the domain box
   (the regular-triangulation adjacency the walk needs, appendix C; the
   raster uses the subset of faces within each cell's sphere, Sec. 3.2),
   per-cell cull radii bounding the non-empty part of each bounded cell, and
   empty-cell flags.  params (host) is copied; its arrays are referenced.
   opts (host) may be NULL.  Synchronises the stream (sizes the adjacency).
   A cell of zero density (occ_logit = -inf, e.g. a Steiner cell) whose power
   cell exceeds the face capacity (256 planes) is dropped: the build is
   repeated as if it were absent (it can never contribute to an image; the
   walk does not enter it), at most three times; pf_scene_info reports the
   count.
   Errors: INVALID (n < 1, NULL array, K/M mismatch, non-positive radius),
   UNSUPPORTED (K or M != 8), OOM, HIP, OVERFLOW (a cell of non-zero density
   exceeded the face capacity; the scene is not created). */
pf_status pf_build_scene(const pf_params* params, const pf_build_opts* opts,
                         void* stream, pf_scene** out);

/* Rebuilds the adjacency, cull radii and flags of an existing scene for new
   parameter values (the sites moved during training), keeping the scene's
   build options and sizing hints.  The previous adjacency seeds the new one
   (a cell starts from its previous neighbours, or from the sites that
   emptied it), which makes small moves cheap; the result is the same as a
   fresh pf_build_scene (faces are written in a canonical order).  params
   (host) as for pf_build_scene; the scene then references the new arrays.
   Must not overlap a render or backward on the scene; the old arrays are
   freed stream-ordered on `stream`.  On error the scene keeps its previous
   state.  Errors: as pf_build_scene. */
pf_status pf_update_scene(pf_scene* scene, const pf_params* params, void* stream);

/* Scene statistics (host struct). */
pf_status pf_scene_info_get(const pf_scene* scene, pf_scene_info* info);

/* Copies the adjacency out: row [n+1] int32 (CSR offsets) and col
   [n_faces] int32 (neighbour index, or -1-f for face f of the domain box:
   0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z).  Device pointers, caller-owned. */
pf_status pf_scene_adjacency(const pf_scene* scene, int32_t* row, int32_t* col, void* stream);

void pf_scene_destroy(pf_scene* scene);

/* Tile rasteriser (Sec. 3.2, rasterization; appendix B order): per camera,
   cull each cell's bound into 16x16 tiles, sort each tile's cells by power
   distance from the camera centre (ties: lower index), composite front to
   back.  cams (host) [ncam]; opts (host) may be NULL; rgba as in the
   conventions.  If state is non-NULL (at most 4096 cameras), *state
   receives a forward state for pf_backward: with opts->state_mode 0 it
   stores the per-pixel contribution records (about 36 B per contribution),
   unless they exceed opts->workspace_limit; with 1 (or past the limit) only
   the cameras, and pf_backward replays the forward.  Synchronises the
   stream (pair list and record pool sizing).
   Errors: INVALID (ncam < 1, bad camera, state_mode not 0/1, negative
   workspace_limit, more than 4096 cameras with a state), OOM, HIP. */
pf_status pf_render_raster(pf_scene* scene, const pf_camera* cams, int32_t ncam,
                           const pf_render_opts* opts, float* rgba,
                           pf_fwd_state** state, void* stream);

/* Ray walk (Sec. 3.2, ray tracing; appendix C): per pixel, start in the
   cell of least power distance from the camera centre, cross faces of the
   power diagram until the ray leaves the domain box, clip each cell by its
   sphere.  Same image as pf_render_raster up to rounding.  Rays cut by
   max_steps are counted in *truncated (host, may be NULL; the count is read
   back, which synchronises the stream).  state as for pf_render_raster: the
   walk's contributions are recorded in the same form, so pf_backward gives
   the gradients of the walk.
   Errors: INVALID (also: camera centre outside the domain box), OOM, HIP. */
pf_status pf_render_trace(pf_scene* scene, const pf_camera* cams, int32_t ncam,
                          const pf_render_opts* opts, float* rgba,
                          int64_t* truncated, pf_fwd_state** state, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the plain
   ray walk of pf_render_trace (no forward state) with its scratch memory (the
   start-cell search and the truncation counter) in a fixed device array of
   PF_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, held
   until the process ends.  The call allocates nothing: no hipMalloc or
   hipFree, no allocator callback, no library cache; the caller passes the
   scene, the cameras and the image.  Every call on a device shares that
   device's array, so calls that overlap on one device (several streams,
   several threads) race and must be serialised by the caller; calls on one
   stream are ordered.  The start-cell search needs at most 16 KiB whatever
   the scene size, so no scene or camera count is beyond the array.
   Arguments as for pf_render_trace with state = NULL; opts->state_mode must
   be 0.  truncated (host, may be NULL) as for pf_render_trace: reading it
   back synchronises the stream, so pass NULL under capture.  Leave
   pf_profile_enable off: its event pairs are created per launch.
   Errors: INVALID (as pf_render_trace, also state_mode != 0), HIP. */
#define PF_NOALLOC_SCRATCH_BYTES 16896
pf_status pf_render_trace_noalloc(pf_scene* scene, const pf_camera* cams, int32_t ncam,
                                  const pf_render_opts* opts, float* rgba, int64_t* truncated,
                                  void* stream);

/* Options of pf_backward (host struct; all fields may be zero / NULL).
   The regularisers of the training objective (supplementary material, loss
   functions) that depend on the rendered rays:
     L_normal = sum over rays and cells of T a max(n_i . d, 0)^2,
   with T the transmittance in front of the cell, a its opacity on the ray,
   n_i its unit normal and d the unit ray direction, is added to L with the
   weight lambda_normal.  The sparsity loss summed over cells,
   sum over rays and cells of T a, equals the sum of the rendered opacity A
   over the rays, so its gradient is obtained by adding its weight to the A
   channel of d_rgba.  Statistics (device pointers, accumulated with +=):
   contribution [n] float, per cell sum over the rays of T a (the per-cell
   sparsity term and the quantity the pruning schedule tracks, Sec. 3.5);
   normal_loss [1] double, the value of L_normal over the rays;
   error [n] float, per cell sum over the rays of T a e, given the per-pixel
   photometric error pixel_error (device, one float per pixel in the image
   layout without the channel axis): the per-cell error that densification
   averages (Sec. 3.5).  Both must be given for the error statistic. */
typedef struct {
  float lambda_normal;
  float* contribution;
  double* normal_loss;
  const float* pixel_error;
  float* error;
} pf_backward_opts;

/* Gradients of L with respect to all cell parameters given dL/dRGBA
   (d_rgba, same layout as the forward's rgba), for the forward recorded in
   state (Sec. 3.1 sum differentiated through Sec. 3.2-3.6).  Adds into
   grads (host struct of device pointers).  opts (host) may be NULL.  A
   store-mode state is consumed (its records are overwritten): a second
   pf_backward on it fails with INVALID.  A recompute-mode state replays its
   forward in windows of consecutive 16x16 tiles: each window's records are
   written into one pool of at most the state's workspace_limit bytes (2 GiB
   without a limit), differentiated, and dropped before the next window is
   replayed, so the memory does not grow with the number of contributions
   (a window whose records do not fit is halved and replayed).  It
   synchronises the stream once per window and may be used again.  The
   gradients equal the store-mode ones up to the order of float atomic adds.
   Errors: INVALID (NULL argument, state/scene mismatch, consumed state,
   non-finite lambda_normal), OOM (also: one tile's records exceed the
   limit), HIP. */
pf_status pf_backward(pf_scene* scene, pf_fwd_state* state, const float* d_rgba,
                      const pf_grads* grads, const pf_backward_opts* opts, void* stream);

/* Frees a forward state, stream-ordered on the stream it was rendered on
   (which must still exist); work already queued there that uses it
   finishes first. */
void pf_state_release(pf_fwd_state* state);

/* Connectivity loss (supplementary material, loss functions) over the Cech
   graph of the scene's spheres as built (pairs i != j with
   |p_i - p_j| < r_i + r_j):
     lambda * sum_i sum_{j in Cech(i)} max(r_i + r_j - |p_i - p_j|, 0)^2.
   Adds its gradient into grads->p and grads->radius (the other fields are
   ignored; either may be NULL) and its value into *loss (device double, may
   be NULL).  Uses the positions and radii the scene was last built from.
   Synchronises the stream.
   Errors: INVALID (NULL scene/grads, non-finite lambda), OVERFLOW (a cell's
   tree traversal exceeded its stack), HIP. */
pf_status pf_connect_loss(const pf_scene* scene, float lambda, const pf_grads* grads, double* loss,
                          void* stream);

/* Steiner cells for the ray walk (supplementary material, Steiner points,
   Alg. 1).  In empty space the unbounded power cells that the walk crosses
   are unconstrained by rendering and can be long and thin; empty cells
   added there shorten the walk.  Runs `rounds` rounds over the sites of
   params (n, p, power, radius are read; device arrays):
     1. candidates x_j = mean + std * z[round][j] per axis, with the mean and
        population standard deviation of the current sites (the scene's and
        those kept in earlier rounds), rounded to float32;
     2. x_j is valid when |x_j - p_i|^2 - r_i^2 > 0 for every current site;
     3. near = argmin_i |x_j - p_i|^2 - r_i^2 (ties: lower index, scene
        sites first, then kept sites in the order kept);
        r_hat = |x_j - p_near| - r_near;
     4. x_j is kept when lo_ratio * r_near <= r_hat <= hi_ratio * r_near.
   All candidates of a round are tested against the sites present at its
   start; the kept ones join, in candidate order, at its end.  Outputs per
   kept cell k (device, capacity cap; rounds * n_cand always suffices):
   out_p [cap][3] site, out_radius [cap] float32(r_hat), out_power [cap]
   weight float32(r_hat^2 - r_near^2 + w_near) (its bisector with the nearest
   cell lies on that cell's sphere; r_hat^2 when w = r^2), out_near [cap]
   index of the nearest site in the combined order (may be NULL).
   round_counts (host, [rounds], may be NULL) receives the number kept per
   round and *n_out (host) the total.  The caller appends the cells to the
   scene as empty cells (occ_logit = -inf: zero density; such cells are
   walked but never rasterised).  z: device [rounds][n_cand][3] standard
   normal draws.  opts (host): rounds 6, lo_ratio 2, hi_ratio 6 in the
   paper.  Synchronises the stream once per round.
   Errors: INVALID (NULL or non-finite arguments, rounds outside 1..64,
   n_cand < 1, lo_ratio > hi_ratio), OVERFLOW (more than cap cells kept:
   *n_out = cap and the outputs hold the first cap), OOM, HIP. */
typedef struct {
  int64_t n_cand;       /* candidates per round */
  int32_t rounds;
  float lo_ratio, hi_ratio;
  int32_t reserved;     /* 0 */
} pf_steiner_opts;

pf_status pf_steiner(const pf_params* params, const float* z, const pf_steiner_opts* opts, int64_t cap,
                     float* out_p, float* out_power, float* out_radius, int32_t* out_near,
                     int64_t* round_counts, int64_t* n_out, void* stream);

/* Exponential moving average for the densify/prune schedule (Sec. 3.5):
   ema[i] = beta * ema[i] + (1 - beta) * value[i] for i < n (device arrays,
   formed in float64, rounded to float32).  Errors: INVALID (NULL, n < 0,
   beta outside [0, 1]), HIP. */
pf_status pf_ema_update(float* ema, const float* value, int64_t n, float beta, void* stream);

/* Densification and pruning (Sec. 3.5).  Cells whose contribution average
   contrib_ema[i] is below prune_below are removed; the kept cells keep
   their order.  Then n_new cells are drawn, with replacement, from the
   multinomial distribution proportional to the kept cells' error averages
   err_ema: draw k takes the first kept cell whose cumulative weight (float64,
   in kept order) exceeds u[k] * total, so cells of weight 0 are never drawn;
   the new cell is a copy of the drawn cell with its site moved to
   p + spread * r * delta[k].  No cell is drawn when no cell is kept or the
   total weight is 0.  Inputs (device): params arrays of n cells, err_ema
   and contrib_ema [n], u [n_new] uniforms in [0, 1), delta [n_new][3]
   standard normal draws.  Outputs (device, caller-allocated for n + n_new
   cells, same layouts as pf_params): out (host struct of the output
   arrays), out_err / out_contrib the averages of
   the output cells (new cells take their parent's), out_parent [n_new] the
   drawn cell's input index (may be NULL); *n_kept and *n_drawn (host) the
   numbers of kept and new cells (the output holds n_kept + n_drawn cells:
   the kept ones first).  Synchronises the stream.  The caller rebuilds the
   scene from the output arrays.
   Errors: INVALID (NULL argument, n_new < 0, non-finite prune_below or
   spread), HIP, OOM. */
typedef struct {
  int64_t n_new;
  float prune_below;
  float spread;
} pf_densify_opts;

typedef struct {
  float *p, *power, *radius, *normal, *occ_logit, *rgb, *tex;
} pf_cell_arrays;

pf_status pf_densify_prune(const pf_params* params, const float* err_ema, const float* contrib_ema,
                           const float* u, const float* delta, const pf_densify_opts* opts,
                           const pf_cell_arrays* out, float* out_err, float* out_contrib, int32_t* out_parent,
                           int64_t* n_kept, int64_t* n_drawn, void* stream);

/* Upper bound on the device bytes the library requests for a raster call
   sequence on `scene` with cameras cams (host) [ncam] and options opts
   (host, may be NULL): what 0, pf_render_raster without a state; what 1,
   pf_render_raster with a state in opts->state_mode; what 2, that state's
   pf_render_raster followed by pf_backward.  The bound counts the bytes the
   library asks its allocator for (the caller's allocator, or its cache,
   which rounds a block up by at most 1/16) that are in use at once during
   the calls, beyond the scene itself.  It is exact in the pair lists: the
   call runs the per-view cull-and-count pass of the rasteriser (one launch
   per group of views, its own temporary memory at most the bound of what 0)
   and synchronises the stream.  For a store-mode state without a
   workspace_limit the records are sized from the scene's last renders, so
   the value is an estimate, not a bound; with a limit, or in recompute mode,
   it is a bound.  Errors: INVALID (NULL argument, ncam < 1, bad camera,
   bad what or options), OOM, HIP. */
pf_status pf_query_workspace(pf_scene* scene, const pf_camera* cams, int32_t ncam, int32_t what,
                             const pf_render_opts* opts, void* stream, int64_t* bytes);

/* Sets the caller's allocator for all later device allocations of the
   library (process-wide; NULL restores the library's own cache).  Blocks
   already handed out go back to the allocator that gave them.  Setting an
   allocator returns the cache's free blocks to the runtime.
   Errors: INVALID (alloc or free missing). */
pf_status pf_set_allocator(const pf_allocator* alloc);

/* Limit of the library's own block cache in bytes (default 48 GiB; blocks
   past it go back to the runtime at once).  Errors: INVALID (bytes < 0). */
pf_status pf_set_cache_limit(int64_t bytes);

/* Requested bytes of the library's device blocks in use now (*live), their
   high-water mark since the last reset (*peak), and the bytes held free in
   the library's cache (*cached); any pointer may be NULL.  reset_peak != 0
   sets the high-water mark to the bytes in use. */
pf_status pf_memory_stats(int64_t* live, int64_t* peak, int64_t* cached, int32_t reset_peak);

/* Number of contribution records (pixel-cell pairs with alpha > 0) and of
   pixels in a forward state, and its mode (0 store, 1 recompute; may be
   NULL) (host outputs).  A recompute-mode state holds no records (0). */
pf_status pf_state_info(const pf_fwd_state* state, int64_t* n_records, int64_t* n_pixels, int32_t* mode);

/* Kernel timing for measurement.  While enabled (on != 0), every kernel the
   library launches is bracketed by HIP events on its stream; pf_profile_read
   waits for those events and returns, per kernel name, the launch count and
   the summed elapsed milliseconds since the last read, then clears them.
   Disabled by default; enabling costs two event records per launch.
   out (host) [max_entries]; *n_out receives the number of entries written. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} pf_profile_entry;

pf_status pf_profile_enable(int32_t on);
pf_status pf_profile_read(pf_profile_entry* out, int32_t max_entries, int32_t* n_out);

/* Thread-local message for the last non-OK status on this thread. */
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* POWERFOAM_H */
