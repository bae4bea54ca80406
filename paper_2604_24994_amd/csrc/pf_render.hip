// Rendering: tile rasteriser and ray walk over a built scene.
//
// Raster, per view (Sec. 3.2, rasterization; appendix B order):
//   k_view_count  per cell: power distance from the camera centre (the sort
//                 key) and the tile rectangle of its cull ball
//   scan          cell offsets into the pair list
//   k_view_emit   (tile, key<<32 | cell) pairs + tile histogram
//   scan/scatter  counting sort by tile
//   k_tile_sort   per tile, sort by (key, cell) in LDS (bitonic, global
//                 memory fallback for long lists)
//   k_raster      one 256-thread workgroup per 16x16 tile, one lane per
//                 pixel, each wave an 8x8 quadrant walking the tile's list
//                 front to back; the list and the cells' records are staged
//                 in LDS 256 entries at a time by the whole workgroup, so a
//                 cell that misses the quadrant costs no memory latency
// Trace, per view (Sec. 3.2, ray tracing; appendix C):
//   k_start_*     argmin power distance from the camera centre
//   k_trace       one lane per ray; per step the piece of the current cell
//                 (same device code as the rasteriser) and the exit face
#include "pf_internal.hpp"
#include "pf_render.hpp"
#include "pf_shade.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace pf {
namespace {

__device__ inline uint32_t order_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Tile rectangle of a ball (camera-space centre X,Y,Z, radius rho).
__device__ bool ball_rect(const pf_camera& c, double X, double Y, double Z, double rho, int tiles_x, int tiles_y,
                          int& x0, int& x1, int& y0, int& y1) {
  const double W = c.width, H = c.height;
  double ulo, uhi, vlo, vhi;
  bool full = false;
  if (c.model == 0) {
    if (Z + rho <= 0.0) return false;
    if (Z - rho <= 1e-9 * (1.0 + fabs(Z))) {
      full = true;
    } else {
      const double zz = Z * Z - rho * rho;
      const double sx = rho * sqrt(fmax(0.0, X * X + zz));
      const double sy = rho * sqrt(fmax(0.0, Y * Y + zz));
      const double kxl = (X * Z - sx) / zz, kxh = (X * Z + sx) / zz;
      const double kyl = (Y * Z - sy) / zz, kyh = (Y * Z + sy) / zz;
      ulo = (double)c.fx * kxl + (double)c.cx;
      uhi = (double)c.fx * kxh + (double)c.cx;
      vlo = (double)c.fy * kyl + (double)c.cy;
      vhi = (double)c.fy * kyh + (double)c.cy;
    }
  } else {
    const double Lc = sqrt(X * X + Y * Y + Z * Z);
    if (Lc <= rho * (1.0 + 1e-9)) {
      full = true;
    } else {
      const double beta = asin(fmin(1.0, rho / Lc));
      const double thc = acos(fmax(-1.0, fmin(1.0, Z / Lc)));
      const double tmax = (double)c.theta_max;
      if (thc - beta > tmax) return false;
      const double f = (double)c.f_fish;
      const double thi = fmin(tmax, thc + beta);
      const double rhi = f * thi;
      if (thc <= beta || thc + beta >= M_PI) {
        ulo = c.cx - rhi; uhi = c.cx + rhi;
        vlo = c.cy - rhi; vhi = c.cy + rhi;
      } else {
        const double tlo = fmax(0.0, thc - beta);
        const double rlo = f * tlo;
        const double phc = atan2(Y, X);
        const double dph = asin(fmin(1.0, sin(beta) / sin(thc)));
        const double pa = phc - dph, pb = phc + dph;
        ulo = vlo = INFINITY;
        uhi = vhi = -INFINITY;
        const double ph[2] = {pa, pb}, rr[2] = {rlo, rhi};
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            const double u = c.cx + rr[j] * cos(ph[i]), v = c.cy + rr[j] * sin(ph[i]);
            ulo = fmin(ulo, u); uhi = fmax(uhi, u);
            vlo = fmin(vlo, v); vhi = fmax(vhi, v);
          }
        // axis-aligned extremes of the outer arc inside [pa, pb]
        for (int q = -4; q <= 4; ++q) {
          const double a = q * (M_PI / 2);
          if (a > pa && a < pb) {
            const double u = c.cx + rhi * cos(a), v = c.cy + rhi * sin(a);
            ulo = fmin(ulo, u); uhi = fmax(uhi, u);
            vlo = fmin(vlo, v); vhi = fmax(vhi, v);
          }
        }
      }
    }
  }
  if (full) {
    x0 = 0; x1 = tiles_x - 1;
    y0 = 0; y1 = tiles_y - 1;
    return true;
  }
  // pixels whose centre (p + 1/2) may lie in [lo, hi], padded by one pixel
  const double pxl = ceil(ulo - 0.5) - 1.0, pxh = floor(uhi - 0.5) + 1.0;
  const double pyl = ceil(vlo - 0.5) - 1.0, pyh = floor(vhi - 0.5) + 1.0;
  if (!(pxh >= 0.0 && pyh >= 0.0 && pxl <= W - 1 && pyl <= H - 1)) return false;
  x0 = (int)fmax(0.0, floor(fmax(pxl, 0.0) / TILE));
  x1 = (int)fmin((double)(tiles_x - 1), floor(fmin(pxh, W - 1) / TILE));
  y0 = (int)fmax(0.0, floor(fmax(pyl, 0.0) / TILE));
  y1 = (int)fmin((double)(tiles_y - 1), floor(fmin(pyh, H - 1) / TILE));
  return x0 <= x1 && y0 <= y1;
}

struct ViewArgs {
  pf_camera cam;
  int tiles_x, tiles_y;
};

// One camera of a batched raster call: its tiles are numbered from
// tile_base and its pixels from pix_base across the whole batch.
struct ViewDev {
  ViewArgs v;
  long long tile_base;
  long long pix_base;
  int view_id;   // camera index within the call
};

// A ball that crosses the plane of a pinhole camera (camera outside the
// ball) has no bounded screen rectangle; the pixel rays that meet it are
// those within the cone of half-angle asin(rho/|c|) around the direction c
// to its centre.  A tile is kept when the angle between its centre ray and
// c is at most that half-angle plus the tile's own angular radius.
struct Cone {
  double ax, ay, az;   // unit direction to the centre, camera axes
  double cmin;         // cosine of the widened half-angle
};

__device__ inline bool cone_tile(const pf_camera& c, const Cone& k, int tx, int ty) {
  const double dx = ((double)(tx * TILE) + 0.5 * TILE - (double)c.cx) / (double)c.fx;
  const double dy = ((double)(ty * TILE) + 0.5 * TILE - (double)c.cy) / (double)c.fy;
  const double dot = dx * k.ax + dy * k.ay + k.az;
  // dot / |d| >= cmin, without the square root
  if (k.cmin <= 0.0 && dot >= 0.0) return true;
  const double d2 = dx * dx + dy * dy + 1.0;
  return k.cmin >= 0.0 ? (dot >= 0.0 && dot * dot >= k.cmin * k.cmin * d2) : (dot * dot <= k.cmin * k.cmin * d2);
}

// Tile footprint of a cell's cull ball in a view: 0 none, 1 the rectangle
// [x0, x1] x [y0, y1], 2 the tiles of that rectangle (all of the view)
// accepted by cone_tile(k).
__device__ inline int cell_rect(const ViewArgs& v, const float4 g, float rho, int& x0, int& x1, int& y0, int& y1,
                                Cone& k) {
  if (!(rho >= 0.0f)) return 0;
  const float* m = v.cam.c2w;
  const double ex = (double)g.x - m[3], ey = (double)g.y - m[7], ez = (double)g.z - m[11];
  const double X = m[0] * ex + m[4] * ey + m[8] * ez;
  const double Y = m[1] * ex + m[5] * ey + m[9] * ez;
  const double Z = m[2] * ex + m[6] * ey + m[10] * ez;
  const double r = (double)rho * (1.0 + 1e-5) + 1e-7;
  if (!ball_rect(v.cam, X, Y, Z, r, v.tiles_x, v.tiles_y, x0, x1, y0, y1)) return 0;
  if (v.cam.model == 0 && Z - r <= 1e-9 * (1.0 + fabs(Z))) {
    const double L = sqrt(X * X + Y * Y + Z * Z);
    if (L > r * (1.0 + 1e-9)) {
      // tile angular radius: half diagonal of a tile plus the one-pixel pad
      const double tile_ang = (0.5 * TILE + 1.0) * 1.4142135623730951 / fmin((double)v.cam.fx, (double)v.cam.fy);
      const double ang = asin(r / L) + tile_ang + 1e-6;
      k.ax = X / L;
      k.ay = Y / L;
      k.az = Z / L;
      k.cmin = ang >= M_PI ? -1.0 : cos(ang);
      return 2;
    }
  }
  return 1;
}

// blockIdx.y = view; one thread per (view, cell).
// Cells whose footprint needs the per-tile cone test are listed in
// cone_list (as view * n + cell) and counted by k_cone_count.
__global__ void k_view_count(const ViewDev* __restrict__ views, const float4* __restrict__ geo,
                             const float* __restrict__ cull, const float* __restrict__ power, int64_t n,
                             uint32_t* __restrict__ cnt, uint32_t* __restrict__ key, uint32_t* __restrict__ cone_list,
                             uint32_t* __restrict__ cone_n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ViewArgs& v = views[blockIdx.y].v;
  const int64_t o = (int64_t)blockIdx.y * n + i;
  const float4 g = geo[i];
  int x0, x1, y0, y1;
  Cone k;
  uint32_t c = 0;
  const int mode = cell_rect(v, g, cull[i], x0, x1, y0, y1, k);
  if (mode == 1) {
    c = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
  } else if (mode == 2) {
    cone_list[atomicAdd(cone_n, 1u)] = (uint32_t)o;
  }
  cnt[o] = c;
  const float* m = v.cam.c2w;
  const double ex = (double)m[3] - g.x, ey = (double)m[7] - g.y, ez = (double)m[11] - g.z;
  key[o] = order_key((float)(ex * ex + ey * ey + ez * ez - (double)power[i]));
}

// blockIdx.y = view; a lane per (view, cell).  A wave emits its cells'
// pixel rectangles together: after a scan of the pair counts over the wave,
// it writes 64 pairs at a time, pair p taken by the lane whose run holds p,
// so that a cell whose footprint covers many tiles is spread over the wave
// rather than holding it, and the stores of a step are contiguous.  A
// cell's pairs keep the order of its rectangle (rows of tiles, then tiles).
__global__ void __launch_bounds__(256) k_view_emit(const ViewDev* __restrict__ views, const float4* __restrict__ geo,
                                                   const float* __restrict__ cull, int64_t n,
                                                   const uint32_t* __restrict__ off, const uint32_t* __restrict__ key,
                                                   uint32_t* __restrict__ ptile, unsigned long long* __restrict__ pval,
                                                   uint32_t* __restrict__ tile_cnt) {
  __shared__ int s_end[4][64];   // end of each lane's run of the wave's pairs
  __shared__ int s_x0[4][64], s_y0[4][64], s_w[4][64];
  __shared__ uint32_t s_o[4][64];
  __shared__ unsigned long long s_val[4][64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const ViewDev& vd = views[blockIdx.y];
  int nt = 0, x0 = 0, x1 = -1, y0 = 0, y1 = -1;
  uint32_t o = 0;
  unsigned long long val = 0;
  if (i < n) {
    const int64_t oi = (int64_t)blockIdx.y * n + i;
    Cone k;
    const int mode = cell_rect(vd.v, geo[i], cull[i], x0, x1, y0, y1, k);
    if (mode == 1) {   // (cone footprints: k_cone_emit)
      nt = (x1 - x0 + 1) * (y1 - y0 + 1);
      o = off[oi];
      val = ((unsigned long long)key[oi] << 32) | (uint32_t)i;
    }
  }
  int end = nt;
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(end, d, 64);
    if (lane >= d) end += t;
  }
  const int total = __shfl(end, 63, 64);
  s_end[wv][lane] = end;
  s_x0[wv][lane] = x0;
  s_y0[wv][lane] = y0;
  s_w[wv][lane] = x1 - x0 + 1;
  s_o[wv][lane] = o;
  s_val[wv][lane] = val;
  __syncthreads();
  const uint32_t tbase = (uint32_t)vd.tile_base;
  const int tiles_x = vd.v.tiles_x;
  for (int base = 0; base < total; base += 64) {
    const int p = base + lane;
    if (p >= total) break;
    // owner: the first lane whose run ends after p
    int lo = 0, hi = 63;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_end[wv][mid] > p) hi = mid;
      else lo = mid + 1;
    }
    const int r = p - (lo == 0 ? 0 : s_end[wv][lo - 1]);
    const int w = s_w[wv][lo];
    const int ty = s_y0[wv][lo] + r / w, tx = s_x0[wv][lo] + r % w;
    const uint32_t t = tbase + (uint32_t)(ty * tiles_x + tx);
    const uint32_t at = s_o[wv][lo] + (uint32_t)r;
    ptile[at] = t;
    pval[at] = s_val[wv][lo];
    atomicAdd(&tile_cnt[t], 1u);
  }
}

// One workgroup per listed (view, cell): its threads test the tiles of the
// view in parallel.
__global__ void __launch_bounds__(256) k_cone_count(const ViewDev* __restrict__ views,
                                                    const float4* __restrict__ geo, const float* __restrict__ cull,
                                                    int64_t n, const uint32_t* __restrict__ cone_list,
                                                    uint32_t* __restrict__ cnt) {
  __shared__ uint32_t part[4];
  const uint32_t o = cone_list[blockIdx.x];
  const int64_t i = (int64_t)(o % (uint64_t)n);
  const ViewArgs& v = views[o / (uint64_t)n].v;
  int x0, x1, y0, y1;
  Cone k;
  (void)cell_rect(v, geo[i], cull[i], x0, x1, y0, y1, k);
  const int tw = x1 - x0 + 1, nt = tw * (y1 - y0 + 1);
  uint32_t c = 0;
  for (int t = threadIdx.x; t < nt; t += 256) c += cone_tile(v.cam, k, x0 + t % tw, y0 + t / tw) ? 1u : 0u;
  for (int sh = 32; sh > 0; sh >>= 1) c += __shfl_xor(c, sh, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[o] = part[0] + part[1] + part[2] + part[3];
}

__global__ void __launch_bounds__(256) k_cone_emit(const ViewDev* __restrict__ views, const float4* __restrict__ geo,
                                                   const float* __restrict__ cull, int64_t n,
                                                   const uint32_t* __restrict__ off, const uint32_t* __restrict__ key,
                                                   const uint32_t* __restrict__ cone_list,
                                                   uint32_t* __restrict__ ptile, unsigned long long* __restrict__ pval,
                                                   uint32_t* __restrict__ tile_cnt) {
  __shared__ uint32_t wsum[4];
  const uint32_t o = cone_list[blockIdx.x];
  const int64_t i = (int64_t)(o % (uint64_t)n);
  const ViewDev& vd = views[o / (uint64_t)n];
  int x0, x1, y0, y1;
  Cone k;
  (void)cell_rect(vd.v, geo[i], cull[i], x0, x1, y0, y1, k);
  const int tw = x1 - x0 + 1, nt = tw * (y1 - y0 + 1);
  const unsigned long long val = ((unsigned long long)key[o] << 32) | (uint32_t)i;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t base = off[o];
  for (int t0 = 0; t0 < nt; t0 += 256) {
    const int t = t0 + threadIdx.x;
    const int tx = x0 + t % tw, ty = y0 + t / tw;
    const bool pass = t < nt && cone_tile(vd.v.cam, k, tx, ty);
    const uint64_t m = __ballot(pass);
    if (lane == 0) wsum[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
      before += w < wv ? wsum[w] : 0u;
      total += wsum[w];
    }
    if (pass) {
      const uint32_t pos = base + before + (uint32_t)__popcll(m & lt);
      const uint32_t tile = (uint32_t)(vd.tile_base + ty * vd.v.tiles_x + tx);
      ptile[pos] = tile;
      pval[pos] = val;
      atomicAdd(&tile_cnt[tile], 1u);
    }
    base += total;
    __syncthreads();
  }
}

__global__ void k_tile_scatter(const uint32_t* __restrict__ ptile, const unsigned long long* __restrict__ pval,
                               int64_t np, const uint32_t* __restrict__ tile_off, uint32_t* __restrict__ fill,
                               unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const uint32_t t = ptile[i];
  const uint32_t pos = tile_off[t] + atomicAdd(&fill[t], 1u);
  out[pos] = pval[i];
}

constexpr int SORT_THREADS = 256;
constexpr int SORT_LDS = 4096;

// Ascending sort of one tile's segment.  Bitonic network in its "flip"
// form (every comparator puts the smaller value at the lower index), so a
// length that is not a power of two is sorted with the missing tail treated
// as +infinity and never touched.
__global__ void __launch_bounds__(SORT_THREADS) k_tile_sort(unsigned long long* __restrict__ vals,
                                                            const uint32_t* __restrict__ tile_off) {
  __shared__ unsigned long long sh[SORT_LDS];
  const uint32_t a = tile_off[blockIdx.x], b = tile_off[blockIdx.x + 1];
  const uint32_t n = b - a;
  if (n <= 1) return;
  uint32_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  const bool lds = n2 <= SORT_LDS;
  unsigned long long* buf = lds ? sh : vals + a;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) sh[i] = vals[a + i];
    __syncthreads();
  }
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = threadIdx.x; t < n2 / 2; t += SORT_THREADS) {
        // t-th comparator of this stage: lower index i has bit j clear
        const uint32_t i = ((t / j) * 2 * j) + (t % j);
        const uint32_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i + j);
        if (p < n) {
          const unsigned long long x = buf[i], y = buf[p];
          if (y < x) {
            buf[i] = y;
            buf[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  if (lds)
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) vals[a + i] = sh[i];
}

struct SceneDev {
  const float4* geo;
  const float4* nrm;
  const float* cull;
  const int32_t* row;
  const int32_t* nrast;
  const int32_t* col;
  const float4* plane;
  const float* rgb;
  const float* tex;
  float tau;
};

constexpr int RB = 256;     // tile-list entries staged in LDS per batch
constexpr int RBLK = 256;   // record slots reserved per wave at a time
constexpr int SBLK = SEG_BLOCK;   // segment slots reserved per wave at a time

__device__ inline unsigned long long bcast64(unsigned long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ inline void tile_pixel(int tiles_x, int& px, int& py, int tile = -1) {
  if (tile < 0) tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  px = tx * TILE + (w & 1) * 8 + (lane & 7);
  py = ty * TILE + (w >> 1) * 8 + (lane >> 3);
}

// COUNT: the work counters of the composite are added to counters[0..5]
// (RASTER_COUNTERS): pixel-cell tests, sphere hits, contributions, and the
// (wave, cell) steps that tested, that computed a piece, that shaded.
// Seven waves per SIMD (at most 72 VGPRs) are asked for explicitly: the
// compiler's own choice lands a few registers above, at six.
template <bool STORE, bool COUNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7)))
k_raster(const ViewDev* __restrict__ views, int nview, SceneDev S, const unsigned long long* __restrict__ list,
         const uint32_t* __restrict__ tile_off, float t_min, float* __restrict__ rgba_all, int4* __restrict__ rec_ri,
         float4* __restrict__ rec_rf, float* __restrict__ rec_rt, int32_t* __restrict__ rec_head,
         unsigned long long* __restrict__ rec_counter, int4* __restrict__ rec_seg, int2* __restrict__ rec_wtail,
         int64_t tile_first, int64_t wtail_base, int64_t rec_cap, int64_t seg_cap,
         unsigned long long* __restrict__ counters) {
  // the tile's sorted cells are staged RB at a time: list entry and the cell
  // record fields every lane needs, loaded by the whole workgroup at once
  __shared__ int s_ci[RB];
  __shared__ float4 s_geo[RB];
  __shared__ float4 s_nrm[RB];
  __shared__ float s_rho[RB];
  __shared__ int s_row[RB];
  __shared__ int s_nr[RB];
  __shared__ int s_more[4];

  // one workgroup per work item (a tile of one of the launch's views); the
  // hardware dispatcher hands the next item to whichever CU frees up, so the
  // tiles of all views of a call (the requests of a serving batch) share
  // the CUs.  (A persistent loop over items held twice the registers and
  // halved the occupancy.)
  const int64_t item = blockIdx.x;
  // tile of the view group; its view: the last one whose tiles start at or before it
  const int64_t gtile = tile_first + item;
  int lo = 0, hi = nview - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= (long long)gtile) lo = mid; else hi = mid - 1;
  }
  const ViewDev& vd = views[lo];
  const int view = vd.view_id;
  const ViewArgs& v = vd.v;
  const int64_t pix_base = vd.pix_base;
  float* rgba = rgba_all + 4 * pix_base;
  int px, py;
  tile_pixel(v.tiles_x, px, py, (int)(gtile - vd.tile_base));
  const bool inside = px < v.cam.width && py < v.cam.height;
  const RayD R = make_ray(v.cam, px + 0.5, py + 0.5);
  bool live = inside && R.valid;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  int head = -1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int pix = py * v.cam.width + px;
  const uint32_t e0 = tile_off[gtile], e1 = tile_off[gtile + 1];
  long long rblk = 0, sblk = 0;   // the wave's current record / segment block
  long long cblk = -1;            // first slot (header) of the wave's current segment block
  int rleft = 0, sleft = 0;
  unsigned long long n_test = 0, n_hit = 0, n_contrib = 0, n_step = 0, n_step_hit = 0, n_step_shade = 0;
  for (uint32_t b0 = e0; b0 < e1; b0 += RB) {
    {
      const uint32_t e = b0 + threadIdx.x;
      if (e < e1) {
        const int c = (int)(uint32_t)list[e];
        s_ci[threadIdx.x] = c;
        s_geo[threadIdx.x] = S.geo[c];
        s_nrm[threadIdx.x] = S.nrm[c];
        s_rho[threadIdx.x] = S.cull[c];
        s_row[threadIdx.x] = S.row[c];
        s_nr[threadIdx.x] = S.nrast[c];
      }
    }
    __syncthreads();
    const int nb = (int)min((uint32_t)RB, e1 - b0);
    for (int q = 0; q < nb; ++q) {
      if (!__any(live)) break;
      const int ci = __builtin_amdgcn_readfirstlane(s_ci[q]);
      const float4 g = s_geo[q];
      const float rho = s_rho[q];
      const Local L = make_local(R, g.x, g.y, g.z);
      const bool hit = live && (rho >= 0.0f) && (L.qq < (double)rho * (double)rho);
      if constexpr (COUNT) {
        n_test += (unsigned long long)__popcll(__ballot(live));
        n_hit += (unsigned long long)__popcll(__ballot(hit));
        ++n_step;
      }
      if (!__any(hit)) continue;
      if constexpr (COUNT) ++n_step_hit;
      const float* tx = S.tex + (int64_t)ci * (KD * TEXW);
      Piece P;
      P.alpha = 0.0f;
      float r = 0.0f, gg = 0.0f, b = 0.0f;
      if (hit) {
        P = piece_geometry<true>(R, L, g.w, S.plane + __builtin_amdgcn_readfirstlane(s_row[q]),
                           __builtin_amdgcn_readfirstlane(s_nr[q]), s_nrm[q], tx, S.tau);
        if (P.alpha > 0.0f) radiance<true>(tx, S.rgb + 3 * (int64_t)ci, P.ux, P.uy, R.fx, R.fy, R.fz, S.tau, r, gg, b);
      }
      const bool contrib = hit && P.alpha > 0.0f;
      if constexpr (COUNT) {
        const uint64_t mc = __ballot(contrib);
        n_contrib += (unsigned long long)__popcll(mc);
        n_step_shade += mc ? 1ull : 0ull;
      }
      if constexpr (STORE) {
        const uint64_t m = __ballot(contrib);
        if (m) {
          // slots come from the wave's own blocks; a new block is reserved
          // with one global atomic when the current one cannot take the append
          const int cnt = __popcll(m);
          if (cnt > rleft) {
            unsigned long long bk = 0;
            if (lane == 0) bk = atomicAdd(&rec_counter[0], (unsigned long long)RBLK);
            rblk = (long long)bcast64(bk);
            rleft = RBLK;
          }
          if (sleft == 0) {
            unsigned long long bk = 0;
            if (lane == 0) bk = atomicAdd(&rec_counter[1], (unsigned long long)SBLK);
            const long long nb = (long long)bcast64(bk);
            // the block's header links it to the wave's previous block
            if (lane == 0 && nb < seg_cap) rec_seg[nb] = make_int4(-1, (int)cblk, 0, 0);
            cblk = nb;
            sblk = nb + 1;
            sleft = SBLK - 1;
          }
          const long long base = rblk, sg = sblk;
          rblk += cnt;
          rleft -= cnt;
          sblk += 1;
          sleft -= 1;
          if (lane == 0 && sg < seg_cap && base + cnt <= rec_cap)
            rec_seg[sg] = make_int4(ci, (int)base, (int)(uint32_t)m, (int)(uint32_t)(m >> 32));
          if (contrib) {
            const long long slot = base + __popcll(m & lt);
            if (slot < rec_cap) {
              rec_ri[slot] = make_int4(ci, pix, head, pack_view_bind(view, P.bind0, P.bind1));
              rec_rf[slot] = make_float4(P.alpha, r, gg, b);
              rec_rt[slot] = T;
              head = (int)slot;
            }
          }
        }
      }
      if (contrib) {
        const float wgt = T * P.alpha;
        cr += wgt * r;
        cg += wgt * gg;
        cb += wgt * b;
        T *= (1.0f - P.alpha);
      }
      live = live && (T >= t_min);
    }
    const bool wl = __any(live);
    if (lane == 0) s_more[wave] = wl ? 1 : 0;
    __syncthreads();
    const bool more = (s_more[0] | s_more[1] | s_more[2] | s_more[3]) != 0;
    __syncthreads();
    if (!more) break;
  }
  if (inside) {
    float* o = rgba + 4 * ((int64_t)py * v.cam.width + px);
    o[0] = cr;
    o[1] = cg;
    o[2] = cb;
    o[3] = 1.0f - T;
    if constexpr (STORE) rec_head[pix_base + pix] = head;
  }
  if constexpr (STORE) {
    // unused slots of the last segment block are marked empty (mask 0)
    for (int j = lane; j < sleft; j += 64)
      if (sblk + j < seg_cap) rec_seg[sblk + j] = make_int4(0, 0, 0, 0);
    if (lane == 0) rec_wtail[(wtail_base + item) * 4 + wave] = make_int2((int)cblk, SBLK - sleft);
  }
  if constexpr (COUNT) {
    if (lane == 0) {
      atomicAdd(&counters[0], n_test);
      atomicAdd(&counters[1], n_hit);
      atomicAdd(&counters[2], n_contrib);
      atomicAdd(&counters[3], n_step);
      atomicAdd(&counters[4], n_step_hit);
      atomicAdd(&counters[5], n_step_shade);
    }
  }
}

// Total records listed by the segments (the block reservation leaves unused
// record slots, so the reserved count is an upper bound).
__global__ void __launch_bounds__(256) k_seg_total(const int4* __restrict__ seg, int64_t nseg,
                                                   unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[4];
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += (int64_t)gridDim.x * blockDim.x)
    acc += (unsigned long long)seg_count(seg[i]);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(total, part[0] + part[1] + part[2] + part[3]);
}

// argmin over cells with a non-empty power cell of pow(o, p_i) in float64;
// ties go to the lower index.  Stage 1: per block; stage 2: one block.
__global__ void __launch_bounds__(256) k_start_partial(const float* __restrict__ p, const float* __restrict__ w,
                                                       const int32_t* __restrict__ flags, int64_t n, double ox,
                                                       double oy, double oz, double* __restrict__ pk,
                                                       long long* __restrict__ pi) {
  double best = INFINITY;
  long long bi = -1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (flags[i] & FLAG_EMPTY_POWER) continue;
    const double ex = ox - p[3 * i], ey = oy - p[3 * i + 1], ez = oz - p[3 * i + 2];
    const double k = ex * ex + ey * ey + ez * ez - (double)w[i];
    if (k < best || (k == best && (bi < 0 || i < bi))) {
      best = k;
      bi = i;
    }
  }
  __shared__ double sk[256];
  __shared__ long long si[256];
  sk[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double k2 = sk[threadIdx.x + s];
      const long long i2 = si[threadIdx.x + s];
      if (i2 >= 0 && (si[threadIdx.x] < 0 || k2 < sk[threadIdx.x] || (k2 == sk[threadIdx.x] && i2 < si[threadIdx.x]))) {
        sk[threadIdx.x] = k2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pk[blockIdx.x] = sk[0];
    pi[blockIdx.x] = si[0];
  }
}

__global__ void __launch_bounds__(256) k_start_final(const double* __restrict__ pk, const long long* __restrict__ pi,
                                                     int nb, int32_t* __restrict__ out) {
  __shared__ double sk[256];
  __shared__ long long si[256];
  double best = INFINITY;
  long long bi = -1;
  for (int b = threadIdx.x; b < nb; b += 256) {
    if (pi[b] >= 0 && (bi < 0 || pk[b] < best || (pk[b] == best && pi[b] < bi))) {
      best = pk[b];
      bi = pi[b];
    }
  }
  sk[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double k2 = sk[threadIdx.x + s];
      const long long i2 = si[threadIdx.x + s];
      if (i2 >= 0 && (si[threadIdx.x] < 0 || k2 < sk[threadIdx.x] || (k2 == sk[threadIdx.x] && i2 < si[threadIdx.x]))) {
        sk[threadIdx.x] = k2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (int32_t)si[0];
}

// STORE: every contribution is also written as a record (as the store-mode
// rasteriser does) with a one-record segment; rec_seg must be zeroed by the
// caller (unused slots of the wave's segment blocks keep an empty mask).
// Six waves per SIMD (at most 80 VGPRs): the walk is bound by the latency of
// its per-step gathers, and occupancy hides it (100 Mrays/s at the three
// waves that 136 unconstrained VGPRs allow, 125 at six).
// COUNT: the walk's work counters are added to counters[0..5]
// (TRACE_COUNTERS): rays walked, cells walked, pieces computed (sphere
// hits), contributions, exit faces scanned, and the most cells one ray
// walked (maximum).
template <bool STORE, bool COUNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_trace(ViewArgs v, int64_t tile_first, SceneDev S, const int32_t* __restrict__ start,
                                               float t_min, int max_steps, float* __restrict__ rgba,
                                               unsigned long long* __restrict__ truncated, int view,
                                               int4* __restrict__ rec_ri, float4* __restrict__ rec_rf,
                                               float* __restrict__ rec_rt, int32_t* __restrict__ rec_head,
                                               unsigned long long* __restrict__ rec_counter,
                                               int4* __restrict__ rec_seg, int64_t rec_cap, int64_t seg_cap,
                                               unsigned long long* __restrict__ counters) {
  int px, py;
  tile_pixel(v.tiles_x, px, py, (int)(tile_first + blockIdx.x));
  const bool inside = px < v.cam.width && py < v.cam.height;
  const RayD R = make_ray(v.cam, px + 0.5, py + 0.5);
  bool live = inside && R.valid;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  int cell = start[0];
  int prev = -1;
  double t_cur = 0.0;
  bool cut = false;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int pix = py * v.cam.width + px;
  int head = -1;
  // the wave's current record / segment blocks; the lanes still walking
  // update them together
  long long rblk = 0, sblk = 0;
  int rleft = 0, sleft = 0;
  unsigned long long n_pieces = 0, n_contrib = 0, n_faces = 0;
  int n_steps = 0;
  const bool walked = live && cell >= 0;
  if (live && cell >= 0) {
    int step = 0;
    for (; step < max_steps; ++step) {
      const float4 g = S.geo[cell];
      const Local L = make_local(R, g.x, g.y, g.z);
      // contribution of this cell (identical code to the rasteriser)
      const float rho = S.cull[cell];
      bool contrib = false;
      Piece P;
      float r = 0.0f, gg = 0.0f, b = 0.0f;
      if (rho >= 0.0f && L.qq < (double)rho * (double)rho) {
        const float* tx = S.tex + (int64_t)cell * (KD * TEXW);
        const int r0 = S.row[cell];
        P = piece_geometry<false>(R, L, g.w, S.plane + r0, S.nrast[cell], S.nrm[cell], tx, S.tau);
        if (P.alpha > 0.0f) {
          radiance<false>(tx, S.rgb + 3 * (int64_t)cell, P.ux, P.uy, R.fx, R.fy, R.fz, S.tau, r, gg, b);
          contrib = true;
        }
        if constexpr (COUNT) {
          ++n_pieces;
          n_contrib += contrib ? 1ull : 0ull;
        }
      }
      if constexpr (STORE) {
        const uint64_t m = __ballot(contrib);
        if (m) {
          const int leader = __ffsll((long long)__ballot(true)) - 1;
          const int cnt = __popcll(m);
          if (cnt > rleft) {
            unsigned long long bk = 0;
            if (lane == leader) bk = atomicAdd(&rec_counter[0], (unsigned long long)RBLK);
            rblk = (long long)bcast64(bk);
            rleft = RBLK;
          }
          if (cnt > sleft) {
            unsigned long long bk = 0;
            if (lane == leader) bk = atomicAdd(&rec_counter[1], (unsigned long long)RBLK);
            sblk = (long long)bcast64(bk);
            sleft = RBLK;
          }
          if (contrib) {
            const long long slot = rblk + __popcll(m & lt), sg = sblk + __popcll(m & lt);
            if (slot < rec_cap) {
              rec_ri[slot] = make_int4(cell, pix, head, pack_view_bind(view, P.bind0, P.bind1));
              rec_rf[slot] = make_float4(P.alpha, r, gg, b);
              rec_rt[slot] = T;
              head = (int)slot;
              if (sg < seg_cap) rec_seg[sg] = make_int4(cell, (int)slot, 1, 0);   // mask 1: one record
            }
          }
          rblk += cnt;
          rleft -= cnt;
          sblk += cnt;
          sleft -= cnt;
        }
      }
      if (contrib) {
        const float wgt = T * P.alpha;
        cr += wgt * r;
        cg += wgt * gg;
        cb += wgt * b;
        T *= (1.0f - P.alpha);
      }
      if (T < t_min) break;
      // exit: nearest face ahead of the current position that the ray leaves through
      const float s_cur = (float)(t_cur + L.b);
      const int f0 = S.row[cell], f1 = S.row[cell + 1];
      if constexpr (COUNT) n_faces += (unsigned long long)(f1 - f0);
      float best = INFINITY, best_any = INFINITY;
      int bf = -1, bf_any = -1;
      for (int f = f0; f < f1; ++f) {
        const int nbr = S.col[f];
        if (nbr == prev) continue;
        const float4 pl = S.plane[f];
        const float a = R.fx * pl.x + R.fy * pl.y + R.fz * pl.z;
        if (!(a > 0.0f)) continue;
        const float s = face_offset(pl, -L.qx, -L.qy, -L.qz) * frcp(a);
        if (s < best_any) { best_any = s; bf_any = f; }
        if (s >= s_cur - 1e-6f * (1.0f + fabsf(s_cur)) && s < best) { best = s; bf = f; }
      }
      if (bf < 0) { bf = bf_any; best = best_any; }
      if (bf < 0) break;
      t_cur = fmax(t_cur, (double)best - L.b);
      const int nx = S.col[bf];
      if (nx < 0) break;   // left the domain box
      prev = cell;
      cell = nx;
    }
    cut = step == max_steps;
    n_steps = step + (step < max_steps ? 1 : 0);
  }
  if (inside) {
    float* o = rgba + 4 * ((int64_t)py * v.cam.width + px);
    o[0] = cr;
    o[1] = cg;
    o[2] = cb;
    o[3] = 1.0f - T;
    if constexpr (STORE) rec_head[pix] = head;
  }
  const uint64_t bc = __ballot(cut);
  if ((threadIdx.x & 63) == 0 && bc) atomicAdd(truncated, (unsigned long long)__popcll(bc));
  if constexpr (COUNT) {
    unsigned long long w_steps = (unsigned long long)n_steps, w_pieces = n_pieces, w_contrib = n_contrib,
                       w_faces = n_faces;
    int w_max = n_steps;
    for (int o = 32; o > 0; o >>= 1) {
      w_steps += __shfl_xor(w_steps, o, 64);
      w_pieces += __shfl_xor(w_pieces, o, 64);
      w_contrib += __shfl_xor(w_contrib, o, 64);
      w_faces += __shfl_xor(w_faces, o, 64);
      w_max = max(w_max, __shfl_xor(w_max, o, 64));
    }
    const uint64_t bw = __ballot(walked);
    if (lane == 0) {
      atomicAdd(&counters[0], (unsigned long long)__popcll(bw));
      atomicAdd(&counters[1], w_steps);
      atomicAdd(&counters[2], w_pieces);
      atomicAdd(&counters[3], w_contrib);
      atomicAdd(&counters[4], w_faces);
      atomicMax(&counters[5], (unsigned long long)w_max);
    }
  }
}

SceneDev scene_dev(const Scene& sc) {
  SceneDev d;
  d.geo = sc.geo;
  d.nrm = sc.nrm;
  d.cull = sc.cull;
  d.row = sc.row;
  d.nrast = sc.nrast;
  d.col = sc.col;
  d.plane = sc.plane;
  d.rgb = sc.prm.rgb;
  d.tex = sc.prm.tex;
  d.tau = sc.prm.tau;
  return d;
}

template <typename T>
struct Buf {
  T* p = nullptr;
  hipStream_t s;
  explicit Buf(hipStream_t st) : s(st) {}
  ~Buf() { if (p) pf::pool_free(p, s); }
  hipError_t alloc(size_t count) { return pf::pool_alloc((void**)&p, sizeof(T) * (count ? count : 1), s); }
};

}  // namespace

bool camera_ok(const pf_camera& c, std::string* why) {
  if (c.model != 0 && c.model != 1) { *why = "camera model must be 0 or 1"; return false; }
  if (c.width < 1 || c.height < 1 || (int64_t)c.width * c.height > (1ll << 31) / 4) {
    *why = "camera size out of range"; return false;
  }
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(c.c2w[i])) { *why = "non-finite camera matrix"; return false; }
  if (c.model == 0 && !(c.fx > 0 && c.fy > 0 && std::isfinite(c.cx) && std::isfinite(c.cy))) {
    *why = "pinhole intrinsics must be finite with fx, fy > 0"; return false;
  }
  if (c.model == 1 && !(c.f_fish > 0 && c.theta_max > 0 && c.theta_max <= 3.14159274f)) {
    *why = "fisheye needs f_fish > 0 and 0 < theta_max <= pi"; return false;
  }
  return true;
}

int raster_group_size(int64_t n, int ncam) {
  // views are processed in groups so that the per-(view, cell) scan fits 32 bits
  return (int)std::max<int64_t>(1, std::min<int64_t>(ncam, ((int64_t)1 << 28) / n));
}

int64_t view_tiles(const pf_camera& c) {
  return (int64_t)((c.width + TILE - 1) / TILE) * ((c.height + TILE - 1) / TILE);
}

int64_t raster_group_bytes(int64_t n, int nv, int64_t ntiles, int64_t np) {
  auto b = [](int64_t count, int64_t size) { return std::max<int64_t>(count, 1) * size; };
  const int64_t nvc = (int64_t)nv * n;
  return b(nv, sizeof(ViewDev)) + b(nvc + 1, 4) * 2 + b(nvc, 4) * 2 + b(ntiles + 1, 4) * 2 + b(ntiles, 4) +
         b(1, 4) + scan_scratch_bytes(nvc + 1) + scan_scratch_bytes(ntiles + 1) + b(np, 4) + b(np, 8) * 2;
}

namespace {

// The binned tile lists of one group of views (every buffer lives until
// the group is done).
struct Group {
  int c0 = 0, nv = 0;
  int64_t ntiles = 0, tiles_before = 0, pix_before = 0;
  uint32_t np = 0;
  Buf<ViewDev> views;
  Buf<uint32_t> cnt, key, off, tcnt, toff, fill, cone_list, cone_n, ptile;
  Buf<unsigned long long> pval, sorted;
  explicit Group(hipStream_t s)
      : views(s), cnt(s), key(s), off(s), tcnt(s), toff(s), fill(s), cone_list(s), cone_n(s), ptile(s), pval(s),
        sorted(s) {}
};

// Cull and count (count_only: stops after the pair count), then emit,
// bucket by tile and sort each tile's list.
pf_status bin_group(Scene& sc, const pf_camera* cams, Group& G, hipStream_t s, bool count_only) {
  const int64_t n = sc.n;
  const int nv = G.nv;
  std::vector<ViewDev> hv(nv);
  int64_t ntiles = 0, pix = G.pix_before;
  for (int v = 0; v < nv; ++v) {
    const pf_camera& cam = cams[G.c0 + v];
    hv[v].v.cam = cam;
    hv[v].v.tiles_x = (cam.width + TILE - 1) / TILE;
    hv[v].v.tiles_y = (cam.height + TILE - 1) / TILE;
    hv[v].tile_base = ntiles;
    hv[v].pix_base = pix;
    hv[v].view_id = G.c0 + v;
    ntiles += (int64_t)hv[v].v.tiles_x * hv[v].v.tiles_y;
    pix += (int64_t)cam.width * cam.height;
  }
  G.ntiles = ntiles;
  const int64_t nvc = (int64_t)nv * n;
  PF_HIP_TRY(G.views.alloc(nv));
  PF_HIP_TRY(hipMemcpyAsync(G.views.p, hv.data(), sizeof(ViewDev) * nv, hipMemcpyHostToDevice, s));
  PF_HIP_TRY(G.cnt.alloc(nvc + 1));
  PF_HIP_TRY(G.key.alloc(nvc));
  PF_HIP_TRY(G.off.alloc(nvc + 1));
  PF_HIP_TRY(G.tcnt.alloc(ntiles + 1));
  PF_HIP_TRY(G.toff.alloc(ntiles + 1));
  PF_HIP_TRY(G.fill.alloc(ntiles));
  PF_HIP_TRY(G.cone_list.alloc(nvc));
  PF_HIP_TRY(G.cone_n.alloc(1));
  PF_HIP_TRY(hipMemsetAsync(G.cone_n.p, 0, sizeof(uint32_t), s));
  const dim3 g((unsigned)((n + 255) / 256), (unsigned)nv);
  {
    ProfScope ps("k_view_count", s);
    k_view_count<<<g, 256, 0, s>>>(G.views.p, sc.geo, sc.cull, sc.prm.power, n, G.cnt.p, G.key.p, G.cone_list.p,
                                   G.cone_n.p);
  }
  PF_HIP_TRY(hipGetLastError());
  uint32_t ncone = 0;
  PF_HIP_TRY(hipMemcpyAsync(&ncone, G.cone_n.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  if (ncone) {
    k_cone_count<<<ncone, 256, 0, s>>>(G.views.p, sc.geo, sc.cull, n, G.cone_list.p, G.cnt.p);
    PF_HIP_TRY(hipGetLastError());
  }
  PF_HIP_TRY(hipMemsetAsync(G.cnt.p + nvc, 0, sizeof(uint32_t), s));
  PF_HIP_TRY(exclusive_scan_u32(G.cnt.p, G.off.p, nvc + 1, nullptr, s));
  uint32_t np = 0;
  PF_HIP_TRY(hipMemcpyAsync(&np, G.off.p + nvc, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  G.np = np;
  double ppc = (double)np / (double)nvc;   // sizing hint (renders may run on several threads)
  __atomic_store(&sc.pairs_per_cell, &ppc, __ATOMIC_RELAXED);
  if (count_only) return PF_OK;
  PF_HIP_TRY(G.ptile.alloc(np));
  PF_HIP_TRY(G.pval.alloc(np));
  PF_HIP_TRY(G.sorted.alloc(np));
  PF_HIP_TRY(hipMemsetAsync(G.tcnt.p, 0, sizeof(uint32_t) * (ntiles + 1), s));
  PF_HIP_TRY(hipMemsetAsync(G.fill.p, 0, sizeof(uint32_t) * ntiles, s));
  {
    ProfScope ps("k_view_emit", s);
    k_view_emit<<<g, 256, 0, s>>>(G.views.p, sc.geo, sc.cull, n, G.off.p, G.key.p, G.ptile.p, G.pval.p, G.tcnt.p);
    if (ncone)
      k_cone_emit<<<ncone, 256, 0, s>>>(G.views.p, sc.geo, sc.cull, n, G.off.p, G.key.p, G.cone_list.p, G.ptile.p,
                                        G.pval.p, G.tcnt.p);
  }
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(exclusive_scan_u32(G.tcnt.p, G.toff.p, ntiles + 1, nullptr, s));
  if (np) {
    k_tile_scatter<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(G.ptile.p, G.pval.p, np, G.toff.p, G.fill.p,
                                                               G.sorted.p);
    PF_HIP_TRY(hipGetLastError());
    ProfScope ps("k_tile_sort", s);
    k_tile_sort<<<(unsigned)ntiles, SORT_THREADS, 0, s>>>(G.sorted.p, G.toff.p);
    PF_HIP_TRY(hipGetLastError());
  }
  return PF_OK;
}

// Composite of the group's tiles [first, first + count) (one launch, one
// workgroup per tile); with records, the wave segment tails go to
// rec->wtail from index wtail_base.
pf_status composite(Scene& sc, Group& G, float t_min, float* rgba, hipStream_t s, const RecBuf* rec,
                    int64_t first, int64_t count, int64_t wtail_base, unsigned long long* counters) {
  if (count <= 0) return PF_OK;
  ProfScope ps(rec ? "k_raster_store" : "k_raster", s);
  const unsigned grid = (unsigned)count;
  if (rec) {
    const RecBuf& rb = *rec;
    if (counters)
      k_raster<true, true><<<grid, 256, 0, s>>>(G.views.p, G.nv, scene_dev(sc), G.sorted.p, G.toff.p, t_min, rgba,
                                                rb.ri, rb.rf, rb.rt, rb.head, rb.counter, rb.seg, rb.wtail, first,
                                                wtail_base, rb.cap, rb.seg_cap, counters);
    else
      k_raster<true, false><<<grid, 256, 0, s>>>(G.views.p, G.nv, scene_dev(sc), G.sorted.p, G.toff.p, t_min, rgba,
                                                 rb.ri, rb.rf, rb.rt, rb.head, rb.counter, rb.seg, rb.wtail, first,
                                                 wtail_base, rb.cap, rb.seg_cap, nullptr);
  } else if (counters) {
    k_raster<false, true><<<grid, 256, 0, s>>>(G.views.p, G.nv, scene_dev(sc), G.sorted.p, G.toff.p, t_min, rgba,
                                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, first, 0,
                                               0, 0, counters);
  } else {
    k_raster<false, false><<<grid, 256, 0, s>>>(G.views.p, G.nv, scene_dev(sc), G.sorted.p, G.toff.p, t_min, rgba,
                                                nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, first,
                                                0, 0, 0, nullptr);
  }
  PF_HIP_TRY(hipGetLastError());
  return PF_OK;
}

}  // namespace

pf_status raster_views(Scene& sc, const pf_camera* cams, int ncam, float t_min, float* rgba, hipStream_t s,
                       const RecBuf* rec, const GroupFn* fn, unsigned long long* counters) {
  const int group = raster_group_size(sc.n, ncam);
  int64_t pix_done = 0, tiles_done = 0;
  for (int c0 = 0; c0 < ncam; c0 += group) {
    Group G(s);
    G.c0 = c0;
    G.nv = std::min(group, ncam - c0);
    G.tiles_before = tiles_done;
    G.pix_before = pix_done;
    pf_status st = bin_group(sc, cams, G, s, false);
    if (st != PF_OK) return st;
    if (fn) {
      const GroupComposite run = [&](int64_t first, int64_t count, const RecBuf* r) {
        return composite(sc, G, t_min, rgba, s, r, first, count, 0, counters);
      };
      st = (*fn)(tiles_done, G.ntiles, run);
    } else {
      st = composite(sc, G, t_min, rgba, s, rec, 0, G.ntiles, tiles_done, counters);
    }
    if (st != PF_OK) return st;
    tiles_done += G.ntiles;
    for (int v = 0; v < G.nv; ++v) pix_done += (int64_t)cams[c0 + v].width * cams[c0 + v].height;
  }
  return PF_OK;
}

pf_status raster_workspace(Scene& sc, const pf_camera* cams, int ncam, hipStream_t s, int64_t* bytes) {
  const int group = raster_group_size(sc.n, ncam);
  int64_t worst = 0, pix_done = 0;
  for (int c0 = 0; c0 < ncam; c0 += group) {
    Group G(s);
    G.c0 = c0;
    G.nv = std::min(group, ncam - c0);
    G.pix_before = pix_done;
    const pf_status st = bin_group(sc, cams, G, s, true);
    if (st != PF_OK) return st;
    worst = std::max(worst, raster_group_bytes(sc.n, G.nv, G.ntiles, G.np));
    for (int v = 0; v < G.nv; ++v) pix_done += (int64_t)cams[c0 + v].width * cams[c0 + v].height;
  }
  *bytes = worst;
  return PF_OK;
}

pf_status seg_record_total(const int4* seg, int64_t nseg, unsigned long long* total_dev, hipStream_t s) {
  PF_HIP_TRY(hipMemsetAsync(total_dev, 0, sizeof(unsigned long long), s));
  if (nseg > 0) {
    const unsigned nb = (unsigned)std::min<int64_t>(1024, (nseg + 255) / 256);
    k_seg_total<<<nb, 256, 0, s>>>(seg, nseg, total_dev);
    PF_HIP_TRY(hipGetLastError());
  }
  return PF_OK;
}

pf_status trace_view(const Scene& sc, const pf_camera& cam, float t_min, int max_steps, float* rgba,
                     unsigned long long* trunc_dev, hipStream_t s, const RecBuf* rec, int view, int64_t pix_base,
                     int64_t tile_first, int64_t tile_count, const TraceScratch* scratch,
                     unsigned long long* counters) {
  const int64_t n = sc.n;
  ViewArgs v;
  v.cam = cam;
  v.tiles_x = (cam.width + TILE - 1) / TILE;
  v.tiles_y = (cam.height + TILE - 1) / TILE;
  const int64_t ntiles = tile_count >= 0 ? tile_count : (int64_t)v.tiles_x * v.tiles_y - tile_first;
  if (ntiles <= 0) return PF_OK;
  const int nb = (int)std::min<int64_t>(TRACE_START_BLOCKS, (n + 255) / 256);
  Buf<double> pk_own(s);
  Buf<long long> pi_own(s);
  Buf<int32_t> start_own(s);
  double* pk = scratch ? scratch->pk : nullptr;
  long long* pi = scratch ? scratch->pi : nullptr;
  int32_t* start = scratch ? scratch->start : nullptr;
  if (!scratch) {
    PF_HIP_TRY(pk_own.alloc(nb));
    PF_HIP_TRY(pi_own.alloc(nb));
    PF_HIP_TRY(start_own.alloc(1));
    pk = pk_own.p;
    pi = pi_own.p;
    start = start_own.p;
  }
  k_start_partial<<<nb, 256, 0, s>>>(sc.prm.p, sc.prm.power, sc.flags, n, cam.c2w[3], cam.c2w[7], cam.c2w[11],
                                     pk, pi);
  PF_HIP_TRY(hipGetLastError());
  k_start_final<<<1, 256, 0, s>>>(pk, pi, nb, start);
  PF_HIP_TRY(hipGetLastError());
  ProfScope ps(rec ? "k_trace_store" : "k_trace", s);
  if (rec) {
    const RecBuf& rb = *rec;
    if (counters)
      k_trace<true, true><<<(unsigned)ntiles, 256, 0, s>>>(v, tile_first, scene_dev(sc), start, t_min, max_steps,
                                                           rgba, trunc_dev, view, rb.ri, rb.rf, rb.rt,
                                                           rb.head + pix_base, rb.counter, rb.seg, rb.cap, rb.seg_cap,
                                                           counters);
    else
      k_trace<true, false><<<(unsigned)ntiles, 256, 0, s>>>(v, tile_first, scene_dev(sc), start, t_min, max_steps,
                                                            rgba, trunc_dev, view, rb.ri, rb.rf, rb.rt,
                                                            rb.head + pix_base, rb.counter, rb.seg, rb.cap,
                                                            rb.seg_cap, nullptr);
  } else if (counters) {
    k_trace<false, true><<<(unsigned)ntiles, 256, 0, s>>>(v, tile_first, scene_dev(sc), start, t_min, max_steps, rgba,
                                                          trunc_dev, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                          nullptr, 0, 0, counters);
  } else {
    k_trace<false, false><<<(unsigned)ntiles, 256, 0, s>>>(v, tile_first, scene_dev(sc), start, t_min, max_steps,
                                                           rgba, trunc_dev, 0, nullptr, nullptr, nullptr, nullptr,
                                                           nullptr, nullptr, 0, 0, nullptr);
  }
  PF_HIP_TRY(hipGetLastError());
  return PF_OK;
}

}  // namespace pf
