// Backward pass of the rasteriser: gradients of L with respect to every cell
// parameter, given dL/dRGBA and the contribution records of a store-mode
// forward.
//
//   k_suffix      per pixel, records back to front:  with the normalised
//                 colour and alpha behind contribution k,
//                   Cb_{k} = a_k c_k + (1 - a_k) Cb_{k+1},  Ab likewise,
//                 dL/da_k = T_k (gC.(c_k - Cb_{k+1}) + gA (1 - Ab_{k+1})),
//                 dL/dc_k = T_k a_k gC                      (Sec. 3.1 sum)
//                 plus, with the normal loss, the same for the scalar
//                 channel max(n.d, 0)^2 weighted by lambda_normal; the
//                 record's T becomes the contribution T a.  Raster records:
//                 k_suffix_seg walks each wave's segments in reverse append
//                 order; walk records: k_suffix follows the pixel chains
//   k_seg_hist /  records grouped by cell through the forward's segment list
//                 (raster records: counted per cell by k_suffix_seg)
//   k_seg_scatter (one atomic per segment of <= 64 contiguous records)
//   k_bwd_cell    one wave per chunk of a cell's records, 64 records at a
//                 time.  Lane = record: re-derives the piece (bounded
//                 interval from its binding sphere / face / ray start,
//                 dipole split with displacement, radiance) and applies the
//                 chain rule by hand, in reverse order of the forward; the
//                 per-record sums (cell parameters, detail-site positions and
//                 displacements) are reduced over the wave four at a time
//                 (permlane32 / permlane16 swaps, then DPP, then an LDS
//                 atomic add).  The next batch's records are loaded while a
//                 batch is processed.
//                 The 6 Spherical-Voronoi gradients of each (detail site k,
//                 axis m) accumulate in registers over the chunk: the two
//                 3-term dot products per (record, (k, m)) come from 32x32x2
//                 FP32 MFMAs (records x site-axis pairs), the exponentials
//                 and sums from the VALU, reading each record's direction,
//                 dL/dc and per-site softmax terms from LDS.  Neighbour
//                 gradients through binding faces gather per face in LDS.
//                 Everything is flushed with one global atomic per (chunk,
//                 parameter).
#include "pf_backward.hpp"
#include "pf_shade.hpp"

#include <algorithm>
#include <vector>

namespace pf {
namespace {

constexpr int BWD_THREADS = 64;     // one wave per workgroup
constexpr int CHUNK = 2048;         // records per workgroup
constexpr int FMAX_B = 128;         // faces gathered in LDS; faces beyond add to global directly
constexpr int NCELL = 12;           // p(3) w r n(3) lambda rgb(3)
constexpr int NSUM = NCELL + 3 * KD;  // + detail-site s(2), d per site
constexpr int ISTAT = NSUM;           // + the cell's contribution sum (statistic)
constexpr int KPAD = 65;            // row pitch of the per-site LDS table (bank spread)

// One workgroup per 16x16 tile of a view, one wave per 8x8 quadrant, lanes
// row-major in the quadrant: the pixel layout of the store-mode raster, so
// that the lanes of a wave walk records its raster wave appended side by side.
__global__ void __launch_bounds__(256) k_suffix(const int32_t* __restrict__ head, int ncam, int64_t tile0,
                                                const float* __restrict__ d_rgba, const int4* __restrict__ ri,
                                                float4* __restrict__ rf, float* __restrict__ rt,
                                                const pf_camera* __restrict__ cams, const float4* __restrict__ nrm,
                                                float lambda_n, double* __restrict__ normal_loss,
                                                const float* __restrict__ pix_err, float* __restrict__ rte) {
  int64_t tile = tile0 + blockIdx.x, base = 0;
  int v = 0;
  for (; v < ncam - 1; ++v) {
    const int nt = ((cams[v].width + TILE - 1) / TILE) * ((cams[v].height + TILE - 1) / TILE);
    if (tile < nt) break;
    tile -= nt;
    base += (int64_t)cams[v].width * cams[v].height;
  }
  const int W = cams[v].width, H = cams[v].height, tiles_x = (W + TILE - 1) / TILE;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = (int)(tile % tiles_x) * TILE + (w & 1) * 8 + (lane & 7);
  const int py = (int)(tile / tiles_x) * TILE + (w >> 1) * 8 + (lane >> 3);
  const bool inside = px < W && py < H;
  const int64_t i = base + (int64_t)py * W + px;
  int k = inside ? head[i] : -1;
  double lpix = 0.0;   // this pixel's sum of T a max(n.d, 0)^2
  if (k >= 0) {
    const float e = pix_err ? pix_err[i] : 0.0f;
    const float gr = d_rgba[4 * i], gg = d_rgba[4 * i + 1], gb = d_rgba[4 * i + 2], ga = d_rgba[4 * i + 3];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    if (lambda_n != 0.0f || normal_loss) {
      const int4 r0 = ri[k];
      const pf_camera& cam = cams[rec_view(r0.w)];
      const RayD R = make_ray(cam, r0.y % cam.width + 0.5, r0.y / cam.width + 0.5);
      fx = R.fx;
      fy = R.fy;
      fz = R.fz;
    }
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, ab = 0.0f, nb = 0.0f;
    while (k >= 0) {
      const int4 r = ri[k];
      const float4 f = rf[k];
      const float T = rt[k];
      const float a = f.x;
      float nu = 0.0f;
      if (lambda_n != 0.0f || normal_loss) {
        const float4 nv = nrm[r.x];
        const float c = fmaxf(nv.x * fx + nv.y * fy + nv.z * fz, 0.0f);
        nu = c * c;
      }
      const float g_alpha = T * (gr * (f.y - cr) + gg * (f.z - cg) + gb * (f.w - cb) + ga * (1.0f - ab) +
                                 lambda_n * (nu - nb));
      const float ta = T * a;
      rf[k] = make_float4(g_alpha, ta * gr, ta * gg, ta * gb);
      rt[k] = ta;   // the contribution T a (read by the per-cell pass)
      if (rte) rte[k] = ta * e;   // its share of the pixel's error
      lpix += (double)ta * (double)nu;
      cr = a * f.y + (1.0f - a) * cr;
      cg = a * f.z + (1.0f - a) * cg;
      cb = a * f.w + (1.0f - a) * cb;
      ab = a + (1.0f - a) * ab;
      nb = a * nu + (1.0f - a) * nb;
      k = r.z;
    }
  }
  if (normal_loss) {
    for (int o = 32; o > 0; o >>= 1) lpix += __shfl_xor(lpix, o, 64);
    if ((threadIdx.x & 63) == 0 && lpix != 0.0) atomicAdd(normal_loss, lpix);
  }
}

// The same pass over a raster's records without the chains: each wave walks
// the segments its raster wave appended, last block first and, in a block,
// last segment first, so that every pixel of the wave meets its records back
// to front as along its chain (the arithmetic is the same, in the same
// order).  A segment's records are contiguous and its cell is uniform: the
// loads and stores are coalesced and no record waits for the one behind it.
// The pass also adds each segment's record count to cnt[cell] (zeroed by
// the caller), the histogram that groups the records by cell.
__global__ void __launch_bounds__(256) k_suffix_seg(const int4* __restrict__ seg, const int2* __restrict__ wtail,
                                                    int ncam, int64_t tile0, const float* __restrict__ d_rgba,
                                                    float4* __restrict__ rf, float* __restrict__ rt,
                                                    const pf_camera* __restrict__ cams, const float4* __restrict__ nrm,
                                                    float lambda_n, double* __restrict__ normal_loss,
                                                    const float* __restrict__ pix_err, float* __restrict__ rte,
                                                    uint32_t* __restrict__ cnt) {
  int64_t tile = tile0 + blockIdx.x, base = 0;
  int v = 0;
  for (; v < ncam - 1; ++v) {
    const int nt = ((cams[v].width + TILE - 1) / TILE) * ((cams[v].height + TILE - 1) / TILE);
    if (tile < nt) break;
    tile -= nt;
    base += (int64_t)cams[v].width * cams[v].height;
  }
  const int W = cams[v].width, H = cams[v].height, tiles_x = (W + TILE - 1) / TILE;
  // (the wave index made visibly wave-uniform, so that the wave's segments
  // are read through scalar loads: 3.4 -> 3.0 ms)
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int px = (int)(tile % tiles_x) * TILE + (w & 1) * 8 + (lane & 7);
  const int py = (int)(tile / tiles_x) * TILE + (w >> 1) * 8 + (lane >> 3);
  const bool inside = px < W && py < H;
  const int64_t i = base + (int64_t)py * W + px;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const bool nl = lambda_n != 0.0f || normal_loss;
  float e = 0.0f, gr = 0.0f, gg = 0.0f, gb = 0.0f, ga = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
  if (inside) {
    e = pix_err ? pix_err[i] : 0.0f;
    gr = d_rgba[4 * i];
    gg = d_rgba[4 * i + 1];
    gb = d_rgba[4 * i + 2];
    ga = d_rgba[4 * i + 3];
    if (nl) {
      const RayD R = make_ray(cams[v], px + 0.5, py + 0.5);
      fx = R.fx;
      fy = R.fy;
      fz = R.fz;
    }
  }
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, ab = 0.0f, nb = 0.0f;
  double lpix = 0.0;   // this pixel's sum of T a max(n.d, 0)^2
  const int2 tl = wtail[(int64_t)blockIdx.x * 4 + w];
  int blk = tl.x, top = tl.y;   // the wave's last block and the slots used in it
  while (blk >= 0) {
    for (int j = top - 1; j >= 1; --j) {   // slot 0 is the block's header
      const int4 g = seg[(int64_t)blk + j];
      const uint64_t m = (uint64_t)(uint32_t)g.z | ((uint64_t)(uint32_t)g.w << 32);
      // the per-cell record counts of the grouping by cell (every segment
      // lies on exactly one wave's chain)
      if (lane == 0 && m) atomicAdd(&cnt[g.x], (uint32_t)__popcll(m));
      if (!((m >> lane) & 1ull)) continue;
      const int64_t k = (int64_t)g.y + __popcll(m & lt);
      const float4 f = rf[k];
      const float T = rt[k];
      const float a = f.x;
      float nu = 0.0f;
      if (nl) {
        const float4 nv = nrm[g.x];
        const float c = fmaxf(nv.x * fx + nv.y * fy + nv.z * fz, 0.0f);
        nu = c * c;
      }
      const float g_alpha = T * (gr * (f.y - cr) + gg * (f.z - cg) + gb * (f.w - cb) + ga * (1.0f - ab) +
                                 lambda_n * (nu - nb));
      const float ta = T * a;
      rf[k] = make_float4(g_alpha, ta * gr, ta * gg, ta * gb);
      rt[k] = ta;
      if (rte) rte[k] = ta * e;
      lpix += (double)ta * (double)nu;
      cr = a * f.y + (1.0f - a) * cr;
      cg = a * f.z + (1.0f - a) * cg;
      cb = a * f.w + (1.0f - a) * cb;
      ab = a + (1.0f - a) * ab;
      nb = a * nu + (1.0f - a) * nb;
    }
    blk = seg[blk].y;   // the header's link to the wave's previous (full) block
    top = SEG_BLOCK;
  }
  if (normal_loss) {
    for (int o = 32; o > 0; o >>= 1) lpix += __shfl_xor(lpix, o, 64);
    if ((threadIdx.x & 63) == 0 && lpix != 0.0) atomicAdd(normal_loss, lpix);
  }
}

__global__ void k_seg_hist(const int4* __restrict__ seg, int64_t nseg, uint32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nseg) {
    const int4 g = seg[i];
    const int c = seg_count(g);
    if (c > 0) atomicAdd(&cnt[g.x], (uint32_t)c);
  }
}

// A lane per segment reserves the segment's run of its cell's order list;
// the wave then writes its segments' runs one after the other, a lane per
// entry (a segment holds at most 64 records), so that every store is
// contiguous across the wave.
__global__ void k_seg_scatter(const int4* __restrict__ seg, int64_t nseg, const uint32_t* __restrict__ off,
                              uint32_t* __restrict__ fill, int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int c = 0, first = 0;
  uint32_t at = 0;
  if (i < nseg) {
    const int4 g = seg[i];
    c = seg_count(g);   // 0: block header or unused slot
    if (c > 0) {
      at = off[g.x] + atomicAdd(&fill[g.x], (uint32_t)c);
      first = g.y;
    }
  }
  for (uint64_t m = __ballot(c > 0); m; m &= m - 1) {
    const int src = __ffsll((long long)m) - 1;
    const int cs = __builtin_amdgcn_readlane(c, src), fs = __builtin_amdgcn_readlane(first, src);
    const uint32_t as = (uint32_t)__builtin_amdgcn_readlane((int)at, src);
    if (lane < cs) order[as + lane] = fs + lane;
  }
}

__global__ void k_chunk_count(const uint32_t* __restrict__ cnt, int64_t n, uint32_t* __restrict__ nch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nch[i] = (cnt[i] + CHUNK - 1) / CHUNK;
}

__global__ void k_chunk_fill(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ off,
                             const uint32_t* __restrict__ choff, int64_t n, int4* __restrict__ chunks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cnt[i];
  for (uint32_t k = 0; k * CHUNK < c; ++k) {
    const uint32_t a = off[i] + k * CHUNK;
    const uint32_t b = off[i] + min(c, (k + 1) * CHUNK);
    chunks[choff[i] + k] = make_int4((int)i, (int)a, (int)b, 0);
  }
}

// Sum of x over the wave, valid in lane 63: DPP butterflies within rows of
// 16 lanes, then the row broadcasts of lane 15 and lane 31.
__device__ inline float wave_total(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xf, 0xf, false));  // quad [1,0,3,2]
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xf, 0xf, false));  // quad [2,3,0,1]
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xf, 0xf, false)); // row half mirror
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xf, 0xf, false)); // row mirror
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xa, 0xf, false)); // row bcast 15
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xc, 0xf, false)); // row bcast 31
  return x;
}

// acc[i] += sum over the wave of (valid ? v : 0); acc is the wave's own LDS.
// The update is an LDS atomic add without return, so that the wave does not
// wait for a read of acc[i] (a read-add-write waited for each of them: 50.7
// instead of 45.0 ms for the kernel).
__device__ inline void sum_to(float* acc, int i, bool valid, float v) {
  const float t = wave_total(valid ? v : 0.0f);
  if ((threadIdx.x & 63) == 63) atomicAdd(&acc[i], t);
}


// Four wave sums at once: acc[dst] += sum over the wave of (valid ? v_j : 0)
// for j = sum4_value(lane), in the first lane of each row of 16.  permlane32
// swaps pair v0 with v1 and v2 with v3, a permlane16 swap pairs the results,
// so that after two adds rows 0..3 of the wave hold partial sums of v0, v2,
// v1, v3; four DPP steps finish the row sums, and the first lane of each row
// adds its value to acc[dst] (LDS atomic).  dst is computed by the caller from
// sum4_value(lane), a per-lane constant, so that the choice of the
// destination costs no branch.
__device__ inline int sum4_value(int lane) { return ((lane >> 4) & 1) * 2 + (lane >> 5); }

__device__ inline void sum4_to(float* acc, int dst, bool valid, float v0, float v1, float v2, float v3) {
  v0 = valid ? v0 : 0.0f;
  v1 = valid ? v1 : 0.0f;
  v2 = valid ? v2 : 0.0f;
  v3 = valid ? v3 : 0.0f;
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v0), __float_as_uint(v1), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v2), __float_as_uint(v3), false, false);
  const float s01 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const float s23 = __uint_as_float(b[0]) + __uint_as_float(b[1]);
  const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(s01), __float_as_uint(s23), false, false);
  float t = __uint_as_float(c[0]) + __uint_as_float(c[1]);
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0xB1, 0xf, 0xf, false));  // quad [1,0,3,2]
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x4E, 0xf, 0xf, false));  // quad [2,3,0,1]
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x141, 0xf, 0xf, false)); // row half mirror
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x140, 0xf, 0xf, false)); // row mirror
  if ((threadIdx.x & 15) == 0) atomicAdd(&acc[dst], t);
}

__device__ inline float softplus_b(float x) { return x > 20.0f ? x : log1pf(expf(x)); }

// A wave-uniform double moved to scalar registers.
__device__ inline double uni(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/x in float64 (x != 0): the hardware reciprocal (about 24 bits on
// gfx950) refined by one Newton step, about 47 bits: the chains below end
// in float32.
__device__ inline double rcp_d(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Length and reciprocal length of a 2-vector from its squared length x2
// (float64): the hardware reciprocal square root (about 24 bits) refined by
// one Newton step, r <- r (3 - x2 r^2) / 2 (about 47 bits), then
// |v| = x2 / |v|.  Both are 0 for x2 = 0.
__device__ inline void len_rlen(double x2, double& len, double& rlen) {
  if (x2 > 0.0) {
    double r = __builtin_amdgcn_rsq(x2);
    const double hx = 0.5 * x2;
    r = r * fma(-hx * r, r, 1.5);
    rlen = r;
    len = x2 * r;
  } else {
    rlen = 0.0;
    len = 0.0;
  }
}

// Softmax backward of the soft-Voronoi weights at texture point u.  With
// z_k = -tau (|u - s_k| - |u|) and ge_k = dL/dz_k (float64), accumulates
// dL/du into (gux, guy) (float64) and the wave's sum of dL/ds_k into acc.
// d/du of the shifted logit, (u - s)/|u - s| - u/|u|, is evaluated as
// (-u (|u - s| - |u|) - s |u|) / (|u - s| |u|), which stays accurate when u
// is far from the sites (grazing rays).  The per-site geometry is float32
// (in float64 the kernel took 6% longer; against the oracle adjoint the
// worst per-component error over the GPU gradient tests rose from 7e-6 to
// 1.6e-4, on the normal of one small scene, the others unchanged).
__device__ inline void sv_backward(const float* __restrict__ tx, double ux_d, double uy_d, const double* ge,
                                   double& gux, double& guy, float* acc, bool valid) {
  const float ux = (float)ux_d, uy = (float)uy_d;
  const float u2 = ux * ux + uy * uy;
  const float iun = u2 > 0.0f ? __builtin_amdgcn_rsqf(u2) : 0.0f;
  const float un = u2 * iun;
  const int j4 = sum4_value(threadIdx.x);   // site k0 + j4 / 2, coordinate j4 % 2
  static_assert(KD % 2 == 0, "the site sums go two sites at a time");
#pragma unroll
  for (int k0 = 0; k0 < KD; k0 += 2) {
    float vx[2], vy[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = k0 + h;
      const float sx = tx[k * TEXW], sy = tx[k * TEXW + 1];
      const float ex = ux - sx, ey = uy - sy;
      const float d2 = ex * ex + ey * ey;
      const float rd = d2 > 0.0f ? __builtin_amdgcn_rsqf(d2) : 0.0f;
      const float dist = d2 * rd;
      float lx, ly;
      if (un > 0.0f && dist > 0.0f) {
        const float e = (sx * sx + sy * sy - 2.0f * (ux * sx + uy * sy)) * frcp(dist + un);   // |u - s| - |u|
        const float f = rd * iun;
        lx = (-ux * e - sx * un) * f;
        ly = (-uy * e - sy * un) * f;
      } else {
        lx = ex * rd;
        ly = ey * rd;
      }
      gux += ge[k] * (double)lx;
      guy += ge[k] * (double)ly;
      const float gk = (float)ge[k];
      vx[h] = -gk * ex * rd;
      vy[h] = -gk * ey * rd;
    }
    sum4_to(acc, NCELL + 3 * k0 + j4 + (j4 >> 1), valid, vx[0], vy[0], vx[1], vy[1]);
  }
}

// Two waves per SIMD: at most 256 VGPRs, which the per-record float64
// chain fills without spilling (at three waves, 168 VGPRs, it spilled and ran
// 5% slower).
__global__ void __launch_bounds__(BWD_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) k_bwd_cell(
    const pf_camera* __restrict__ cams, const int4* __restrict__ ri, const float4* __restrict__ rf,
    const int32_t* __restrict__ order, const int4* __restrict__ chunks, const float* __restrict__ prm_p,
    const float* __restrict__ radius, const float* __restrict__ normal, const float* __restrict__ lamv,
    const float* __restrict__ tex, const int32_t* __restrict__ row, const int32_t* __restrict__ nrast,
    const int32_t* __restrict__ col, const float4* __restrict__ plane, float sigma_scale, float tau_, pf_grads G,
    const float* __restrict__ rta, float lambda_n, float* __restrict__ contribution) {
  __shared__ float4 st_dir[64];          // per record: ray direction (float), 0
  __shared__ float4 st_gc[64];           // per record: dL/dc, 0
  __shared__ float2 st_k[KD][KPAD];      // per record and site: softmax shift, dL/dw_k
  __shared__ float acc[NSUM + 1];
  __shared__ float4 facc[FMAX_B];
  __shared__ double s_fr[12];            // the cell's face frame (wave-uniform)
  // zeros, read back as a per-batch offset that the compiler cannot see
  // through: values derived from it are recomputed in every batch instead of
  // being hoisted out of the record loop and held (an LDS load, unlike an
  // empty asm statement, is no memory write, so the texture reads stay
  // scalar loads)
  __shared__ int s_zero[64];

  const int4 ch = chunks[blockIdx.x];
  const int ci = ch.x;
  const int lane = threadIdx.x;
  const int r0 = row[ci];
  const int nf = nrast[ci];
  const int nfl = min(nf, FMAX_B);
  const float* __restrict__ txc = tex + (int64_t)ci * KD * TEXW;
  for (int t = lane; t < NSUM + 1; t += BWD_THREADS) acc[t] = 0.0f;
  s_zero[lane] = 0;
  for (int t = lane; t < nfl; t += BWD_THREADS) facc[t] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

  // cell constants, computed exactly as the build's per-cell record
  const float px = prm_p[3 * ci], py = prm_p[3 * ci + 1], pz = prm_p[3 * ci + 2];
  const float rad = radius[ci];
  const float nrx = normal[3 * ci], nry = normal[3 * ci + 1], nrz = normal[3 * ci + 2];
  const float lam = lamv[ci];
  const float sigma = sigma_scale * softplus_b(lam);
  const float tau = tau_;
  // float64 face frame (for the displacement chain): n_hat, t1, t2 of
  // Duff et al., the sign and frame constant, 1/|n|.  It is wave-uniform but
  // float64 arithmetic runs on the vector unit, so it is kept in LDS and
  // re-read where used rather than held in (and spilled from) vector
  // registers across the record loop.
  if (lane == 0) {
    const double dninv = 1.0 / sqrt((double)nrx * nrx + (double)nry * nry + (double)nrz * nrz);
    const double dnx = nrx * dninv, dny = nry * dninv, dnz = nrz * dninv;
    const double dsg = copysign(1.0, dnz);
    const double a = -1.0 / (dsg + dnz);
    const double b = dnx * dny * a;
    s_fr[0] = dnx; s_fr[1] = dny; s_fr[2] = dnz;
    s_fr[3] = 1.0 + dsg * dnx * dnx * a; s_fr[4] = dsg * b; s_fr[5] = -dsg * dnx;
    s_fr[6] = b; s_fr[7] = dsg + dny * dny * a; s_fr[8] = -dny;
    s_fr[9] = dsg; s_fr[10] = a; s_fr[11] = dninv;
  }
  __syncthreads();

  // (site, axis) pair of this lane when the transposed phase's sums are
  // flushed
  const int km = lane >> 3, mm = lane & 7;
  // The transposed phase takes its two 3-term dot products per (record,
  // site-axis pair) from 32x32x2 FP32 MFMAs: logits L[r][km] = d_r . a_km
  // (axes scaled by log2(e)) and G[r][km] = gC_r . c_km, each as two MFMAs
  // over the components (0, 1) and (2, 3 = 0).  An MFMA result gives lane l
  // the column km = 32 cb + l % 32 and the rows r = 8 (v / 4) + 4 (l / 32)
  // + v % 4 of register v, so a lane accumulates two site-axis pairs (cb = 0,
  // 1) over its half of the records, and the halves are added at the end.
  const int hh = lane >> 5, j32 = lane & 31;
  float Ba[2][2], Bc[2][2];   // B operands [cb][step]: component 2 step + hh of a_km (scaled) and c_km
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int kmx = 32 * cb + j32;
    const float* t = txc + (kmx >> 3) * TEXW;
    const int m = kmx & 7;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int comp = 2 * st + hh;
      Ba[cb][st] = comp < 3 ? t[3 + 3 * m + comp] * LOG2E_F : 0.0f;
      Bc[cb][st] = comp < 3 ? t[3 + 3 * MA + 3 * m + comp] : 0.0f;
    }
  }
  float sa[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};   // dL/da partial sums [cb][xyz]
  float sc[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};   // dL/dc partial sums [cb][rgb]

  // the records of the next batch are loaded while this one is processed:
  // its order entries at the start of a batch, the records themselves once
  // the batch's own camera and face loads have returned
  int4 n_rec = make_int4(0, 0, -1, 0);
  float4 n_gf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float n_ta = 0.0f;
  if (ch.y + lane < ch.z) {
    const int ridx = order[ch.y + lane];
    n_rec = ri[ridx];
    n_gf = rf[ridx];
    n_ta = rta[ridx];
  }
  for (int base = ch.y; base < ch.z; base += 64) {
    // the texture is re-read per record batch (scalar loads, offset by the
    // opaque zero) rather than held in registers across the loop
    const int zo = s_zero[(base >> 6) & 63];   // 0
    const float* __restrict__ tx = txc + __builtin_amdgcn_readfirstlane(zo);
    const int idx = base + lane;
    const bool valid = idx < ch.z;
    const int nvalid = min(64, ch.z - base);
    const int4 rec = n_rec;
    const float4 gf = n_gf;
    const float ta = n_ta;   // the contribution T a
    const int nidx = idx + 64;
    const bool n_valid = nidx < ch.z;
    const int n_ridx = order[min(nidx, ch.z - 1)];   // (in the chunk; used only if n_valid)
    const int view = rec_view(rec.w);
    const int b0 = rec_bind0(rec.w), b1 = rec_bind1(rec.w);
    // the binding faces' planes, loaded before the ray set-up
    const float4 pl0 = (b0 >= 0 && b0 < nf) ? plane[r0 + b0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 pl1 = (b1 >= 0 && b1 < nf) ? plane[r0 + b1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // the camera is copied at once (its loads issued together) rather than
    // read field by field behind the branches of the ray set-up
    const pf_camera cam = cams[valid ? view : 0];
    const int pxl = rec.y % cam.width, pyl = rec.y / cam.width;
    const RayD R = make_ray(cam, pxl + 0.5, pyl + 0.5);
    const float fx = R.fx, fy = R.fy, fz = R.fz;
    const float g_alpha = gf.x;
    const float gcr = gf.y, gcg = gf.z, gcb = gf.w;
    st_dir[lane] = make_float4(fx, fy, fz, 0.0f);
    st_gc[lane] = make_float4(gcr, gcg, gcb, 0.0f);

    // ---------------- forward recompute.  Interval ends in float32 as in
    // piece_geometry; the face frame, displacement and texture point in
    // float64: for rays nearly parallel to the face the derivatives with
    // respect to the normal are small differences of terms ~1/(d.n)^2.
    // the cell's site and radius pass an opaque copy, so that their float64
    // conversions are made here rather than hoisted out of the loop (and
    // spilled)
    const float fz0 = __int_as_float(zo);   // +0
    const float cpx = px + fz0, cpy = py + fz0, cpz = pz + fz0, crad = rad + fz0;
    const Local L = make_local(R, cpx, cpy, cpz);
    const double Dd = (double)crad * (double)crad - L.qq;
    const float sq = fsqrt((float)fmax(Dd, 1e-30));
    const float a0 = fx * pl0.x + fy * pl0.y + fz * pl0.z;
    const float a1 = fx * pl1.x + fy * pl1.y + fz * pl1.z;
    const float s0 = (b0 == -1) ? -sq
                     : (b0 == -2) ? L.beta
                                  : face_offset(pl0, -L.qx, -L.qy, -L.qz) * frcp(a0);
    const float s1 = (b1 == -1) ? sq : face_offset(pl1, -L.qx, -L.qy, -L.qz) * frcp(a1);
    n_rec = make_int4(0, 0, -1, 0);
    n_gf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    n_ta = 0.0f;
    if (n_valid) {
      n_rec = ri[n_ridx];
      n_gf = rf[n_ridx];
      n_ta = rta[n_ridx];
    }
    const double ddx = R.dx, ddy = R.dy, ddz = R.dz;
    const double qdx = L.dqx, qdy = L.dqy, qdz = L.dqz;
    // (an opaque offset, so that the frame is read here, not hoisted)
    int fo = zo;
    double dnx = s_fr[fo], dny = s_fr[fo + 1], dnz = s_fr[fo + 2];
    double d1x = s_fr[fo + 3], d1y = s_fr[fo + 4], d1z = s_fr[fo + 5];
    double d2x = s_fr[fo + 6], d2y = s_fr[fo + 7], d2z = s_fr[fo + 8];
    const double den = ddx * dnx + ddy * dny + ddz * dnz;
    const double qn = qdx * dnx + qdy * dny + qdz * dnz;
    const double qt1 = qdx * d1x + qdy * d1y + qdz * d1z;
    const double qt2 = qdx * d2x + qdy * d2y + qdz * d2z;
    const double dt1 = ddx * d1x + ddy * d1y + ddz * d1z;
    const double dt2 = ddx * d2x + ddy * d2y + ddz * d2z;
    const bool nzden = den != 0.0;
    double idn = 0.0, sbar = 0.0, sxx = 0.0, delta = 0.0;
    float wd[KD];   // displacement weights at ubar
    double ubx = 0.0, uby = 0.0;
    double j0 = s0, j1 = s1;
    int sel0 = 0, sel1 = 0;   // 1: the end is the displaced face
    double ux, uy, S;
    if (nzden) {
      idn = rcp_d(den);
      sbar = -qn * idn;
      ubx = qt1 + sbar * dt1;
      uby = qt2 + sbar * dt2;
      sv_weights(tx, (float)ubx, (float)uby, tau, wd);
#pragma unroll
      for (int k = 0; k < KD; ++k) delta += (double)wd[k] * (double)tx[k * TEXW + 2];
      sxx = (delta - qn) * idn;
      if (den > 0.0) {
        sel1 = sxx < (double)s1;
        j1 = sel1 ? sxx : (double)s1;
      } else {
        sel0 = sxx > (double)s0;
        j0 = sel0 ? sxx : (double)s0;
      }
      S = sxx;
    } else {
#pragma unroll
      for (int k = 0; k < KD; ++k) wd[k] = 0.0f;
      S = 0.5 * ((double)s0 + (double)s1);
      if (!(qn < 0.0)) j1 = j0;
    }
    ux = qt1 + S * dt1;
    uy = qt2 + S * dt2;
    const float ell = (float)fmax(j1 - j0, 0.0);
    const float alpha = 1.0f - __expf(-sigma * ell);

    // ---------------- opacity
    const float om = 1.0f - alpha;
    const float g_ell = (ell > 0.0f) ? g_alpha * sigma * om : 0.0f;
    const float g_sigma = g_alpha * ell * om;
    const float g_lam = g_sigma * sigma_scale * frcp(1.0f + __expf(-lam));
    float g_s0 = 0.0f, g_s1 = 0.0f;
    double g_sx = 0.0;
    if (nzden || qn < 0.0) {
      if (sel1) g_sx += g_ell; else g_s1 += g_ell;
      if (sel0) g_sx -= g_ell; else g_s0 -= g_ell;
    }

    // ---------------- radiance: weights at u, the sites' Spherical-Voronoi
    // colours sv_k(d) and the softmax backward of the weights
    float wr[KD];
    sv_weights(tx, (float)ux, (float)uy, tau, wr);
    double sum_wg = 0.0;
    float gwr[KD];
    const float gx = fx * LOG2E_F, gy = fy * LOG2E_F, gz = fz * LOG2E_F;
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      float sum, sr, sg, sb;
      const float sh = sv_lobes(tx + k * TEXW, gx, gy, gz, sum, sr, sg, sb);
      const float inv = frcp(sum);
      gwr[k] = (gcr * sr + gcg * sg + gcb * sb) * inv;   // dL/dw_k = gC . sv_k
      sum_wg += (double)wr[k] * (double)gwr[k];
      // w_k softmax_m(a_km.d) = 2^(a_km.d log2(e) - shift_k), shift_k = sh - log2(w_k / sum)
      const float wi = wr[k] * inv;
      st_k[k][lane] = make_float2(valid && wi > 0.0f ? sh - __log2f(wi) : INFINITY, gwr[k]);
    }
    double gux = 0.0, guy = 0.0;
    {
      double ge[KD];
#pragma unroll
      for (int k = 0; k < KD; ++k) ge[k] = -(double)tau * (double)wr[k] * ((double)gwr[k] - sum_wg);
      sv_backward(tx, ux, uy, ge, gux, guy, acc, valid);
    }
    // u = (qt1 + S dt1, qt2 + S dt2)
    double g_qt1 = gux, g_qt2 = guy, g_dt1 = gux * S, g_dt2 = guy * S;
    const double g_S = gux * dt1 + guy * dt2;
    if (nzden) g_sx += g_S;
    else { g_s0 += (float)(0.5 * g_S); g_s1 += (float)(0.5 * g_S); }

    // ---------------- displaced face sx = (delta - qn)/den
    double g_qn = 0.0, g_den = 0.0;
    if (nzden) {
      const double g_delta = g_sx * idn;
      g_qn -= g_sx * idn;
      g_den -= g_sx * sxx * idn;
      double sum_w = 0.0;
      double gw[KD];
      static_assert(KD % 4 == 0 && NCELL % 4 == 0, "these wave sums go four at a time");
#pragma unroll
      for (int k = 0; k < KD; k += 4)
        sum4_to(acc, NCELL + 3 * (k + sum4_value(lane)) + 2, valid,
                (float)(g_delta * (double)wd[k]), (float)(g_delta * (double)wd[k + 1]),
                (float)(g_delta * (double)wd[k + 2]), (float)(g_delta * (double)wd[k + 3]));
#pragma unroll
      for (int k = 0; k < KD; ++k) {
        gw[k] = g_delta * (double)tx[k * TEXW + 2];
        sum_w += (double)wd[k] * gw[k];
      }
      double gubx = 0.0, guby = 0.0;
      {
        double ge[KD];
#pragma unroll
        for (int k = 0; k < KD; ++k) ge[k] = -(double)tau * (double)wd[k] * (gw[k] - sum_w);
        sv_backward(tx, ubx, uby, ge, gubx, guby, acc, valid);
      }
      // ubar = (qt1 + sbar dt1, qt2 + sbar dt2), sbar = -qn/den
      g_qt1 += gubx;
      g_qt2 += guby;
      g_dt1 += gubx * sbar;
      g_dt2 += guby * sbar;
      const double g_sbar = gubx * dt1 + guby * dt2;
      g_qn -= g_sbar * idn;
      g_den += g_sbar * qn * idn * idn;
    }

    // ---------------- frame: q.nhat, d.nhat, q.t1, d.t1, q.t2, d.t2 (float64)
    fo = s_zero[(base >> 6) & 63];
    dnx = s_fr[fo]; dny = s_fr[fo + 1]; dnz = s_fr[fo + 2];
    d1x = s_fr[fo + 3]; d1y = s_fr[fo + 4]; d1z = s_fr[fo + 5];
    d2x = s_fr[fo + 6]; d2y = s_fr[fo + 7]; d2z = s_fr[fo + 8];
    float gqx = (float)(g_qn * dnx + g_qt1 * d1x + g_qt2 * d2x);
    float gqy = (float)(g_qn * dny + g_qt1 * d1y + g_qt2 * d2y);
    float gqz = (float)(g_qn * dnz + g_qt1 * d1z + g_qt2 * d2z);
    const double gnx_h = g_qn * qdx + g_den * ddx, gny_h = g_qn * qdy + g_den * ddy, gnz_h = g_qn * qdz + g_den * ddz;
    const double g1x = g_qt1 * qdx + g_dt1 * ddx, g1y = g_qt1 * qdy + g_dt1 * ddy, g1z = g_qt1 * qdz + g_dt1 * ddz;
    const double g2x = g_qt2 * qdx + g_dt2 * ddx, g2y = g_qt2 * qdy + g_dt2 * ddy, g2z = g_qt2 * qdz + g_dt2 * ddz;
    // orthonormal basis of Duff et al. (JCGT 2017), differentiated
    const double sg = s_fr[fo + 9], oa = s_fr[fo + 10], dninv = s_fr[fo + 11];
    const double oa2 = oa * oa;
    double gnxd = gnx_h + g1x * (2.0 * sg * dnx * oa) + g1y * sg * dny * oa - g1z * sg + g2x * dny * oa;
    double gnyd = gny_h + g1y * sg * dnx * oa + g2x * dnx * oa + g2y * 2.0 * dny * oa - g2z;
    double gnzd = gnz_h + g1x * sg * dnx * dnx * oa2 + g1y * sg * dnx * dny * oa2 + g2x * dnx * dny * oa2 +
                  g2y * dny * dny * oa2;
    // nhat = n / |n|
    // normal loss: d/dnhat of lambda T a max(nhat.d, 0)^2
    if (lambda_n != 0.0f) {
      const double c = ddx * dnx + ddy * dny + ddz * dnz;
      if (c > 0.0) {
        const double gk = 2.0 * (double)lambda_n * (double)ta * c;
        gnxd += gk * ddx;
        gnyd += gk * ddy;
        gnzd += gk * ddz;
      }
    }
    const double gdot = gnxd * dnx + gnyd * dny + gnzd * dnz;
    const float gnx = (float)((gnxd - gdot * dnx) * dninv);
    const float gny = (float)((gnyd - gdot * dny) * dninv);
    const float gnz = (float)((gnzd - gdot * dnz) * dninv);

    // ---------------- ends of the bounded interval
    float g_beta = 0.0f, g_r = 0.0f, g_wi = 0.0f;
    float gpx = 0.0f, gpy = 0.0f, gpz = 0.0f;   // explicit p_i terms (planes)
    auto end_grad = [&](int b, const float4& pl, float s, float a, float ge, bool upper) {
      if (ge == 0.0f) return;
      if (b == -1) {                       // s = +-sqrt(r^2 - |q|^2)
        const float inv = frcp(sq);
        const float sgn = upper ? 1.0f : -1.0f;
        gqx -= sgn * ge * L.qx * inv;
        gqy -= sgn * ge * L.qy * inv;
        gqz -= sgn * ge * L.qz * inv;
        g_r += sgn * ge * rad * inv;
      } else if (b == -2) {                // s = beta (ray start)
        g_beta += ge;
      } else if (b < nf) {                 // s = (h - q.m)/(d.m), neighbour face
        // 1/(d.m) from the float64 direction: for a face the ray grazes, d.m
        // cancels and the float32 product loses the digits that the
        // derivatives (all proportional to 1/(d.m)) need
        const float ia = (float)rcp_d(R.dx * (double)pl.x + R.dy * (double)pl.y + R.dz * (double)pl.z);
        gqx -= ge * pl.x * ia;
        gqy -= ge * pl.y * ia;
        gqz -= ge * pl.z * ia;
        const float gmx = ge * (pl.x - L.qx - s * fx) * ia;
        const float gmy = ge * (pl.y - L.qy - s * fy) * ia;
        const float gmz = ge * (pl.z - L.qz - s * fz) * ia;
        const float gh = ge * ia;
        gpx -= gmx;
        gpy -= gmy;
        gpz -= gmz;
        g_wi += 0.5f * gh;
        if (b < FMAX_B) {
          atomicAdd(&facc[b].x, gmx);
          atomicAdd(&facc[b].y, gmy);
          atomicAdd(&facc[b].z, gmz);
          atomicAdd(&facc[b].w, -0.5f * gh);
        } else {
          const int j = col[r0 + b];
          if (j >= 0) {
            if (G.p) {
              atomicAdd(G.p + 3 * (int64_t)j, gmx);
              atomicAdd(G.p + 3 * (int64_t)j + 1, gmy);
              atomicAdd(G.p + 3 * (int64_t)j + 2, gmz);
            }
            if (G.power) atomicAdd(G.power + j, -0.5f * gh);
          }
        }
      }
    };
    if (valid) {
      end_grad(b0, pl0, s0, a0, g_s0, false);
      end_grad(b1, pl1, s1, a1, g_s1, true);
    }
    // q = oc - beta d, beta = oc.d, oc = o - p_i
    const float gqd = gqx * fx + gqy * fy + gqz * fz;
    gpx += -(gqx - gqd * fx) - g_beta * fx;
    gpy += -(gqy - gqd * fy) - g_beta * fy;
    gpz += -(gqz - gqd * fz) - g_beta * fz;

    // ---------------- per-record sums over the wave (lanes past the chunk
    // add zero)
    {
      const float cellv[NCELL] = {gpx, gpy, gpz, g_wi, g_r, gnx, gny, gnz, g_lam, gcr, gcg, gcb};
#pragma unroll
      for (int i = 0; i < NCELL; i += 4)
        sum4_to(acc, i + sum4_value(lane), valid, cellv[i], cellv[i + 1], cellv[i + 2], cellv[i + 3]);
      if (contribution) sum_to(acc, ISTAT, valid, ta);
    }

    // ---------------- Spherical-Voronoi gradients over (record, site-axis
    // pair (k, m)):
    //   v = softmax_m(a_km . d),  dL/dc_km += w_k v gC,
    //   dL/da_km += w_k v (gC.c_km - gC.sv_k) d
    // with w_k v = 2^(a_km.d log2(e) - shift) (the per-record shift in st_k)
    __builtin_amdgcn_wave_barrier();
    // rows of records past the chunk hold direction, dL/dc = 0 and an
    // infinite shift, so they add exact zeros
    typedef float f16v __attribute__((ext_vector_type(16)));
    const f16v zero16 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int ks0 = j32 >> 3, ks1 = (32 + j32) >> 3;   // sites of the lane's two columns
    for (int rb = 0; rb < 2 && 32 * rb < nvalid; ++rb) {
      // A operands: component 2 step + hh of record 32 rb + l % 32
      const float4 da = st_dir[32 * rb + j32];
      const float4 ga = st_gc[32 * rb + j32];
      const float ad0 = hh ? da.y : da.x, ad1 = hh ? 0.0f : da.z;
      const float ag0 = hh ? ga.y : ga.x, ag1 = hh ? 0.0f : ga.z;
      f16v L0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ad0, Ba[0][0], zero16, 0, 0, 0);
      L0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ad1, Ba[0][1], L0, 0, 0, 0);
      f16v L1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ad0, Ba[1][0], zero16, 0, 0, 0);
      L1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ad1, Ba[1][1], L1, 0, 0, 0);
      f16v G0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ag0, Bc[0][0], zero16, 0, 0, 0);
      G0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ag1, Bc[0][1], G0, 0, 0, 0);
      f16v G1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ag0, Bc[1][0], zero16, 0, 0, 0);
      G1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ag1, Bc[1][1], G1, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 32 * rb + 8 * (v >> 2) + 4 * hh + (v & 3);
        const float4 dd = st_dir[r];
        const float4 gc = st_gc[r];
        const float2 k0 = st_k[ks0][r], k1 = st_k[ks1][r];
        const float vw0 = __builtin_amdgcn_exp2f(L0[v] - k0.x), vw1 = __builtin_amdgcn_exp2f(L1[v] - k1.x);
        const float gl0 = vw0 * (G0[v] - k0.y), gl1 = vw1 * (G1[v] - k1.y);
        sa[0][0] += gl0 * dd.x; sa[0][1] += gl0 * dd.y; sa[0][2] += gl0 * dd.z;
        sa[1][0] += gl1 * dd.x; sa[1][1] += gl1 * dd.y; sa[1][2] += gl1 * dd.z;
        sc[0][0] += vw0 * gc.x; sc[0][1] += vw0 * gc.y; sc[0][2] += vw0 * gc.z;
        sc[1][0] += vw1 * gc.x; sc[1][1] += vw1 * gc.y; sc[1][2] += vw1 * gc.z;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // flush
  for (int t = lane; t < NSUM; t += BWD_THREADS) {
    const float v = acc[t];
    if (v == 0.0f) continue;
    float* dst = nullptr;
    if (t < 3) dst = G.p ? G.p + 3 * (int64_t)ci + t : nullptr;
    else if (t == 3) dst = G.power ? G.power + ci : nullptr;
    else if (t == 4) dst = G.radius ? G.radius + ci : nullptr;
    else if (t < 8) dst = G.normal ? G.normal + 3 * (int64_t)ci + (t - 5) : nullptr;
    else if (t == 8) dst = G.occ_logit ? G.occ_logit + ci : nullptr;
    else if (t < NCELL) dst = G.rgb ? G.rgb + 3 * (int64_t)ci + (t - 9) : nullptr;
    else {
      const int k = (t - NCELL) / 3, c = (t - NCELL) % 3;
      dst = G.tex ? G.tex + (int64_t)ci * KD * TEXW + k * TEXW + c : nullptr;
    }
    if (dst) atomicAdd(dst, v);
  }
  if (contribution && lane == 0 && acc[ISTAT] != 0.0f) atomicAdd(contribution + ci, acc[ISTAT]);
  // the two record halves of each site-axis pair: after the swap lane l
  // holds the pair km = l (cb 0 in the lower half, cb 1 in the upper)
  float va[3], vc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(sa[0][c]), __float_as_uint(sa[1][c]), false, false);
    va[c] = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(sc[0][c]), __float_as_uint(sc[1][c]), false, false);
    vc[c] = __uint_as_float(b[0]) + __uint_as_float(b[1]);
  }
  if (G.tex) {
    float* gt = G.tex + (int64_t)ci * KD * TEXW + km * TEXW;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (va[c] != 0.0f) atomicAdd(gt + 3 + 3 * mm + c, va[c]);
      if (vc[c] != 0.0f) atomicAdd(gt + 3 + 3 * MA + 3 * mm + c, vc[c]);
    }
  }
  for (int f = lane; f < nfl; f += BWD_THREADS) {
    const int j = col[r0 + f];
    if (j < 0) continue;
    const float4 v = facc[f];
    if (G.p) {
      if (v.x != 0.0f) atomicAdd(G.p + 3 * (int64_t)j, v.x);
      if (v.y != 0.0f) atomicAdd(G.p + 3 * (int64_t)j + 1, v.y);
      if (v.z != 0.0f) atomicAdd(G.p + 3 * (int64_t)j + 2, v.z);
    }
    if (G.power && v.w != 0.0f) atomicAdd(G.power + j, v.w);
  }
}

// Per-cell error statistic: sum over a cell's records of T a e (one wave per
// chunk of a cell's records, one atomic per chunk).
__global__ void __launch_bounds__(64) k_cell_err(const int4* __restrict__ chunks, const int32_t* __restrict__ order,
                                                 const float* __restrict__ rte, float* __restrict__ err) {
  const int4 ch = chunks[blockIdx.x];
  float v = 0.0f;
  for (int idx = ch.y + (int)threadIdx.x; idx < ch.z; idx += 64) v += rte[order[idx]];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (threadIdx.x == 0 && v != 0.0f) atomicAdd(err + ch.x, v);
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

int64_t backward_bytes(int64_t n, int64_t cap, bool want_err) {
  auto b = [](int64_t count, int64_t size) { return std::max<int64_t>(count, 1) * size; };
  // chunks: sum over cells of ceil(records / CHUNK) <= records / CHUNK + cells with records
  const int64_t nchunks = cap / CHUNK + std::min(n, cap) + 1;
  return (want_err ? b(cap, 4) : 0) + b(n + 1, 4) * 4 + b(n, 4) + b(cap, 4) + 2 * scan_scratch_bytes(n + 1) +
         b(nchunks, 16);
}

pf_status backward_impl(const Scene& sc, const BwdState& st, const float* d_rgba, const pf_grads& g,
                        const BwdOpts& opt, hipStream_t s) {
  const int64_t n = sc.n;
  const int64_t nrec = st.nrec;
  if (nrec == 0) return PF_OK;
  const unsigned gp = (unsigned)st.ntiles;
  const bool want_err = opt.error && opt.pixel_error;
  Buf<float> rte(s);
  // indexed like the records: slots are reserved per wave in blocks, so
  // indices run up to the pool capacity, not to the record count
  if (want_err) PF_HIP_TRY(rte.alloc(st.rec.cap));
  Buf<uint32_t> cnt(s), off(s), fill(s), nch(s), choff(s);
  Buf<int32_t> order(s);
  PF_HIP_TRY(cnt.alloc(n + 1));
  PF_HIP_TRY(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * (n + 1), s));
  {
    ProfScope ps("k_suffix", s);
    if (st.rec.wtail)   // raster records: walk the waves' segments (and count the records per cell)
      k_suffix_seg<<<gp, 256, 0, s>>>(st.rec.seg, st.rec.wtail, st.ncam, st.tile0, d_rgba, st.rec.rf, st.rec.rt,
                                      st.cams_dev,
                                      sc.nrm, opt.lambda_normal, opt.normal_loss,
                                      want_err ? opt.pixel_error : nullptr, want_err ? rte.p : nullptr, cnt.p);
    else                // ray-walk records: follow the per-pixel chains
      k_suffix<<<gp, 256, 0, s>>>(st.rec.head, st.ncam, st.tile0, d_rgba, st.rec.ri, st.rec.rf, st.rec.rt, st.cams_dev,
                                  sc.nrm,
                                  opt.lambda_normal, opt.normal_loss, want_err ? opt.pixel_error : nullptr,
                                  want_err ? rte.p : nullptr);
  }
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(off.alloc(n + 1));
  PF_HIP_TRY(fill.alloc(n));
  PF_HIP_TRY(nch.alloc(n + 1));
  PF_HIP_TRY(choff.alloc(n + 1));
  PF_HIP_TRY(order.alloc(nrec));
  PF_HIP_TRY(hipMemsetAsync(fill.p, 0, sizeof(uint32_t) * n, s));
  const unsigned gsg = (unsigned)((st.nseg + 255) / 256), gc = (unsigned)((n + 255) / 256);
  if (st.nseg && !st.rec.wtail) {   // (raster records were counted by k_suffix_seg)
    ProfScope ps("k_seg_hist", s);
    k_seg_hist<<<gsg, 256, 0, s>>>(st.rec.seg, st.nseg, cnt.p);
  }
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(exclusive_scan_u32(cnt.p, off.p, n + 1, nullptr, s));
  if (st.nseg) {
    ProfScope ps("k_seg_scatter", s);
    k_seg_scatter<<<gsg, 256, 0, s>>>(st.rec.seg, st.nseg, off.p, fill.p, order.p);
  }
  PF_HIP_TRY(hipGetLastError());
  k_chunk_count<<<gc, 256, 0, s>>>(cnt.p, n, nch.p);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(hipMemsetAsync(nch.p + n, 0, sizeof(uint32_t), s));
  PF_HIP_TRY(exclusive_scan_u32(nch.p, choff.p, n + 1, nullptr, s));
  uint32_t nchunks = 0;
  PF_HIP_TRY(hipMemcpyAsync(&nchunks, choff.p + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  Buf<int4> chunks(s);
  PF_HIP_TRY(chunks.alloc(nchunks));
  k_chunk_fill<<<gc, 256, 0, s>>>(cnt.p, off.p, choff.p, n, chunks.p);
  PF_HIP_TRY(hipGetLastError());
  if (nchunks) {
    ProfScope ps("k_bwd_cell", s);
    k_bwd_cell<<<nchunks, BWD_THREADS, 0, s>>>(st.cams_dev, st.rec.ri, st.rec.rf, order.p, chunks.p, sc.prm.p,
                                                sc.prm.radius, sc.prm.normal, sc.prm.occ_logit, sc.prm.tex, sc.row,
                                                sc.nrast, sc.col, sc.plane, sc.prm.sigma_scale, sc.prm.tau, g,
                                                st.rec.rt, opt.lambda_normal, opt.contribution);
  }
  PF_HIP_TRY(hipGetLastError());
  if (want_err && nchunks) {
    k_cell_err<<<nchunks, 64, 0, s>>>(chunks.p, order.p, rte.p, opt.error);
    PF_HIP_TRY(hipGetLastError());
  }
  return PF_OK;
}

}  // namespace pf
