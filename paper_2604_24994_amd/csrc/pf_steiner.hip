// Steiner cells for the ray walk (supplementary material, section on Steiner
// points, Alg. 1).
//
// Per round: the per-axis mean and standard deviation of the current sites
// (scene cells and the Steiner cells kept so far) turn the caller's standard
// normal draws into candidate points.  The candidates are then judged in
// order, each against the scene, the cells of earlier rounds and the cells
// kept earlier in the same round (the set grows inside the loop over the
// sample): a candidate outside every sphere takes the radius
// `|x - p_near| - r_near` to the sphere of its least-power cell (power
// `|x - p|^2 - r^2`) and is kept when that radius lies within
// [lo r_near, hi r_near].  The new cell's power weight
// `r_hat^2 - r_near^2 + w_near` puts its bisector with the nearest cell on
// that cell's sphere (`r_hat^2` when w = r^2).
//
// The in-order loop is made data-parallel in three steps:
//   k_st_eval     every candidate against the sites present at the round's
//                 start: least power and its cell.  A candidate inside a
//                 sphere there stays invalid (the set only grows).
//   k_st_conf     for each valid candidate, the earlier valid candidates
//                 that could change its verdict if kept.  A kept cell k
//                 changes candidate j only if its power at x_j is below j's
//                 round-start least power b_j, i.e. |x_j - x_k|^2 < b_j + r_k^2,
//                 and r_k <= sqrt(b_k) (the distance to the nearest sphere is
//                 at most the square root of the power there), so the pairs
//                 with |x_j - x_k|^2 < b_j + b_k (widened for rounding) are
//                 listed; every other earlier cell leaves j's least power
//                 and nearest cell as they are.
//   k_st_resolve  launched until every valid candidate is decided: a
//                 candidate is decided once all of its listed candidates were
//                 decided in an earlier launch, by folding the kept ones into
//                 its round-start least power in candidate order (strict
//                 improvement: ties keep the lower index, scene cells first).
// Every decision is the one the in-order loop takes.
//
// Layout: the sites of a round are Morton-sorted into an implicit 64-ary tree
// (per node: box and largest radius); one wave per candidate walks it depth
// first, children in increasing order of their power lower bound
// `dist(x, box)^2 - r_max^2`, 64 children or sites per step.  Powers and
// radii are formed in float64 from the float32 values without contraction,
// so every decision is the one the float64 definition takes.
#include "pf_internal.hpp"

#include <algorithm>
#include <climits>
#include <vector>

namespace pf {

namespace {

constexpr int ST_THREADS = 256;
constexpr int ST_BLOCKS = 512;            // fixed, so the statistics' summation order is fixed
constexpr int ST_STACK = 64 * MAXLVL;     // depth-first stack bound: 64 entries per level

template <typename T>
struct Tmp {
  T* p = nullptr;
  hipStream_t s;
  explicit Tmp(hipStream_t st) : s(st) {}
  ~Tmp() { if (p) pf::pool_free(p, s); }
  hipError_t alloc(size_t count) { return pf::pool_alloc((void**)&p, sizeof(T) * (count ? count : 1), s); }
};

__device__ inline uint32_t spread10_s(uint32_t v) {
  v &= 0x3FF;
  v = (v | (v << 16)) & 0x030000FF;
  v = (v | (v << 8)) & 0x0300F00F;
  v = (v | (v << 4)) & 0x030C30C3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}

// Block sums (float64) of x, y, z and box (float) over the m sites, for
// stat = {mean[3], std[3], box_lo[3], box_hi[3]}.  pass 0: sums of
// coordinates and the box; pass 1: sums of squared deviations from the mean.
__global__ void __launch_bounds__(ST_THREADS) k_st_partial(const float* __restrict__ up, int64_t m, int pass,
                                                           const double* __restrict__ stat,
                                                           double* __restrict__ part) {
#pragma clang fp contract(off)
  double s[3] = {0.0, 0.0, 0.0};
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double mu[3] = {0.0, 0.0, 0.0};
  if (pass == 1)
    for (int a = 0; a < 3; ++a) mu[a] = stat[a];
  for (int64_t i = (int64_t)blockIdx.x * ST_THREADS + threadIdx.x; i < m; i += (int64_t)ST_BLOCKS * ST_THREADS) {
    for (int a = 0; a < 3; ++a) {
      const float v = up[3 * i + a];
      if (pass == 0) {
        s[a] += (double)v;
        lo[a] = fminf(lo[a], v);
        hi[a] = fmaxf(hi[a], v);
      } else {
        const double d = (double)v - mu[a];
        s[a] += d * d;
      }
    }
  }
  __shared__ double red[9][ST_THREADS];
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = s[a];
    red[3 + a][threadIdx.x] = lo[a];
    red[6 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int w = ST_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] += red[a][threadIdx.x + w];
        red[3 + a][threadIdx.x] = fmin(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + w]);
        red[6 + a][threadIdx.x] = fmax(red[6 + a][threadIdx.x], red[6 + a][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 9) part[blockIdx.x * 9 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(ST_THREADS) k_st_final(const double* __restrict__ part, int64_t m, int pass,
                                                         double* __restrict__ stat) {
#pragma clang fp contract(off)
  __shared__ double red[9][ST_BLOCKS];
  for (int b = threadIdx.x; b < ST_BLOCKS; b += ST_THREADS)
    for (int q = 0; q < 9; ++q) red[q][b] = part[b * 9 + q];
  __syncthreads();
  for (int w = ST_BLOCKS / 2; w > 0; w >>= 1) {
    for (int b = threadIdx.x; b < w; b += ST_THREADS)
      for (int a = 0; a < 3; ++a) {
        red[a][b] += red[a][b + w];
        red[3 + a][b] = fmin(red[3 + a][b], red[3 + a][b + w]);
        red[6 + a][b] = fmax(red[6 + a][b], red[6 + a][b + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    if (pass == 0) {
      stat[a] = red[a][0] / (double)m;
      stat[6 + a] = red[3 + a][0];
      stat[9 + a] = red[6 + a][0];
    } else {
      stat[3 + a] = sqrt(red[a][0] / (double)m);
    }
  }
}

__global__ void k_st_morton(const float* __restrict__ up, int64_t m, const double* __restrict__ stat,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    const double lo = stat[6 + a], ext = stat[9 + a] - lo;
    const double t = ext > 0.0 ? ((double)up[3 * i + a] - lo) * (1024.0 / ext) : 0.0;
    q[a] = (uint32_t)fmin(fmax(t, 0.0), 1023.0);
  }
  keys[i] = spread10_s(q[0]) | (spread10_s(q[1]) << 1) | (spread10_s(q[2]) << 2);
  vals[i] = (uint32_t)i;
}

__global__ void k_st_gather(const float* __restrict__ up, const float* __restrict__ ur,
                            const uint32_t* __restrict__ order, int64_t m, float4* __restrict__ sp,
                            int32_t* __restrict__ sidx) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t i = order[k];
  sp[k] = make_float4(up[3 * i], up[3 * i + 1], up[3 * i + 2], ur[i]);
  sidx[k] = (int32_t)i;
}

// One wave per parent node: box and largest radius of up to 64 children.
__global__ void __launch_bounds__(64) k_st_level(const float4* __restrict__ sp, const float4* __restrict__ clo,
                                                 const float4* __restrict__ chi, int64_t nchild,
                                                 float4* __restrict__ olo, float4* __restrict__ ohi) {
  const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, rmax = 0.0f;
  if (c < nchild) {
    if (sp) {
      const float4 s = sp[c];
      lo[0] = hi[0] = s.x;
      lo[1] = hi[1] = s.y;
      lo[2] = hi[2] = s.z;
      rmax = s.w;
    } else {
      const float4 a = clo[c], b = chi[c];
      lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
      hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
      rmax = b.w;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
    rmax = fmaxf(rmax, __shfl_xor(rmax, o, 64));
  }
  if (threadIdx.x == 0) {
    olo[blockIdx.x] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    ohi[blockIdx.x] = make_float4(hi[0], hi[1], hi[2], rmax);
  }
}

__device__ inline double slack(double best) { return 1e-9 * (1.0 + fabs(best)); }

// One wave per candidate: least power over the round-start sites and its
// cell (ties: lower index).
__global__ void __launch_bounds__(64) k_st_eval(const float* __restrict__ z, int64_t n_cand,
                                                 const double* __restrict__ stat, const float4* __restrict__ sp,
                                                 const int32_t* __restrict__ sidx, int64_t m,
                                                 const float4* __restrict__ nlo, const float4* __restrict__ nhi,
                                                 Levels lv,
                                                 uint32_t* __restrict__ vflag, float4* __restrict__ cx,
                                                 double* __restrict__ cbest, int32_t* __restrict__ cnear,
                                                 unsigned int* __restrict__ overflow) {
#pragma clang fp contract(off)
  __shared__ int stk[ST_STACK];
  __shared__ double skey[ST_STACK];
  __shared__ double lbs[64];
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  // the candidate, rounded to the float32 site it would become
  float xf[3];
  for (int a = 0; a < 3; ++a) {
    const double t = stat[3 + a] * (double)z[3 * j + a];
    xf[a] = __double2float_rn(stat[a] + t);
  }
  const double x = xf[0], y = xf[1], zc = xf[2];
  double best = INFINITY;
  int bi = INT_MAX;
  int top = 1;
  if (lane == 0) {
    stk[0] = lv.n << 24;
    skey[0] = -INFINITY;
  }
  __syncthreads();
  while (top > 0) {
    --top;
    const int ent = stk[top];
    const double key = skey[top];
    __syncthreads();
    if (key > best + slack(best)) continue;
    const int L = ent >> 24;
    const long long idx = ent & 0xFFFFFF;
    if (L == 1) {
      const int64_t s = idx * 64 + lane;
      double pw = INFINITY;
      int id = INT_MAX;
      if (s < m) {
        const float4 q = sp[s];
        const double dx = x - (double)q.x, dy = y - (double)q.y, dz = zc - (double)q.z;
        const double rr = (double)q.w * (double)q.w;
        pw = ((dx * dx + dy * dy) + dz * dz) - rr;
        id = sidx[s];
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double p2 = __shfl_xor(pw, o, 64);
        const int i2 = __shfl_xor(id, o, 64);
        if (p2 < pw || (p2 == pw && i2 < id)) {
          pw = p2;
          id = i2;
        }
      }
      if (pw < best || (pw == best && id < bi)) {
        best = pw;
        bi = id;
      }
      continue;
    }
    const long long c = idx * 64 + lane;
    double lb = INFINITY;
    bool keep = false;
    if (c < lv.cnt[L - 1]) {
      const float4 a = nlo[lv.off[L - 1] + c], b = nhi[lv.off[L - 1] + c];
      const double ex = fmax(0.0, fmax((double)a.x - x, x - (double)b.x));
      const double ey = fmax(0.0, fmax((double)a.y - y, y - (double)b.y));
      const double ez = fmax(0.0, fmax((double)a.z - zc, zc - (double)b.z));
      lb = ((ex * ex + ey * ey) + ez * ez) - (double)b.w * (double)b.w;
      keep = lb <= best + slack(best);
    }
    lbs[lane] = lb;
    __syncthreads();
    const uint64_t mk = __ballot(keep);
    const int nk = __popcll(mk);
    if (top + nk > ST_STACK) {
      if (lane == 0) atomicAdd(overflow, 1u);
      break;
    }
    if (keep) {
      // larger bounds deeper in the stack: the least bound is taken first
      int rank = 0;
      for (int k = 0; k < 64; ++k) {
        if (!((mk >> k) & 1ull)) continue;
        const double o = lbs[k];
        rank += (o > lb || (o == lb && k < lane)) ? 1 : 0;
      }
      stk[top + rank] = ((L - 1) << 24) | (int)c;
      skey[top + rank] = lb;
    }
    top += nk;
    __syncthreads();
  }
  if (lane != 0) return;
  const bool valid = best > 0.0 && bi != INT_MAX;
  vflag[j] = valid ? 1u : 0u;
  cx[j] = make_float4(xf[0], xf[1], xf[2], 0.0f);
  cbest[j] = best;
  cnear[j] = valid ? bi : -1;
}

// Valid candidates, in candidate order, with their round-start least power,
// its cell and the widened square of the largest radius they can take.
__global__ void k_st_compact(const uint32_t* __restrict__ vflag, const uint32_t* __restrict__ vpos, int64_t n_cand,
                             const float4* __restrict__ cx, const double* __restrict__ cbest,
                             const int32_t* __restrict__ cnear, float4* __restrict__ vx, double* __restrict__ vb,
                             double* __restrict__ vrho, int32_t* __restrict__ vnear) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_cand || !vflag[j]) return;
  const uint32_t v = vpos[j];
  const float4 x = cx[j];
  const double b = cbest[j];
  vx[v] = x;
  vb[v] = b;
  // r_hat = b / (|x - p| + r) <= sqrt(b); the float64 and float32 roundings
  // of the kept radius are covered by the relative and absolute widening
  const double ax = fmax(fabs((double)x.x), fmax(fabs((double)x.y), fabs((double)x.z)));
  const double r = sqrt(b) * (1.0 + 1e-6) + 1e-7 * (1.0 + ax);
  vrho[v] = r * r;
  vnear[v] = cnear[j];
}

constexpr int CF_THREADS = 256;
constexpr int RES_OPEN = 0x7F7F7F7F;   // k_st_resolve: not decided yet (the byte fill 0x7F)

// Earlier valid candidates that can change candidate v's verdict (FILL =
// false: their count; true: their indices, in increasing order).
template <bool FILL>
__global__ void __launch_bounds__(CF_THREADS) k_st_conf(const float4* __restrict__ vx, const double* __restrict__ vb,
                                                         const double* __restrict__ vrho, int64_t nv,
                                                         uint32_t* __restrict__ cnt, const uint32_t* __restrict__ off,
                                                         int32_t* __restrict__ list,
                                                         unsigned long long* __restrict__ total) {
  __shared__ float4 sx[CF_THREADS];
  __shared__ double sr[CF_THREADS];
  const int64_t v = (int64_t)blockIdx.x * CF_THREADS + threadIdx.x;
  const int64_t vmax = min(nv - 1, (int64_t)blockIdx.x * CF_THREADS + CF_THREADS - 1);
  float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  double bj = 0.0;
  if (v < nv) {
    x = vx[v];
    bj = vb[v];
  }
  uint32_t c = 0;
  uint32_t o = (FILL && v < nv) ? off[v] : 0u;
  for (int64_t t0 = 0; t0 < vmax; t0 += CF_THREADS) {
    __syncthreads();
    const int64_t k = t0 + threadIdx.x;
    if (k < nv) {
      sx[threadIdx.x] = vx[k];
      sr[threadIdx.x] = vrho[k];
    }
    __syncthreads();
    if (v < nv) {
      const int kend = (int)min((int64_t)CF_THREADS, v - t0);
      for (int q = 0; q < kend; ++q) {
        const float4 y = sx[q];
        const double dx = (double)x.x - (double)y.x, dy = (double)x.y - (double)y.y, dz = (double)x.z - (double)y.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < (bj + sr[q]) * (1.0 + 1e-12)) {
          if (FILL) list[o + c] = (int32_t)(t0 + q);
          ++c;
        }
      }
    }
  }
  if (!FILL) {
    if (v < nv) cnt[v] = c;
    unsigned long long t = c;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(total, t);
  }
}

// One launch of the in-order resolution (see the file header).  it: the
// launch's number; res[v] the launch that decided v (RES_OPEN: not yet).
// tag[v] >= 0: the nearest cell is site tag[v] of the round-start set;
// tag[v] < 0: it is the valid candidate -1 - tag[v] of this round.
__global__ void k_st_resolve(const float4* __restrict__ vx, const double* __restrict__ vb,
                             const int32_t* __restrict__ vnear, int64_t nv, const uint32_t* __restrict__ off,
                             const int32_t* __restrict__ list, const float* __restrict__ up,
                             const float* __restrict__ ur, const float* __restrict__ uw, double lo_ratio,
                             double hi_ratio, int it, int32_t* __restrict__ res, uint32_t* __restrict__ kept,
                             float* __restrict__ vr, float* __restrict__ vw, int32_t* __restrict__ tag,
                             unsigned int* __restrict__ done) {
#pragma clang fp contract(off)
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv || res[v] != RES_OPEN) return;
  const uint32_t c0 = off[v], c1 = off[v + 1];
  for (uint32_t c = c0; c < c1; ++c)
    if (res[list[c]] >= it) return;   // an earlier candidate is still open
  const float4 x = vx[v];
  const double xx = x.x, xy = x.y, xz = x.z;
  double best = vb[v];
  int t = vnear[v];
  double npx = up[3 * (int64_t)t], npy = up[3 * (int64_t)t + 1], npz = up[3 * (int64_t)t + 2];
  double nr = ur[t], nw = uw[t];
  for (uint32_t c = c0; c < c1; ++c) {
    const int k = list[c];
    if (!kept[k]) continue;
    const float4 y = vx[k];
    const double rk = vr[k];
    const double dx = xx - (double)y.x, dy = xy - (double)y.y, dz = xz - (double)y.z;
    const double pw = ((dx * dx + dy * dy) + dz * dz) - rk * rk;
    if (pw < best) {
      best = pw;
      t = -1 - k;
      npx = y.x; npy = y.y; npz = y.z;
      nr = rk;
      nw = vw[k];
    }
  }
  uint32_t ok = 0;
  float rh_f = 0.0f, wh_f = 0.0f;
  if (best > 0.0) {
    const double dx = xx - npx, dy = xy - npy, dz = xz - npz;
    const double d = sqrt((dx * dx + dy * dy) + dz * dz);
    const double rh = d - nr;
    ok = (lo_ratio * nr <= rh && rh <= hi_ratio * nr) ? 1u : 0u;
    rh_f = __double2float_rn(rh);
    wh_f = __double2float_rn((rh * rh - nr * nr) + nw);
  }
  kept[v] = ok;
  vr[v] = rh_f;
  vw[v] = wh_f;
  tag[v] = t;
  res[v] = it;
  atomicAdd(done, 1u);
}

// Kept candidates, in candidate order, to the caller's outputs (from `a`)
// and to the site set (from `m`).
__global__ void k_st_emit(const uint32_t* __restrict__ kept, const uint32_t* __restrict__ kpos, int64_t nv,
                          const float4* __restrict__ vx, const float* __restrict__ vr, const float* __restrict__ vw,
                          const int32_t* __restrict__ tag, int64_t a, int64_t m, int64_t cap,
                          float* __restrict__ out_p, float* __restrict__ out_w, float* __restrict__ out_r,
                          int32_t* __restrict__ out_near, float* __restrict__ up, float* __restrict__ ur,
                          float* __restrict__ uw) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv || !kept[v]) return;
  const int64_t k = kpos[v];
  if (a + k >= cap) return;
  const float4 c = vx[v];
  const int64_t o = a + k, u = m + k;
  out_p[3 * o] = c.x;
  out_p[3 * o + 1] = c.y;
  out_p[3 * o + 2] = c.z;
  out_r[o] = vr[v];
  out_w[o] = vw[v];
  const int t = tag[v];
  if (out_near) out_near[o] = t >= 0 ? t : (int32_t)(m + kpos[-1 - t]);
  up[3 * u] = c.x;
  up[3 * u + 1] = c.y;
  up[3 * u + 2] = c.z;
  ur[u] = vr[v];
  uw[u] = vw[v];
}

Levels levels_for(int64_t count, long long* total_nodes) {
  Levels lv{};
  lv.cnt[0] = count;
  long long tot = 0;
  int L = 0;
  do {
    ++L;
    lv.cnt[L] = (lv.cnt[L - 1] + 63) / 64;
    lv.off[L] = tot;
    tot += lv.cnt[L];
  } while (lv.cnt[L] > 1 && L < MAXLVL);
  lv.n = L;
  *total_nodes = tot;
  return lv;
}

}  // namespace

pf_status steiner_impl(const pf_params& prm, const float* z, const pf_steiner_opts& opt, int64_t cap, float* out_p,
                       float* out_power, float* out_radius, int32_t* out_near, int64_t* round_counts,
                       int64_t* n_out, hipStream_t s) {
  const int64_t n = prm.n, total = n + cap;
  Tmp<float> up(s), ur(s), uw(s);
  PF_HIP_TRY(up.alloc(3 * total));
  PF_HIP_TRY(ur.alloc(total));
  PF_HIP_TRY(uw.alloc(total));
  PF_HIP_TRY(hipMemcpyAsync(up.p, prm.p, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, s));
  PF_HIP_TRY(hipMemcpyAsync(ur.p, prm.radius, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  PF_HIP_TRY(hipMemcpyAsync(uw.p, prm.power, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  long long max_nodes = 0;
  const Levels lv_max = levels_for(total, &max_nodes);
  if (lv_max.cnt[lv_max.n] != 1) {
    set_error("pf_steiner: too many sites for the search tree");
    return PF_ERR_UNSUPPORTED;
  }
  const int64_t nc = opt.n_cand;
  Tmp<double> stat(s), part(s), cbest(s), vb(s), vrho(s);
  Tmp<uint32_t> keys(s), order(s), vflag(s), vpos(s), tot(s), ccnt(s), coff(s), kept(s), kpos(s);
  Tmp<float4> sp(s), nlo(s), nhi(s), cx(s), vx(s);
  Tmp<int32_t> sidx(s), cnear(s), vnear(s), res(s), tag(s);
  Tmp<float> vr(s), vw(s);
  Tmp<unsigned int> ovf(s), done(s);
  Tmp<unsigned long long> ctot(s);
  PF_HIP_TRY(stat.alloc(12));
  PF_HIP_TRY(part.alloc(9 * ST_BLOCKS));
  PF_HIP_TRY(keys.alloc(total));
  PF_HIP_TRY(order.alloc(total));
  PF_HIP_TRY(sp.alloc(total));
  PF_HIP_TRY(sidx.alloc(total));
  PF_HIP_TRY(nlo.alloc(max_nodes));
  PF_HIP_TRY(nhi.alloc(max_nodes));
  PF_HIP_TRY(vflag.alloc(nc));
  PF_HIP_TRY(vpos.alloc(nc));
  PF_HIP_TRY(tot.alloc(2));
  PF_HIP_TRY(cx.alloc(nc));
  PF_HIP_TRY(cbest.alloc(nc));
  PF_HIP_TRY(cnear.alloc(nc));
  PF_HIP_TRY(vx.alloc(nc));
  PF_HIP_TRY(vb.alloc(nc));
  PF_HIP_TRY(vrho.alloc(nc));
  PF_HIP_TRY(vnear.alloc(nc));
  PF_HIP_TRY(ccnt.alloc(nc + 1));
  PF_HIP_TRY(coff.alloc(nc + 1));
  PF_HIP_TRY(res.alloc(nc));
  PF_HIP_TRY(kept.alloc(nc));
  PF_HIP_TRY(kpos.alloc(nc));
  PF_HIP_TRY(tag.alloc(nc));
  PF_HIP_TRY(vr.alloc(nc));
  PF_HIP_TRY(vw.alloc(nc));
  PF_HIP_TRY(ovf.alloc(1));
  PF_HIP_TRY(done.alloc(1));
  PF_HIP_TRY(ctot.alloc(1));
  PF_HIP_TRY(hipMemsetAsync(ovf.p, 0, sizeof(unsigned int), s));

  int64_t a = 0;
  bool full = false;
  for (int r = 0; r < opt.rounds; ++r) {
    const int64_t m = n + a;
    const unsigned gm = (unsigned)((m + 255) / 256);
    {
      ProfScope ps("k_st_stats", s);
      for (int pass = 0; pass < 2; ++pass) {
        k_st_partial<<<ST_BLOCKS, ST_THREADS, 0, s>>>(up.p, m, pass, stat.p, part.p);
        k_st_final<<<1, ST_THREADS, 0, s>>>(part.p, m, pass, stat.p);
      }
    }
    PF_HIP_TRY(hipGetLastError());
    k_st_morton<<<gm, 256, 0, s>>>(up.p, m, stat.p, keys.p, order.p);
    PF_HIP_TRY(hipGetLastError());
    PF_HIP_TRY(radix_sort_u32(keys.p, order.p, m, 30, s));
    k_st_gather<<<gm, 256, 0, s>>>(up.p, ur.p, order.p, m, sp.p, sidx.p);
    PF_HIP_TRY(hipGetLastError());
    long long nodes = 0;
    const Levels lv = levels_for(m, &nodes);
    for (int l = 1; l <= lv.n; ++l) {
      k_st_level<<<(unsigned)lv.cnt[l], 64, 0, s>>>(l == 1 ? sp.p : nullptr, l == 1 ? nullptr : nlo.p + lv.off[l - 1],
                                                     l == 1 ? nullptr : nhi.p + lv.off[l - 1], lv.cnt[l - 1],
                                                     nlo.p + lv.off[l], nhi.p + lv.off[l]);
      PF_HIP_TRY(hipGetLastError());
    }
    {
      ProfScope ps("k_st_eval", s);
      k_st_eval<<<(unsigned)nc, 64, 0, s>>>(z + 3 * nc * (int64_t)r, nc, stat.p, sp.p, sidx.p, m, nlo.p, nhi.p, lv,
                                            vflag.p, cx.p, cbest.p, cnear.p, ovf.p);
    }
    PF_HIP_TRY(hipGetLastError());
    // valid candidates, in candidate order
    PF_HIP_TRY(exclusive_scan_u32(vflag.p, vpos.p, nc, tot.p, s));
    const unsigned gc = (unsigned)((nc + 255) / 256);
    k_st_compact<<<gc, 256, 0, s>>>(vflag.p, vpos.p, nc, cx.p, cbest.p, cnear.p, vx.p, vb.p, vrho.p, vnear.p);
    PF_HIP_TRY(hipGetLastError());
    uint32_t nv = 0;
    unsigned int over = 0;
    PF_HIP_TRY(hipMemcpyAsync(&nv, tot.p, sizeof(nv), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipMemcpyAsync(&over, ovf.p, sizeof(over), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    if (over) {
      set_error("pf_steiner: search stack exceeded");
      return PF_ERR_OVERFLOW;
    }
    uint32_t nkept = 0;
    if (nv > 0) {
      // the earlier candidates each valid one must wait for
      const unsigned gv = (unsigned)((nv + CF_THREADS - 1) / CF_THREADS);
      PF_HIP_TRY(hipMemsetAsync(ctot.p, 0, sizeof(unsigned long long), s));
      {
        ProfScope ps("k_st_conf", s);
        k_st_conf<false><<<gv, CF_THREADS, 0, s>>>(vx.p, vb.p, vrho.p, nv, ccnt.p, nullptr, nullptr, ctot.p);
      }
      PF_HIP_TRY(hipGetLastError());
      unsigned long long nconf64 = 0;
      PF_HIP_TRY(hipMemcpyAsync(&nconf64, ctot.p, sizeof(nconf64), hipMemcpyDeviceToHost, s));
      PF_HIP_TRY(hipStreamSynchronize(s));
      if (nconf64 >= (1ull << 31)) {
        set_error("pf_steiner: more than 2^31 candidate pairs to resolve in one round; draw fewer candidates");
        return PF_ERR_OVERFLOW;
      }
      PF_HIP_TRY(hipMemsetAsync(ccnt.p + nv, 0, sizeof(uint32_t), s));
      PF_HIP_TRY(exclusive_scan_u32(ccnt.p, coff.p, (int64_t)nv + 1, tot.p + 1, s));
      uint32_t nconf = 0;
      PF_HIP_TRY(hipMemcpyAsync(&nconf, tot.p + 1, sizeof(nconf), hipMemcpyDeviceToHost, s));
      PF_HIP_TRY(hipStreamSynchronize(s));
      Tmp<int32_t> clist(s);
      PF_HIP_TRY(clist.alloc(nconf));
      {
        ProfScope ps("k_st_conf", s);
        k_st_conf<true><<<gv, CF_THREADS, 0, s>>>(vx.p, vb.p, vrho.p, nv, nullptr, coff.p, clist.p, nullptr);
      }
      PF_HIP_TRY(hipGetLastError());
      // in-order decisions: every launch decides at least the earliest open
      // candidate, so at most nv launches
      PF_HIP_TRY(hipMemsetAsync(res.p, 0x7F, sizeof(int32_t) * nv, s));   // RES_OPEN, above any launch number
      PF_HIP_TRY(hipMemsetAsync(done.p, 0, sizeof(unsigned int), s));
      const unsigned gr = (unsigned)((nv + 255) / 256);
      int it = 0, batch = 4;   // launches between checks, doubled up to 64 (extra launches find nothing open)
      for (;;) {
        {
          ProfScope ps("k_st_resolve", s);
          for (int q = 0; q < batch; ++q, ++it)
            k_st_resolve<<<gr, 256, 0, s>>>(vx.p, vb.p, vnear.p, nv, coff.p, clist.p, up.p, ur.p, uw.p,
                                            (double)opt.lo_ratio, (double)opt.hi_ratio, it, res.p, kept.p, vr.p,
                                            vw.p, tag.p, done.p);
        }
        PF_HIP_TRY(hipGetLastError());
        unsigned int nd = 0;
        PF_HIP_TRY(hipMemcpyAsync(&nd, done.p, sizeof(nd), hipMemcpyDeviceToHost, s));
        PF_HIP_TRY(hipStreamSynchronize(s));
        if (nd >= nv) break;
        batch = std::min(2 * batch, 64);
        if (it > (int)nv + 4) {
          set_error("pf_steiner: in-order resolution did not finish");
          return PF_ERR_HIP;
        }
      }
      PF_HIP_TRY(exclusive_scan_u32(kept.p, kpos.p, nv, tot.p, s));
      k_st_emit<<<gr, 256, 0, s>>>(kept.p, kpos.p, nv, vx.p, vr.p, vw.p, tag.p, a, m, cap, out_p, out_power,
                                   out_radius, out_near, up.p, ur.p, uw.p);
      PF_HIP_TRY(hipGetLastError());
      PF_HIP_TRY(hipMemcpyAsync(&nkept, tot.p, sizeof(nkept), hipMemcpyDeviceToHost, s));
      PF_HIP_TRY(hipStreamSynchronize(s));
    }
    const int64_t kept_r = nkept;
    if (round_counts) round_counts[r] = kept_r;
    if (a + kept_r > cap) {
      a = cap;
      full = true;
      break;
    }
    a += kept_r;
  }
  *n_out = a;
  if (full) {
    set_error("pf_steiner: more cells kept than the output capacity " + std::to_string(cap) +
              " (rounds * n_cand always suffices)");
    return PF_ERR_OVERFLOW;
  }
  return PF_OK;
}

}  // namespace pf
