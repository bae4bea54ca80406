// Scene build: face adjacency of the power diagram clipped to the domain
// box, tight cull radii and hidden-cell flags.
//
// What is computed: for every cell i the faces of
//   Pi_i = { x : |x-p_i|^2 - w_i <= |x-p_j|^2 - w_j }  (appendix B)
// inside the domain box; these are the regular-triangulation edges the ray
// walk crosses (appendix C).  Faces whose plane lies within r_i of p_i are
// listed first: only they can cut the bounded cell Pi_i n B(p_i, r_i) that
// the rasteriser composites (Sec. 3.2).
//
// How (gfx950): sites are Morton-sorted and grouped into an implicit 64-ary
// tree (leaves of 64 consecutive sites; each node keeps an AABB and the
// largest weight below it).  One wave64 owns one cell and holds its convex
// polytope in registers as up to 128 vertices, two per lane, each vertex the
// intersection of three planes with positive orientation det(m_a,m_b,m_c).
// Clipping by a plane removes the vertices beyond it and re-triangulates the
// cavity: every edge (a,b) from a removed vertex to a kept one yields the new
// vertex (a,b,k).  An LDS table maps directed edges to vertex slots.
// Candidates come nearest-first from the cell's own leaf, then from a tree
// walk that prunes a node when no site in its box can be closer in power
// than p_i to any current vertex:  dist(v,box)^2 - maxw >= |v-p_i|^2 - w_i.
// Everything in the clipper is float64 in cell-local coordinates (FP64 runs
// at the unpacked FP32 rate on CDNA).
#include "pf_internal.hpp"

#include <type_traits>
#include <vector>

namespace pf {
namespace {

constexpr int PM_MID = 128;       // plane capacity of the second pass (edge table in LDS)
constexpr int SPL_MID = 4;        // vertex slots per lane of the second pass
constexpr int PM_BIG = 256;       // plane capacity of the third pass (edge table in HBM)
constexpr int SPL_BIG = 8;        // vertex slots per lane of the third pass
// traversal stack: the unvisited siblings along one root-to-leaf path,
// (levels - 2) x 63 + 64 + the root's children: 190 entries at 16M sites
constexpr int STACK = 192;
constexpr int WIT = 8;           // per empty cell: sites whose planes emptied it (seeds of the next build)
constexpr int RING_K = 16;        // rank of the leaf mate that sets the first ring radius
// Upper bound on candidate clips plus node visits per cell; a cell that
// reaches it is reported as over capacity instead of running on.
constexpr int WORK_LIMIT = 1 << 22;


__device__ inline uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline float wave_min(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ inline float wave_max(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}
// Wave-wide reductions of a double with DPP moves (all 64 lanes active):
// butterflies within rows of 16 lanes, then the row broadcasts of lanes 15
// and 31 leave the result in lane 63, which is read back to every lane.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_d(double x, double old) {
  const long long xb = __double_as_longlong(x), ob = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)ob, (int)xb, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(ob >> 32), (int)(xb >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double lane63_d(double x) {
  const long long xb = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)xb, 63), hi = __builtin_amdgcn_readlane((int)(xb >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_max_d(double x) {
  x = fmax(x, dpp_d<0xB1, 0xf>(x, -INFINITY));    // quad perm [1,0,3,2]
  x = fmax(x, dpp_d<0x4E, 0xf>(x, -INFINITY));    // quad perm [2,3,0,1]
  x = fmax(x, dpp_d<0x141, 0xf>(x, -INFINITY));   // row half mirror
  x = fmax(x, dpp_d<0x140, 0xf>(x, -INFINITY));   // row mirror
  x = fmax(x, dpp_d<0x142, 0xa>(x, -INFINITY));   // row bcast 15
  x = fmax(x, dpp_d<0x143, 0xc>(x, -INFINITY));   // row bcast 31
  return lane63_d(x);
}
__device__ inline double wave_sum_d(double x) {
  x += dpp_d<0xB1, 0xf>(x, 0.0);
  x += dpp_d<0x4E, 0xf>(x, 0.0);
  x += dpp_d<0x141, 0xf>(x, 0.0);
  x += dpp_d<0x140, 0xf>(x, 0.0);
  x += dpp_d<0x142, 0xa>(x, 0.0);
  x += dpp_d<0x143, 0xc>(x, 0.0);
  return lane63_d(x);
}

// Per-block partial bounds of the spheres and weights:
// [minx,miny,minz,maxx,maxy,maxz,maxw,minr] per block.
__global__ void __launch_bounds__(256) k_bounds(const float* __restrict__ p, const float* __restrict__ w,
                                                const float* __restrict__ r, int64_t n,
                                                float* __restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float wmax = -INFINITY, rmin = INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float ri = r[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float c = p[3 * i + a];
      lo[a] = fminf(lo[a], c - ri);
      hi[a] = fmaxf(hi[a], c + ri);
    }
    wmax = fmaxf(wmax, w[i]);
    rmin = fminf(rmin, ri);
  }
  __shared__ float red[4][8];
  float v[8] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], wmax, rmin};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    bool is_min = (q < 3) || (q == 7);
    v[q] = is_min ? wave_min(v[q]) : wave_max(v[q]);
    if (lane == 0) red[wv][q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    int q = threadIdx.x;
    bool is_min = (q < 3) || (q == 7);
    float a = red[0][q];
    for (int k = 1; k < 4; ++k) a = is_min ? fminf(a, red[k][q]) : fmaxf(a, red[k][q]);
    part[blockIdx.x * 8 + q] = a;
  }
}

__global__ void k_morton(const float* __restrict__ p, int64_t n, float3 lo, float3 inv,
                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
  float l[3] = {lo.x, lo.y, lo.z}, s[3] = {inv.x, inv.y, inv.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float t = (p[3 * i + a] - l[a]) * s[a];
    t = fminf(fmaxf(t, 0.0f), 1023.0f);
    q[a] = (uint32_t)t;
  }
  keys[i] = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
  vals[i] = (uint32_t)i;
}

__global__ void k_gather_sites(const float* __restrict__ p, const float* __restrict__ w,
                               const float* __restrict__ r, const uint32_t* __restrict__ order, int64_t n,
                               float4* __restrict__ sp, int32_t* __restrict__ sidx, float* __restrict__ srad) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t i = order[k];
  sp[k] = make_float4(p[3 * i], p[3 * i + 1], p[3 * i + 2], w[i]);
  sidx[k] = (int32_t)i;
  srad[k] = r[i];
}

// One wave per parent node: AABB and max weight of up to 64 children.
__global__ void __launch_bounds__(64) k_tree_level(const float4* __restrict__ sp, const float* __restrict__ srad,
                                                   const float4* __restrict__ clo, const float4* __restrict__ chi,
                                                   int64_t nchild, float4* __restrict__ olo,
                                                   float4* __restrict__ ohi) {
  const int lane = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, w = -INFINITY;
  float rmax = 0.0f;
  if (c < nchild) {
    if (sp) {
      float4 s = sp[c];
      lo[0] = hi[0] = s.x;
      lo[1] = hi[1] = s.y;
      lo[2] = hi[2] = s.z;
      w = s.w;
      rmax = srad[c];
    } else {
      float4 a = clo[c], b = chi[c];
      lo[0] = a.x; lo[1] = a.y; lo[2] = a.z; w = a.w;
      hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
      rmax = b.w;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min(lo[a]);
    hi[a] = wave_max(hi[a]);
  }
  w = wave_max(w);
  rmax = wave_max(rmax);
  if (lane == 0) {
    olo[blockIdx.x] = make_float4(lo[0], lo[1], lo[2], w);
    ohi[blockIdx.x] = make_float4(hi[0], hi[1], hi[2], rmax);
  }
}

// ---------------------------------------------------------------------------
// Clipper of one cell, run by one wave.  SPL vertex slots per lane (64*SPL
// vertices), PM plane capacity; the directed-edge -> vertex-slot table has
// PM*PM entries of type EOT and lives in LDS (small variant) or in a per-cell
// HBM workspace (large variant, for the few cells of very high degree).

template <int SPL, int PM>
struct Shared {
  double pl[PM][4];               // planes (m.x, m.y, m.z, h), cell-local
  int nb[PM];                     // neighbour (original index) or -1-f
  union {                         // never live at the same time (one wave per block)
    int tid[64 * SPL];            // repack staging: packed plane triple
    float key[64];                // per-lane ordering keys
  };
  double tpos[64 * SPL][3];
  int stack[STACK];
  unsigned char used[PM];
  unsigned short remap[PM];
  unsigned long long omask[SPL];  // removed-vertex masks of the current clip
  double cpl[64][4];              // flagged candidates in processing order: m, h
  int corig[64];
  int wl[64];                     // warm start: the candidates taken from the previous adjacency
};

enum ClipResult { NOCUT = 0, CUT = 1, EMPTY = 2, OVER_V = 3, OVER_P = 4, OVER_W = 5, OVER_S = 6 };

__device__ inline bool is_over(int st) { return st >= OVER_V; }

template <int SPL>
struct Poly {
  int id[SPL];                    // packed (a | b<<8 | c<<16), slot lane + 64*s
  double x[SPL], y[SPL], z[SPL];  // vertex positions
  int ntri;                       // wave-uniform vertex count
  double r2;                      // max |v|^2 (ball around p_i)
  double cx, cy, cz, rc2;         // ball around the vertex centroid
};

__device__ inline void unpack(int id, int& a, int& b, int& c) {
  a = id & 255;
  b = (id >> 8) & 255;
  c = (id >> 16) & 255;
}


template <int PM, typename EOT>
__device__ inline void reg_edges(EOT* eo, int id, int slot) {
  int a, b, c;
  unpack(id, a, b, c);
  eo[a * PM + b] = (EOT)slot;
  eo[b * PM + c] = (EOT)slot;
  eo[c * PM + a] = (EOT)slot;
}

template <int SPL, int PM>
__device__ inline void plane_triple(const Shared<SPL, PM>& S, int a, int b, double mx, double my, double mz,
                                    double h, double& x, double& y, double& z) {
  const double ax = S.pl[a][0], ay = S.pl[a][1], az = S.pl[a][2], ah = S.pl[a][3];
  const double bx = S.pl[b][0], by = S.pl[b][1], bz = S.pl[b][2], bh = S.pl[b][3];
  // c23 = b x k, c31 = k x a, c12 = a x b
  const double c23x = by * mz - bz * my, c23y = bz * mx - bx * mz, c23z = bx * my - by * mx;
  const double c31x = my * az - mz * ay, c31y = mz * ax - mx * az, c31z = mx * ay - my * ax;
  const double c12x = ay * bz - az * by, c12y = az * bx - ax * bz, c12z = ax * by - ay * bx;
  const double det = ax * c23x + ay * c23y + az * c23z;
  const double inv = 1.0 / det;
  x = (ah * c23x + bh * c31x + h * c12x) * inv;
  y = (ah * c23y + bh * c31y + h * c12y) * inv;
  z = (ah * c23z + bh * c31z + h * c12z) * inv;
}

template <int SPL>
__device__ inline void update_bounds(Poly<SPL>& P) {
  const int lane = threadIdx.x;
  double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    if (lane + 64 * s < P.ntri) {
      m = fmax(m, P.x[s] * P.x[s] + P.y[s] * P.y[s] + P.z[s] * P.z[s]);
      sx += P.x[s];
      sy += P.y[s];
      sz += P.z[s];
    }
  }
  P.r2 = wave_max_d(m);
  const double inv = 1.0 / (double)P.ntri;
  P.cx = wave_sum_d(sx) * inv;
  P.cy = wave_sum_d(sy) * inv;
  P.cz = wave_sum_d(sz) * inv;
  double mc = 0.0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    if (lane + 64 * s < P.ntri) {
      const double dx = P.x[s] - P.cx, dy = P.y[s] - P.cy, dz = P.z[s] - P.cz;
      mc = fmax(mc, dx * dx + dy * dy + dz * dz);
    }
  }
  P.rc2 = wave_max_d(mc);
}

// Clip the polytope by plane kp (already stored in S.pl[kp]).
template <int SPL, int PM, typename EOT>
__device__ ClipResult clip(Shared<SPL, PM>& S, EOT* eo, Poly<SPL>& P, int kp, double mx, double my, double mz,
                           double h) {
  constexpr int NT = 64 * SPL;
  const int lane = threadIdx.x;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  bool in[SPL], out[SPL];
  uint64_t ob[SPL];
  int nout = 0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    in[s] = lane + 64 * s < P.ntri;
    out[s] = in[s] && (mx * P.x[s] + my * P.y[s] + mz * P.z[s] > h);
    ob[s] = __ballot(out[s]);
    nout += __popcll(ob[s]);
  }
  if (nout == 0) return NOCUT;
  if (nout == P.ntri) return EMPTY;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < SPL; ++s) S.omask[s] = ob[s];
  }
  __syncthreads();

  // new vertices: each edge from a removed vertex to a kept one
  bool e[3 * SPL];
  int ex[3 * SPL], ey[3 * SPL];
  int my_new = 0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    int a, b, c;
    unpack(P.id[s], a, b, c);
    const int xs[3] = {a, b, c}, ys[3] = {b, c, a};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      ex[3 * s + q] = xs[q];
      ey[3 * s + q] = ys[q];
      bool keep_opp = false;
      if (out[s]) {
        const int opp = (int)eo[ys[q] * PM + xs[q]] & (NT - 1);
        keep_opp = ((S.omask[opp >> 6] >> (opp & 63)) & 1ull) == 0ull;
      }
      e[3 * s + q] = out[s] && keep_opp;
      my_new += e[3 * s + q] ? 1 : 0;
    }
  }
  // exclusive prefix sum and total of my_new (< 2^NB) from one ballot per bit
  constexpr int NB = SPL <= 2 ? 3 : SPL <= 5 ? 4 : 5;
  int excl = 0, total_new = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const uint64_t bm = __ballot((my_new >> b) & 1);
    excl += __popcll(bm & lt) << b;
    total_new += __popcll(bm) << b;
  }
  const int nkeep = P.ntri - nout;
  if (nkeep + total_new > NT) return OVER_V;

  int kbase = 0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const bool keep = in[s] && !out[s];
    const uint64_t kb = __ballot(keep);
    if (keep) {
      const int pos = kbase + __popcll(kb & lt);
      S.tid[pos] = P.id[s];
      S.tpos[pos][0] = P.x[s]; S.tpos[pos][1] = P.y[s]; S.tpos[pos][2] = P.z[s];
    }
    kbase += __popcll(kb);
  }
  int pos = nkeep + excl;
#pragma unroll
  for (int q = 0; q < 3 * SPL; ++q) {
    if (e[q]) {
      double x, y, z;
      plane_triple(S, ex[q], ey[q], mx, my, mz, h, x, y, z);
      S.tid[pos] = ex[q] | (ey[q] << 8) | (kp << 16);
      S.tpos[pos][0] = x; S.tpos[pos][1] = y; S.tpos[pos][2] = z;
      ++pos;
    }
  }
  __syncthreads();
  P.ntri = nkeep + total_new;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int t = lane + 64 * s;
    if (t < P.ntri) {
      P.id[s] = S.tid[t];
      P.x[s] = S.tpos[t][0]; P.y[s] = S.tpos[t][1]; P.z[s] = S.tpos[t][2];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s)
    if (lane + 64 * s < P.ntri) reg_edges<PM>(eo, P.id[s], lane + 64 * s);
  __syncthreads();
  update_bounds(P);
  return CUT;
}

// Whether the bisector plane (m, h) can reach the polytope: it must come
// within the bounding ball around the vertex centroid (or p_i coincides
// with the other site).
template <int SPL>
__device__ inline bool may_cut(const Poly<SPL>& P, double mx, double my, double mz, double mm, double h) {
  const double t = h - (mx * P.cx + my * P.cy + mz * P.cz);
  return t < 0.0 || t * t < P.rc2 * mm || mm == 0.0;
}

struct Cand {
  double mx, my, mz, mm, h;
  int orig;
  bool ok;
};

__device__ inline Cand load_cand(const float4* __restrict__ sp, const int32_t* __restrict__ sidx, int64_t j,
                                 bool valid, double px, double py, double pz, double wi) {
  Cand c;
  c.ok = valid;
  c.mx = c.my = c.mz = c.mm = c.h = 0.0;
  c.orig = -1;
  if (valid) {
    float4 s = sp[j];
    c.mx = (double)s.x - px;
    c.my = (double)s.y - py;
    c.mz = (double)s.z - pz;
    c.mm = c.mx * c.mx + c.my * c.my + c.mz * c.mz;
    c.h = 0.5 * (c.mm + wi - (double)s.w);
    c.orig = sidx[j];
  }
  return c;
}

// Drops planes that no longer bound the polytope and renumbers the rest,
// so that the plane capacity limits live faces only.  Returns the new plane
// count.
template <int SPL, int PM, typename EOT>
__device__ int compact_planes(Shared<SPL, PM>& S, EOT* eo, Poly<SPL>& P, int nplanes) {
  constexpr int NR = (PM + 63) / 64;
  const int lane = threadIdx.x;
  for (int q = lane; q < PM; q += 64) S.used[q] = 0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    if (lane + 64 * s < P.ntri) {
      int a, b, c;
      unpack(P.id[s], a, b, c);
      S.used[a] = 1; S.used[b] = 1; S.used[c] = 1;
    }
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  bool u[NR];
  int dst[NR];
  double pl[NR][4];
  int nbv[NR];
  int base = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = lane + 64 * r;
    u[r] = q < nplanes && q < PM && S.used[q];
    const uint64_t m = __ballot(u[r]);
    dst[r] = base + __popcll(m & lt);
    base += __popcll(m);
    if (u[r]) {
      for (int c = 0; c < 4; ++c) pl[r][c] = S.pl[q][c];
      nbv[r] = S.nb[q];
      S.remap[q] = (unsigned short)dst[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (u[r]) {
      for (int c = 0; c < 4; ++c) S.pl[dst[r]][c] = pl[r][c];
      S.nb[dst[r]] = nbv[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    if (lane + 64 * s < P.ntri) {
      int a, b, c;
      unpack(P.id[s], a, b, c);
      P.id[s] = S.remap[a] | (S.remap[b] << 8) | (S.remap[c] << 16);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s)
    if (lane + 64 * s < P.ntri) reg_edges<PM>(eo, P.id[s], lane + 64 * s);
  __syncthreads();
  return base;
}

// Whether the plane (m, h) cuts off a vertex of the current polytope (the
// vertex list after the last clip is in S.tpos).
template <int SPL, int PM>
__device__ inline bool cuts_vertices(const Shared<SPL, PM>& S, int ntri, double mx, double my, double mz,
                                     double h) {
  for (int t = 0; t < ntri; ++t)
    if (mx * S.tpos[t][0] + my * S.tpos[t][1] + mz * S.tpos[t][2] > h) return true;
  return false;
}

// Number of flagged lanes whose key orders before this lane's (ties by
// lane); keys of the wave in S.key.
template <int SPL, int PM>
__device__ inline int lane_rank(const Shared<SPL, PM>& S, uint64_t flagged, float key) {
  const int lane = threadIdx.x;
  int rank = 0;
  while (flagged) {
    const int t = __ffsll((long long)flagged) - 1;
    flagged &= flagged - 1;
    const float kt = S.key[t];
    rank += (kt < key || (kt == key && t < lane)) ? 1 : 0;
  }
  return rank;
}

// Processes one batch of candidates (one per lane).  The polytope only
// shrinks, so a candidate whose plane misses every current vertex can never
// cut later and is dropped at once; the others are clipped in order of
// their bisector's offset from p_i (most constraining first).
// Returns false when the cell became empty or overflowed (state in status).
template <int SPL, int PM, typename EOT>
__device__ bool process_batch(Shared<SPL, PM>& S, EOT* eo, Poly<SPL>& P, int& nplanes, int& status, const Cand& c,
                              int self_orig, int& work) {
  const int lane = threadIdx.x;
  const bool f = c.ok && (c.mm == 0.0 || (may_cut(P, c.mx, c.my, c.mz, c.mm, c.h) &&
                                          cuts_vertices(S, P.ntri, c.mx, c.my, c.mz, c.h)));
  const uint64_t fm = __ballot(f);
  if (fm == 0ull) return true;
  const int nflag = __popcll(fm);
  // most constraining first: order by the plane's offset from p_i, h/|m|
  // (coincident sites first)
  const float okey = c.mm > 0.0 ? (float)(c.h / sqrt(c.mm)) : -INFINITY;
  S.key[lane] = f ? okey : INFINITY;
  __syncthreads();
  if (f) {
    const int r = lane_rank(S, fm, okey);
    S.cpl[r][0] = c.mx; S.cpl[r][1] = c.my; S.cpl[r][2] = c.mz; S.cpl[r][3] = c.h;
    S.corig[r] = c.orig;
  }
  __syncthreads();
  for (int r = 0; r < nflag; ++r) {
    if (++work > WORK_LIMIT) {
      status = OVER_W;
      return false;
    }
    const double mx = S.cpl[r][0], my = S.cpl[r][1], mz = S.cpl[r][2], h = S.cpl[r][3];
    const double mm = mx * mx + my * my + mz * mz;
    const int orig = S.corig[r];
    if (mm == 0.0) {
      // coincident sites: the one with the smaller weight (or, on a tie,
      // the larger index) owns nothing
      if (h < 0.0 || (h == 0.0 && orig < self_orig)) {
        status = EMPTY;
        return false;
      }
      continue;
    }
    if (!may_cut(P, mx, my, mz, mm, h)) continue;
    if (nplanes == PM) {
      nplanes = compact_planes(S, eo, P, nplanes);
      if (nplanes == PM) {
        status = OVER_P;
        return false;
      }
    }
    if (lane == 0) {
      S.pl[nplanes][0] = mx; S.pl[nplanes][1] = my; S.pl[nplanes][2] = mz; S.pl[nplanes][3] = h;
      S.nb[nplanes] = orig;
    }
    __syncthreads();
    const ClipResult res = clip(S, eo, P, nplanes, mx, my, mz, h);
    if (res == CUT) {
      ++nplanes;
    } else if (res == EMPTY || is_over(res)) {
      status = res;
      return false;
    }
  }
  return true;
}

// MODE 0: all cells, sorted position k = blockIdx.x, faces at stride
// FACE_CAP by original index, edge table in LDS.  MODE 1: the cells listed
// in klist (sorted positions), faces at stride PM_BIG in slot blockIdx.x
// (recorded in bigslot), edge table in LDS.  MODE 2: listed cells that
// already own a slot, edge table in an HBM workspace (for PM*PM too large
// for LDS).
template <int SPL, int PM, int MODE>
__global__ void __launch_bounds__(64) k_clip(const float4* __restrict__ sp, const int32_t* __restrict__ sidx,
                                             int64_t n, const float4* __restrict__ nlo,
                                             const float4* __restrict__ nhi, Levels lv, float3 bmin,
                                             float3 bmax, const float* __restrict__ radius,
                                             const int32_t* __restrict__ klist, unsigned short* __restrict__ eo_g,
                                             int32_t* __restrict__ faces, int32_t* __restrict__ bigslot,
                                             int32_t* __restrict__ counts, int32_t* __restrict__ nrast,
                                             float* __restrict__ cull, int32_t* __restrict__ flags,
                                             const int32_t* __restrict__ wrow, const int32_t* __restrict__ wcol,
                                             const int32_t* __restrict__ wwit, const int32_t* __restrict__ spos,
                                             int32_t* __restrict__ wit_out) {
  constexpr bool LISTED = MODE >= 1, EO_HBM = MODE == 2;
  using EOT = typename std::conditional<(64 * SPL > 256), unsigned short, unsigned char>::type;
  static_assert(EO_HBM ? std::is_same<EOT, unsigned short>::value : true, "HBM edge table holds 16-bit slots");
  __shared__ Shared<SPL, PM> S;
  __shared__ EOT eo_lds[EO_HBM ? 1 : PM * PM];
  EOT* eo;
  if constexpr (EO_HBM) eo = (EOT*)(eo_g + (int64_t)blockIdx.x * PM * PM);
  else eo = eo_lds;
  const int lane = threadIdx.x;
  const int64_t k = LISTED ? (int64_t)klist[blockIdx.x] : (int64_t)blockIdx.x;
  const float4 me = sp[k];
  const int32_t self = sidx[k];
  const double px = me.x, py = me.y, pz = me.z, wi = me.w;
  const double ri = radius[self];

  // domain box as the initial polytope
  const double bh[6] = {(double)bmax.x - px, px - (double)bmin.x, (double)bmax.y - py,
                        py - (double)bmin.y, (double)bmax.z - pz, pz - (double)bmin.z};
  if (lane < 6) {
    const int ax = lane >> 1;
    const double sgn = (lane & 1) ? -1.0 : 1.0;
    S.pl[lane][0] = ax == 0 ? sgn : 0.0;
    S.pl[lane][1] = ax == 1 ? sgn : 0.0;
    S.pl[lane][2] = ax == 2 ? sgn : 0.0;
    S.pl[lane][3] = bh[lane];
    S.nb[lane] = -1 - lane;
  }
  Poly<SPL> P;
  P.ntri = 8;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    P.id[s] = 0;
    P.x[s] = P.y[s] = P.z[s] = 0.0;
  }
  if (lane < 8) {
    const int sx = (lane & 1) ? -1 : 1, sy = (lane & 2) ? -1 : 1, sz = (lane & 4) ? -1 : 1;
    const int X = sx > 0 ? 0 : 1, Y = sy > 0 ? 2 : 3, Z = sz > 0 ? 4 : 5;
    // orientation det(m_X, m_Y, m_Z) = sx*sy*sz
    P.id[0] = (sx * sy * sz > 0) ? (X | (Y << 8) | (Z << 16)) : (Y | (X << 8) | (Z << 16));
    P.x[0] = sx > 0 ? bh[0] : -bh[1];
    P.y[0] = sy > 0 ? bh[2] : -bh[3];
    P.z[0] = sz > 0 ? bh[4] : -bh[5];
  }
  if (lane < 8) {
    S.tpos[lane][0] = P.x[0]; S.tpos[lane][1] = P.y[0]; S.tpos[lane][2] = P.z[0];
  }
  __syncthreads();
  if (lane < 8) reg_edges<PM>(eo, P.id[0], lane);
  __syncthreads();
  update_bounds(P);
  int nplanes = 6;
  // a dropped cell (weight -inf) has an empty power cell and cuts no other
  int status = wi > -INFINITY ? CUT : EMPTY;
  int work = 0;

  // phase 1, warm start from a previous build: a cell that had faces starts
  // from its previous neighbours (sites that moved little keep most of
  // them), then one unrestricted traversal certifies it; a cell that was
  // empty starts from the sites that emptied it, which usually empty it
  // again at once.  Otherwise (or if that fails) the own leaf (Morton
  // neighbours) and rings.
  const int64_t leaf = k / LEAF;
  const int wb = (MODE <= 1 && wrow) ? wrow[self] : 0;
  const int wcnt = (MODE <= 1 && wrow) ? wrow[self + 1] - wb : 0;
  const bool warm = wcnt > 0;
  int nwl = 0;
  double dmax = 0.0;
  if (MODE <= 1 && wrow && status == CUT && (warm || wwit)) {
    nwl = warm ? min(wcnt, 64) : WIT;
    const int v = lane < nwl ? (warm ? wcol[wb + lane] : wwit[(int64_t)self * WIT + lane]) : -1;
    const bool ok = v >= 0 && v < n && v != self;
    S.wl[lane] = ok ? v : -1;
    __syncthreads();
    const Cand c = load_cand(sp, sidx, ok ? (int64_t)spos[v] : 0, ok, px, py, pz, wi);
    process_batch(S, eo, P, nplanes, status, c, self, work);
    if (warm) dmax = INFINITY;
  }
  if (!warm && status == CUT) {
    const int64_t j = leaf * LEAF + lane;
    bool ok = j < n && j != k;
    double d2 = INFINITY;
    if (ok) {
      const float4 q = sp[j];
      const double dx = (double)q.x - px, dy = (double)q.y - py, dz = (double)q.z - pz;
      d2 = dx * dx + dy * dy + dz * dz;
    }
    // first ring radius: the RING_K-th nearest leaf mate, at most r_i (a
    // Morton leaf can straddle a jump of the curve and span the scene)
    const uint64_t okm = __ballot(ok);
    S.key[lane] = ok ? (float)d2 : INFINITY;
    __syncthreads();
    const int target = min(RING_K, __popcll(okm) - 1);
    const uint64_t sel = __ballot(ok && lane_rank(S, okm, (float)d2) == target);
    __syncthreads();
    const double dk = sel ? __shfl(d2, __ffsll((long long)sel) - 1, 64) : 0.0;
    dmax = fmax(fmin(sqrt(dk), ri), 1e-6);
    Cand c = load_cand(sp, sidx, j, ok, px, py, pz, wi);
    for (int q = 0; q < nwl; ++q) c.ok = c.ok && S.wl[q] != c.orig;   // seeds already taken
    process_batch(S, eo, P, nplanes, status, c, self, work);
  }

  // phase 2: the other sites in rings [dmin, dmax) of doubling radius, which
  // brings near sites first across the whole tree and keeps the transient
  // polytope small.  Each ring walks the tree depth first, most constraining
  // child first, pruning by the current polytope; a ring that left no
  // prunable work beyond dmax ends the search.
  double dmin = 0.0;
  while (status == CUT) {
    bool skipped = false;
    int top = 1;
    if (lane == 0) S.stack[0] = (lv.n << 24) | 0;
    __syncthreads();
    while (top > 0 && status == CUT) {
      if (++work > WORK_LIMIT) {
        status = OVER_W;
        break;
      }
      const int ent = S.stack[top - 1];
      --top;
      const int L = ent >> 24;
      const long long idx = ent & 0xFFFFFF;
      if (L == 1) {
        if (idx == leaf && !warm) continue;
        const int64_t j = idx * LEAF + lane;
        const bool ok = j < n && j != k;
        const Cand c0 = load_cand(sp, sidx, j, ok, px, py, pz, wi);
        const bool beyond = ok && c0.mm >= dmax * dmax;
        if (__ballot(beyond && may_cut(P, c0.mx, c0.my, c0.mz, c0.mm, c0.h)) != 0ull) skipped = true;
        Cand c = c0;
        c.ok = ok && !beyond && c0.mm >= dmin * dmin;
        // a warm-start candidate was already taken
        for (int q = 0; q < nwl; ++q) c.ok = c.ok && S.wl[q] != c0.orig;
        if (__ballot(c.ok) == 0ull) continue;
        if (!process_batch(S, eo, P, nplanes, status, c, self, work)) break;
        continue;
      }
      // children are nodes of level L-1
      const long long cnum = lv.cnt[L - 1];
      const long long cidx = idx * 64 + lane;
      const bool valid = cidx < cnum;
      double lx = 0, ly = 0, lz = 0, hx = 0, hy = 0, hz = 0, W = 0;
      bool keep = false;
      double dkey = INFINITY;
      if (valid) {
        const float4 a = nlo[lv.off[L - 1] + cidx], b = nhi[lv.off[L - 1] + cidx];
        lx = (double)a.x - px; ly = (double)a.y - py; lz = (double)a.z - pz; W = a.w;
        hx = (double)b.x - px; hy = (double)b.y - py; hz = (double)b.z - pz;
        // ball around p_i
        const double dx = fmax(0.0, fmax(lx, -hx)), dy = fmax(0.0, fmax(ly, -hy)), dz = fmax(0.0, fmax(lz, -hz));
        const double D = sqrt(dx * dx + dy * dy + dz * dz);
        const double R = sqrt(P.r2);
        const bool far0 = D > R && (D - R) * (D - R) - W >= P.r2 - wi;
        // ball around the vertex centroid
        const double ex = fmax(0.0, fmax(lx - P.cx, P.cx - hx)), ey = fmax(0.0, fmax(ly - P.cy, P.cy - hy));
        const double ez = fmax(0.0, fmax(lz - P.cz, P.cz - hz));
        const double Dc = sqrt(ex * ex + ey * ey + ez * ez), Rc = sqrt(P.rc2);
        const double cn = sqrt(P.cx * P.cx + P.cy * P.cy + P.cz * P.cz) + Rc;
        const bool far1 = Dc > Rc && (Dc - Rc) * (Dc - Rc) - W >= cn * cn - wi;
        keep = !(far0 || far1);
        if (keep && D >= dmax) {
          skipped = true;   // wait for a later ring
          keep = false;
        }
        // lower bound of the bisector offset h/|m| of any site in the box
        if (keep) dkey = (D * D + wi - W) / (2.0 * fmax(D, 1e-12));
      }
      if (__ballot(valid && skipped) != 0ull) skipped = true;
      // exact per-vertex test, one child box per lane: can any site in the
      // box beat p_i at a vertex of the current polytope?
      bool cut = false;
      if (keep) {
        for (int t = 0; t < P.ntri && !cut; ++t) {
          const double vx = S.tpos[t][0], vy = S.tpos[t][1], vz = S.tpos[t][2];
          const double dx = fmax(0.0, fmax(lx - vx, vx - hx));
          const double dy = fmax(0.0, fmax(ly - vy, vy - hy));
          const double dz = fmax(0.0, fmax(lz - vz, vz - hz));
          cut = dx * dx + dy * dy + dz * dz - W < vx * vx + vy * vy + vz * vz - wi;
        }
      }
      const uint64_t cm = __ballot(cut);
      if (cm != 0ull) {
        const int nc = __popcll(cm);
        if (top + nc > STACK) {
          status = OVER_S;
          break;
        }
        // most constraining child (smallest offset bound) on top of the stack
        S.key[lane] = cut ? (float)dkey : INFINITY;
        __syncthreads();
        if (cut) S.stack[top + nc - 1 - lane_rank(S, cm, (float)dkey)] = ((L - 1) << 24) | (int)(idx * 64 + lane);
        top += nc;
      }
      __syncthreads();
    }
    if (!skipped) break;
    // rings double until they lie beyond every vertex of the polytope; the
    // remaining sites can then only cut through their weight, and one
    // unrestricted traversal certifies the cell
    dmin = dmax;
    dmax = (dmin * dmin >= P.r2) ? INFINITY : 2.0 * dmax;
  }

  // --- outputs
  int32_t* out;
  if constexpr (MODE == 0) {
    out = faces + (int64_t)self * FACE_CAP;
  } else if constexpr (MODE == 1) {
    out = faces + (int64_t)blockIdx.x * PM_BIG;
    if (lane == 0) bigslot[self] = (int32_t)blockIdx.x;
  } else {
    out = faces + (int64_t)bigslot[self] * PM_BIG;
  }
  if (status == EMPTY || is_over(status)) {
    // the most recent planes (the last one emptied the cell), for the next build
    if (wit_out && lane < WIT) {
      const int q = nplanes - lane;
      wit_out[(int64_t)self * WIT + lane] = (status == EMPTY && q >= 0 && q < PM) ? S.nb[q] : -1;
    }
    if (lane == 0) {
      counts[self] = 0;
      nrast[self] = 0;
      cull[self] = -1.0f;
      const int why = status == OVER_V ? FLAG_OVER_VERTS : status == OVER_P ? FLAG_OVER_PLANES
                    : status == OVER_W ? FLAG_OVER_WORK : FLAG_OVER_STACK;
      flags[self] = status == EMPTY ? FLAG_EMPTY_POWER : (FLAG_OVERFLOW | why);
    }
    return;
  }
  for (int q = lane; q < PM; q += 64) S.used[q] = 0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    if (lane + 64 * s < P.ntri) {
      int a, b, c;
      unpack(P.id[s], a, b, c);
      S.used[a] = 1; S.used[b] = 1; S.used[c] = 1;
    }
  }
  __syncthreads();
  // categories: 0 raster neighbour face, 1 other neighbour face, 2 box face
  constexpr int NR = (PM + 63) / 64;
  int cat[NR];
  double viol = -INFINITY;  // max over faces of the signed distance of p_i outside
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = lane + 64 * r;
    cat[r] = 3;
    if (q < nplanes && S.used[q]) {
      if (S.nb[q] < 0) {
        cat[r] = 2;
      } else {
        const double mx = S.pl[q][0], my = S.pl[q][1], mz = S.pl[q][2], h = S.pl[q][3];
        const double mn = sqrt(mx * mx + my * my + mz * mz);
        cat[r] = (fabs(h) <= ri * mn * (1.0 + 1e-6)) ? 0 : 1;
        viol = fmax(viol, -h / mn);
      }
    }
  }
  // faces by category, each category in increasing neighbour order (the
  // order in which the planes were taken does not show in the output)
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (lane + 64 * r < PM) S.used[lane + 64 * r] = (unsigned char)cat[r];
  __syncthreads();
  int cbase[3] = {0, 0, 0};
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int ccat = 0; ccat < 3; ++ccat) cbase[ccat] += __popcll(__ballot(cat[r] == ccat));
  const int nr = cbase[0];
  const int base = cbase[0] + cbase[1] + cbase[2];
  cbase[2] = cbase[0] + cbase[1];
  cbase[1] = cbase[0];
  cbase[0] = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = lane + 64 * r;
    if (cat[r] < 3) {
      const int me = S.nb[q];
      int pos = 0;
      for (int t = 0; t < nplanes; ++t)
        pos += (S.used[t] == cat[r] && (S.nb[t] < me || (S.nb[t] == me && t < q))) ? 1 : 0;
      out[cbase[cat[r]] + pos] = me;
    }
  }
  viol = wave_max_d(viol);
  const double R = sqrt(P.r2);
  if (lane == 0) {
    counts[self] = base;
    nrast[self] = nr;
    const bool hidden = viol > ri;
    cull[self] = hidden ? -1.0f : (float)fmin(ri, R * (1.0 + 1e-6));
    flags[self] = 0;
  }
}


// Connectivity loss over the Cech graph (supplementary material, loss
// functions): one wave per cell i walks the site tree for the spheres that
// overlap B(p_i, r_i) (nodes pruned by box distance > r_i + largest radius
// below).  With ov_ij = r_i + r_j - d_ij, each overlapping pair appears in
// L(i) and in L(j), so the derivative of the total with respect to r_i is
// 4 lambda sum_j ov_ij and with respect to p_i is
// 4 lambda sum_j ov_ij (p_j - p_i)/d_ij; every cell adds only its own
// gradient, so no atomics touch a neighbour.
__global__ void __launch_bounds__(64) k_connect(const float4* __restrict__ sp, const float* __restrict__ srad,
                                                const int32_t* __restrict__ sidx, int64_t n,
                                                const float4* __restrict__ nlo, const float4* __restrict__ nhi,
                                                Levels lv, float lambda, float* __restrict__ gp,
                                                float* __restrict__ gr, double* __restrict__ loss,
                                                unsigned int* __restrict__ overflow) {
  __shared__ int stack[STACK];
  const int lane = threadIdx.x;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t k = blockIdx.x;
  const float4 me = sp[k];
  const double px = me.x, py = me.y, pz = me.z, ri = srad[k];
  double lsum = 0.0, gsum = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  int top = 1;
  if (lane == 0) stack[0] = (lv.n << 24) | 0;
  __syncthreads();
  while (top > 0) {
    const int ent = stack[top - 1];
    --top;
    const int L = ent >> 24;
    const long long idx = ent & 0xFFFFFF;
    if (L == 1) {
      const int64_t j = idx * LEAF + lane;
      if (j < n && j != k) {
        const float4 q = sp[j];
        const double dx = (double)q.x - px, dy = (double)q.y - py, dz = (double)q.z - pz;
        const double rs = ri + (double)srad[j];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < rs * rs) {
          const double d = sqrt(d2);
          const double ov = rs - d;
          lsum += ov * ov;
          gsum += ov;
          if (d > 0.0) {   // d ov / d p_i = (p_j - p_i) / d
            gx += ov * dx / d;
            gy += ov * dy / d;
            gz += ov * dz / d;
          }
        }
      }
      continue;
    }
    const long long cidx = idx * 64 + lane;
    bool keep = false;
    if (cidx < lv.cnt[L - 1]) {
      const float4 a = nlo[lv.off[L - 1] + cidx], b = nhi[lv.off[L - 1] + cidx];
      const double ex = fmax(0.0, fmax((double)a.x - px, px - (double)b.x));
      const double ey = fmax(0.0, fmax((double)a.y - py, py - (double)b.y));
      const double ez = fmax(0.0, fmax((double)a.z - pz, pz - (double)b.z));
      const double reach = ri + (double)b.w;
      keep = ex * ex + ey * ey + ez * ez < reach * reach;
    }
    const uint64_t m = __ballot(keep);
    const int nc = __popcll(m);
    if (top + nc > STACK) {
      if (lane == 0) atomicAdd(overflow, 1u);
      break;
    }
    if (keep) stack[top + __popcll(m & lt)] = ((L - 1) << 24) | (int)cidx;
    top += nc;
    __syncthreads();
  }
  lsum = wave_sum_d(lsum);
  gsum = wave_sum_d(gsum);
  gx = wave_sum_d(gx);
  gy = wave_sum_d(gy);
  gz = wave_sum_d(gz);
  if (lane == 0) {
    const int32_t self = sidx[k];
    const double f = 4.0 * (double)lambda;
    if (gr && gsum != 0.0) atomicAdd(gr + self, (float)(f * gsum));
    if (gp && (gx != 0.0 || gy != 0.0 || gz != 0.0)) {
      atomicAdd(gp + 3 * (int64_t)self, (float)(f * gx));
      atomicAdd(gp + 3 * (int64_t)self + 1, (float)(f * gy));
      atomicAdd(gp + 3 * (int64_t)self + 2, (float)(f * gz));
    }
    if (loss && lsum != 0.0) atomicAdd(loss, (double)lambda * lsum);
  }
}

__global__ void k_list_overflow(const int32_t* __restrict__ flags, const int32_t* __restrict__ spos, int64_t n,
                                int32_t* __restrict__ klist, unsigned int* __restrict__ nlist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (flags[i] & FLAG_OVERFLOW)) klist[atomicAdd(nlist, 1u)] = spos[i];
}

__global__ void k_inverse(const int32_t* __restrict__ sidx, int64_t n, int32_t* __restrict__ spos) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) spos[sidx[k]] = (int32_t)k;
}

__global__ void k_fill(const float* __restrict__ p, const float* __restrict__ w, int64_t n,
                       const int32_t* __restrict__ faces_tmp, const int32_t* __restrict__ faces_big,
                       const int32_t* __restrict__ bigslot, const uint32_t* __restrict__ row,
                       const int32_t* __restrict__ counts, float3 bmin, float3 bmax,
                       int32_t* __restrict__ col, float4* __restrict__ plane) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2], wi = w[i];
  const int c = counts[i];
  const uint32_t off = row[i];
  for (int f = 0; f < c; ++f) {
    const int b = bigslot[i];
    const int v = b >= 0 ? faces_big[(int64_t)b * PM_BIG + f] : faces_tmp[i * FACE_CAP + f];
    float4 pl;
    if (v >= 0) {
      const double mx = (double)p[3 * v] - px, my = (double)p[3 * v + 1] - py, mz = (double)p[3 * v + 2] - pz;
      const double h = 0.5 * (mx * mx + my * my + mz * mz + wi - (double)w[v]);
      pl = make_float4((float)mx, (float)my, (float)mz, (float)h);
    } else {
      const int bf = -1 - v, ax = bf >> 1;
      const float sgn = (bf & 1) ? -1.0f : 1.0f;
      const double lim = (bf & 1) ? -((ax == 0 ? (double)bmin.x : ax == 1 ? (double)bmin.y : (double)bmin.z) -
                                      (ax == 0 ? px : ax == 1 ? py : pz))
                                  : (ax == 0 ? (double)bmax.x : ax == 1 ? (double)bmax.y : (double)bmax.z) -
                                        (ax == 0 ? px : ax == 1 ? py : pz);
      pl = make_float4(ax == 0 ? sgn : 0.0f, ax == 1 ? sgn : 0.0f, ax == 2 ? sgn : 0.0f, (float)lim);
    }
    col[off + f] = v;
    plane[off + f] = pl;
  }
}

__device__ inline float softplus_f(float x) { return x > 20.0f ? x : log1pf(expf(x)); }

// Packed records; a cell of zero density (e.g. an empty Steiner cell, whose
// logit is -inf) is never binned for the raster: it cannot contribute.
__global__ void k_prep(const float* __restrict__ p, const float* __restrict__ r, const float* __restrict__ nrm,
                       const float* __restrict__ lam, float sigma_scale, int64_t n, float4* __restrict__ geo,
                       float4* __restrict__ onrm, float* __restrict__ cull) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  geo[i] = make_float4(p[3 * i], p[3 * i + 1], p[3 * i + 2], r[i]);
  const float nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
  const float inv = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
  const float sigma = sigma_scale * softplus_f(lam[i]);
  onrm[i] = make_float4(nx * inv, ny * inv, nz * inv, sigma);
  if (!(sigma > 0.0f)) cull[i] = -1.0f;
}

// out: [hidden, overflow, over-vertices, over-planes, over-work, over-stack]
__global__ void k_count_flags(const int32_t* __restrict__ flags, const float* __restrict__ cull, int64_t n,
                              unsigned long long* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = i < n ? flags[i] : 0;
  const bool b[6] = {i < n && cull[i] < 0.0f, (f & FLAG_OVERFLOW) != 0, (f & FLAG_OVER_VERTS) != 0,
                     (f & FLAG_OVER_PLANES) != 0, (f & FLAG_OVER_WORK) != 0, (f & FLAG_OVER_STACK) != 0};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const uint64_t m = __ballot(b[q]);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&out[q], (unsigned long long)__popcll(m));
  }
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  hipStream_t s;
  explicit DevBuf(hipStream_t st) : s(st) {}
  ~DevBuf() { if (p) pf::pool_free(p, s); }
  hipError_t alloc(size_t count) { return pf::pool_alloc((void**)&p, sizeof(T) * (count ? count : 1), s); }
  void reset() {
    if (p) pf::pool_free(p, s);
    p = nullptr;
  }
};

// Zero-density cells that overflowed every build pass are dropped: their
// sorted-site weight becomes -inf, so a rebuild gives them an empty power
// cell and lets them cut no other cell.
__global__ void k_drop_void(const int32_t* __restrict__ flags, const int32_t* __restrict__ spos,
                            const float* __restrict__ lam, float sigma_scale, int64_t n, float4* __restrict__ sp,
                            unsigned int* __restrict__ ndrop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !(flags[i] & FLAG_OVERFLOW)) return;
  if (sigma_scale * softplus_f(lam[i]) > 0.0f) return;
  sp[spos[i]].w = -INFINITY;
  atomicAdd(ndrop, 1u);
}

}  // namespace

pf_status connect_loss_impl(const Scene& sc, float lambda, const pf_grads& g, double* loss_dev, hipStream_t s) {
  if (!sc.t_sp) {
    set_error("pf_connect_loss: the scene has no site tree");
    return PF_ERR_INVALID;
  }
  DevBuf<unsigned int> ovf(s);
  PF_HIP_TRY(ovf.alloc(1));
  PF_HIP_TRY(hipMemsetAsync(ovf.p, 0, sizeof(unsigned int), s));
  {
    ProfScope ps("k_connect", s);
    k_connect<<<(unsigned)sc.n, 64, 0, s>>>(sc.t_sp, sc.t_srad, sc.t_sidx, sc.n, sc.t_lo, sc.t_hi, sc.t_lv, lambda,
                                            g.p, g.radius, loss_dev, ovf.p);
  }
  PF_HIP_TRY(hipGetLastError());
  unsigned int h = 0;
  PF_HIP_TRY(hipMemcpyAsync(&h, ovf.p, sizeof(h), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  if (h) {
    set_error("pf_connect_loss: " + std::to_string(h) + " cells exceeded the traversal stack");
    return PF_ERR_OVERFLOW;
  }
  return PF_OK;
}

void free_scene(Scene* sc, hipStream_t s, bool async) {
  void* ptrs[] = {sc->geo,  sc->nrm,    sc->cull,   sc->flags, sc->row,  sc->nrast, sc->col,
                  sc->plane, sc->t_sp, sc->t_sidx, sc->t_srad, sc->t_lo, sc->t_hi, sc->wit};
  // synchronous: renders on any stream may still read the arrays
  if (!async) (void)hipDeviceSynchronize();
  for (void* q : ptrs)
    if (q) pf::pool_free(q, async ? s : nullptr);
  sc->geo = sc->nrm = nullptr;
  sc->cull = nullptr;
  sc->flags = sc->row = sc->nrast = sc->col = nullptr;
  sc->plane = nullptr;
  sc->t_sp = sc->t_lo = sc->t_hi = nullptr;
  sc->t_sidx = nullptr;
  sc->t_srad = nullptr;
  sc->wit = nullptr;
}

pf_status build_scene_impl(const pf_params& prm, const pf_build_opts& opt, hipStream_t s, Scene* sc,
                           const Scene* prev) {
  const int64_t n = prm.n;
  // warm start from a previous build of the same cells
  const bool use_prev = prev && prev->n == n && prev->row && prev->col;
  const int32_t* warm_row = use_prev ? prev->row : nullptr;
  const int32_t* warm_col = use_prev ? prev->col : nullptr;
  const int32_t* warm_wit = use_prev ? prev->wit : nullptr;
  sc->n = n;
  sc->prm = prm;

  // bounds of the spheres
  const int nbk = (int)std::min<int64_t>(1024, (n + 255) / 256);
  DevBuf<float> part(s);
  PF_HIP_TRY(part.alloc((size_t)nbk * 8));
  k_bounds<<<nbk, 256, 0, s>>>(prm.p, prm.power, prm.radius, n, part.p);
  PF_HIP_TRY(hipGetLastError());
  std::vector<float> hp((size_t)nbk * 8);
  PF_HIP_TRY(hipMemcpyAsync(hp.data(), part.p, sizeof(float) * hp.size(), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float rmin = INFINITY;
  for (int b = 0; b < nbk; ++b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], hp[b * 8 + a]);
      hi[a] = std::max(hi[a], hp[b * 8 + 3 + a]);
    }
    rmin = std::min(rmin, hp[b * 8 + 7]);
  }
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a])) {
      set_error("pf_build_scene: non-finite site or radius");
      return PF_ERR_INVALID;
    }
  }
  if (!(rmin > 0.0f)) {
    set_error("pf_build_scene: radii must be positive");
    return PF_ERR_INVALID;
  }
  const bool user_box = opt.box_min[0] <= opt.box_max[0];
  const float pad = opt.box_pad > 0.0f ? opt.box_pad : 0.01f;
  for (int a = 0; a < 3; ++a) {
    float l = lo[a], h = hi[a];
    if (user_box) {
      l = std::min(l, opt.box_min[a]);
      h = std::max(h, opt.box_max[a]);
    }
    const float ext = std::max(h - l, 1e-6f);
    sc->box_min[a] = l - pad * ext;
    sc->box_max[a] = h + pad * ext;
  }
  const float3 bmin = make_float3(sc->box_min[0], sc->box_min[1], sc->box_min[2]);
  const float3 bmax = make_float3(sc->box_max[0], sc->box_max[1], sc->box_max[2]);

  // Morton order of the sites
  DevBuf<uint32_t> keys(s), order(s);
  PF_HIP_TRY(keys.alloc(n));
  PF_HIP_TRY(order.alloc(n));
  const float3 inv = make_float3(1024.0f / (bmax.x - bmin.x), 1024.0f / (bmax.y - bmin.y),
                                 1024.0f / (bmax.z - bmin.z));
  const unsigned g256 = (unsigned)((n + 255) / 256);
  k_morton<<<g256, 256, 0, s>>>(prm.p, n, bmin, inv, keys.p, order.p);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(radix_sort_u32(keys.p, order.p, n, 30, s));
  // the sorted sites and the tree stay with the scene (sphere-overlap queries)
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->t_sp, sizeof(float4) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->t_sidx, sizeof(int32_t) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->t_srad, sizeof(float) * n, s));
  struct { float4* p; } sp{sc->t_sp};
  struct { int32_t* p; } sidx{sc->t_sidx};
  k_gather_sites<<<g256, 256, 0, s>>>(prm.p, prm.power, prm.radius, order.p, n, sp.p, sidx.p, sc->t_srad);
  PF_HIP_TRY(hipGetLastError());

  // implicit 64-ary tree over n sorted sites: per node the box of its sites,
  // their largest weight and largest sphere radius
  auto build_tree = [&](const float4* sites, const float* srad, int64_t count, Levels& lvl, float4*& lo_p,
                        float4*& hi_p) -> pf_status {
    lvl = Levels{};
    lvl.cnt[0] = count;
    long long total_nodes = 0;
    int L = 0;
    do {
      ++L;
      if (L > MAXLVL) {
        set_error("pf_build_scene: too many sites for the build tree");
        return PF_ERR_UNSUPPORTED;
      }
      lvl.cnt[L] = (lvl.cnt[L - 1] + 63) / 64;
      lvl.off[L] = total_nodes;
      total_nodes += lvl.cnt[L];
    } while (lvl.cnt[L] > 1);
    lvl.n = L;
    PF_HIP_TRY(pf::pool_alloc((void**)&lo_p, sizeof(float4) * total_nodes, s));
    PF_HIP_TRY(pf::pool_alloc((void**)&hi_p, sizeof(float4) * total_nodes, s));
    for (int l = 1; l <= lvl.n; ++l) {
      const bool from_sites = l == 1;
      k_tree_level<<<(unsigned)lvl.cnt[l], 64, 0, s>>>(from_sites ? sites : nullptr, from_sites ? srad : nullptr,
                                                       from_sites ? nullptr : lo_p + lvl.off[l - 1],
                                                       from_sites ? nullptr : hi_p + lvl.off[l - 1],
                                                       lvl.cnt[l - 1], lo_p + lvl.off[l], hi_p + lvl.off[l]);
      PF_HIP_TRY(hipGetLastError());
    }
    return PF_OK;
  };
  {
    const pf_status st = build_tree(sp.p, sc->t_srad, n, sc->t_lv, sc->t_lo, sc->t_hi);
    if (st != PF_OK) return st;
  }
  const Levels lv = sc->t_lv;
  struct { float4* p; } nlo{sc->t_lo}, nhi{sc->t_hi};

  // per-cell clipping
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->cull, sizeof(float) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->flags, sizeof(int32_t) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->wit, sizeof(int32_t) * WIT * n, s));
  PF_HIP_TRY(hipMemsetAsync(sc->wit, 0xFF, sizeof(int32_t) * WIT * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->nrast, sizeof(int32_t) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->row, sizeof(int32_t) * (n + 1), s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->geo, sizeof(float4) * n, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->nrm, sizeof(float4) * n, s));
  DevBuf<int32_t> faces_tmp(s), counts(s), bigslot(s), spos(s), klist(s), faces_big(s);
  DevBuf<unsigned short> eo_big(s);
  DevBuf<unsigned int> nbig_d(s), ndrop_d(s);
  PF_HIP_TRY(faces_tmp.alloc((size_t)n * FACE_CAP));
  PF_HIP_TRY(counts.alloc(n + 1));
  PF_HIP_TRY(bigslot.alloc(n));
  PF_HIP_TRY(spos.alloc(n));
  PF_HIP_TRY(klist.alloc(n));
  PF_HIP_TRY(nbig_d.alloc(1));
  PF_HIP_TRY(ndrop_d.alloc(1));
  k_inverse<<<g256, 256, 0, s>>>(sidx.p, n, spos.p);
  PF_HIP_TRY(hipGetLastError());
  auto list_overflow = [&](unsigned int& count) -> pf_status {
    PF_HIP_TRY(hipMemsetAsync(nbig_d.p, 0, sizeof(unsigned int), s));
    k_list_overflow<<<g256, 256, 0, s>>>(sc->flags, spos.p, n, klist.p, nbig_d.p);
    PF_HIP_TRY(hipGetLastError());
    PF_HIP_TRY(hipMemcpyAsync(&count, nbig_d.p, sizeof(count), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    return PF_OK;
  };
  // all passes; repeated (at most 3 more times) while zero-density cells
  // overflow and are dropped
  sc->n_dropped = 0;
  for (int attempt = 0;; ++attempt) {
  PF_HIP_TRY(hipMemsetAsync(bigslot.p, 0xFF, sizeof(int32_t) * n, s));
  {
    ProfScope ps_clip("k_clip", s);
    k_clip<2, FACE_CAP, 0><<<(unsigned)n, 64, 0, s>>>(sp.p, sidx.p, n, nlo.p, nhi.p, lv, bmin, bmax, prm.radius,
                                                         nullptr, nullptr, faces_tmp.p, nullptr, counts.p,
                                                         sc->nrast, sc->cull, sc->flags, warm_row, warm_col,
                                                         warm_wit, spos.p, sc->wit);
  }
  PF_HIP_TRY(hipGetLastError());
  // second pass (twice the capacity, edge table still in LDS) for the cells
  // that overflowed, third pass (4x, edge table in HBM) for what is left
  unsigned int nbig = 0;
  {
    const pf_status st = list_overflow(nbig);
    if (st != PF_OK) return st;
  }
  sc->n_big = nbig;
  faces_big.reset();
  eo_big.reset();
  if (nbig) {
    PF_HIP_TRY(faces_big.alloc((size_t)nbig * PM_BIG));
    {
      ProfScope ps_big("k_clip_mid", s);
      k_clip<SPL_MID, PM_MID, 1><<<nbig, 64, 0, s>>>(sp.p, sidx.p, n, nlo.p, nhi.p, lv, bmin, bmax, prm.radius,
                                                    klist.p, nullptr, faces_big.p, bigslot.p, counts.p, sc->nrast,
                                                    sc->cull, sc->flags, warm_row, warm_col, warm_wit, spos.p,
                                                    sc->wit);
    }
    PF_HIP_TRY(hipGetLastError());
    unsigned int nbig3 = 0;
    const pf_status st = list_overflow(nbig3);
    if (st != PF_OK) return st;
    if (nbig3) {
      PF_HIP_TRY(eo_big.alloc((size_t)nbig3 * PM_BIG * PM_BIG));
      ProfScope ps_big("k_clip_big", s);
      k_clip<SPL_BIG, PM_BIG, 2><<<nbig3, 64, 0, s>>>(sp.p, sidx.p, n, nlo.p, nhi.p, lv, bmin, bmax, prm.radius,
                                                     klist.p, eo_big.p, faces_big.p, bigslot.p, counts.p,
                                                     sc->nrast, sc->cull, sc->flags, nullptr, nullptr, nullptr, nullptr,
                                                     sc->wit);
      PF_HIP_TRY(hipGetLastError());
    }
  }
  if (attempt == 3) break;
  unsigned int ndrop = 0;
  PF_HIP_TRY(hipMemsetAsync(ndrop_d.p, 0, sizeof(unsigned int), s));
  k_drop_void<<<g256, 256, 0, s>>>(sc->flags, spos.p, prm.occ_logit, prm.sigma_scale, n, sp.p, ndrop_d.p);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(hipMemcpyAsync(&ndrop, ndrop_d.p, sizeof(ndrop), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  if (ndrop == 0) break;
  sc->n_dropped += ndrop;
  }

  k_prep<<<g256, 256, 0, s>>>(prm.p, prm.radius, prm.normal, prm.occ_logit, prm.sigma_scale, n, sc->geo,
                              sc->nrm, sc->cull);
  PF_HIP_TRY(hipGetLastError());
  DevBuf<unsigned long long> cnt(s);
  PF_HIP_TRY(cnt.alloc(6));
  PF_HIP_TRY(hipMemsetAsync(cnt.p, 0, 6 * sizeof(unsigned long long), s));
  k_count_flags<<<g256, 256, 0, s>>>(sc->flags, sc->cull, n, cnt.p);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(hipMemsetAsync(counts.p + n, 0, sizeof(int32_t), s));
  PF_HIP_TRY(exclusive_scan_u32((const uint32_t*)counts.p, (uint32_t*)sc->row, n + 1, nullptr, s));
  uint32_t total = 0;
  unsigned long long hc[6] = {0, 0, 0, 0, 0, 0};
  PF_HIP_TRY(hipMemcpyAsync(&total, sc->row + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipMemcpyAsync(hc, cnt.p, sizeof(hc), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  sc->n_faces = total;
  sc->n_hidden = (int64_t)hc[0];
  sc->n_overflow = (int64_t)hc[1];
  if (sc->n_overflow) {
    set_error("pf_build_scene: " + std::to_string(sc->n_overflow) + " of " + std::to_string(n) +
              " cells exceeded a per-cell capacity (vertices " + std::to_string(hc[2]) + ", planes " +
              std::to_string(hc[3]) + ", work " + std::to_string(hc[4]) + ", stack " + std::to_string(hc[5]) +
              "; " + std::to_string(sc->n_big) + " cells took the high-degree pass)");
    return PF_ERR_OVERFLOW;
  }
  // capacity in steps of 2^18 faces: rebuilds of similar size reuse the pool's blocks
  const size_t fcap = ((size_t)total + (1u << 18)) & ~(size_t)((1u << 18) - 1);
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->col, sizeof(int32_t) * fcap, s));
  PF_HIP_TRY(pf::pool_alloc((void**)&sc->plane, sizeof(float4) * fcap, s));
  k_fill<<<g256, 256, 0, s>>>(prm.p, prm.power, n, faces_tmp.p, faces_big.p, bigslot.p, (const uint32_t*)sc->row,
                              counts.p, bmin, bmax,
                              sc->col, sc->plane);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(hipStreamSynchronize(s));
  return PF_OK;
}

}  // namespace pf
