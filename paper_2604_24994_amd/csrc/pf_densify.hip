// Densification and pruning (Sec. 3.5): moving averages of the per-cell
// error and contribution, removal of cells whose contribution average is
// below a threshold, and new cells drawn from the multinomial distribution
// proportional to the error average of the remaining cells.
//
// Steps on the device: keep flags and their prefix sum (kept cells stay in
// order); the kept cells' error averages in float64 and their inclusive
// prefix sum (tiles of 2048, then one workgroup over the tile totals); one
// binary search per draw for the first cumulative weight above u * total;
// row copies of every parameter array for the kept cells and for the new
// cells (copies of their parents, moved by spread * r * delta).
#include "pf_internal.hpp"

namespace pf {

namespace {

constexpr int DT = 256;            // threads per block
constexpr int DI = 8;              // items per thread in the scan tiles
constexpr int DTILE = DT * DI;

template <typename T>
struct Tmp {
  T* p = nullptr;
  hipStream_t s;
  explicit Tmp(hipStream_t st) : s(st) {}
  ~Tmp() { if (p) pf::pool_free(p, s); }
  hipError_t alloc(size_t count) { return pf::pool_alloc((void**)&p, sizeof(T) * (count ? count : 1), s); }
};

__global__ void k_ema(float* __restrict__ ema, const float* __restrict__ value, int64_t n, float beta) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = beta;
  ema[i] = __double2float_rn(b * (double)ema[i] + (1.0 - b) * (double)value[i]);
}

__global__ void k_keep(const float* __restrict__ contrib, int64_t n, float below, uint32_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keep[i] = contrib[i] >= below ? 1u : 0u;
}

__global__ void k_kept_index(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ pos, int64_t n,
                             const float* __restrict__ err, int32_t* __restrict__ kidx, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && keep[i]) {
    kidx[pos[i]] = (int32_t)i;
    w[pos[i]] = (double)err[i];
  }
}

// Block-wide inclusive scan of one double per thread (fixed order).
__device__ inline double block_incl_scan_d(double x, double* total) {
  __shared__ double ws[DT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wv] = x;
  __syncthreads();
  double off = 0.0, tot = 0.0;
  for (int k = 0; k < DT / 64; ++k) {
    if (k < wv) off += ws[k];
    tot += ws[k];
  }
  __syncthreads();
  *total = tot;
  return off + x;
}

// Inclusive prefix sums within tiles of DTILE values; tile totals to tsum.
__global__ void __launch_bounds__(DT) k_dscan_tile(double* __restrict__ w, int64_t n, double* __restrict__ tsum) {
  const int64_t base = (int64_t)blockIdx.x * DTILE + (int64_t)threadIdx.x * DI;
  double v[DI];
  double run = 0.0;
  for (int k = 0; k < DI; ++k) {
    v[k] = base + k < n ? w[base + k] : 0.0;
    run += v[k];
    v[k] = run;
  }
  double tot;
  const double incl = block_incl_scan_d(run, &tot);
  const double excl = incl - run;
  for (int k = 0; k < DI; ++k)
    if (base + k < n) w[base + k] = excl + v[k];
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// Exclusive prefix of the tile totals, one workgroup, in order.
__global__ void __launch_bounds__(DT) k_dscan_tiles(double* __restrict__ tsum, int64_t ntile) {
  double carry = 0.0;
  for (int64_t b = 0; b < ntile; b += DT) {
    const int64_t i = b + threadIdx.x;
    const double x = i < ntile ? tsum[i] : 0.0;
    double tot;
    const double incl = block_incl_scan_d(x, &tot);
    if (i < ntile) tsum[i] = carry + incl - x;
    carry += tot;
  }
}

__global__ void k_dscan_add(double* __restrict__ w, int64_t n, const double* __restrict__ tsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] += tsum[i / DTILE];
}

// One draw per thread: the first kept position whose cumulative weight
// exceeds u * total (zero-weight cells are never drawn).
__global__ void k_draw(const double* __restrict__ cdf, int64_t nk, const float* __restrict__ u, int64_t nd,
                       const int32_t* __restrict__ kidx, int32_t* __restrict__ parent) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  const double x = (double)u[k] * cdf[nk - 1];
  int64_t lo = 0, hi = nk - 1;   // answer in [lo, hi]
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cdf[mid] > x) hi = mid;
    else lo = mid + 1;
  }
  parent[k] = kidx[lo];
}

// Row copies of the small per-cell arrays: rows [0, nk) from the kept cells,
// rows [nk, nk + nd) from the parents (position moved).
__global__ void k_copy_rows(pf_params in, pf_cell_arrays out, const int32_t* __restrict__ kidx, int64_t nk,
                            const int32_t* __restrict__ parent, const float* __restrict__ delta, int64_t nd,
                            float spread, const float* __restrict__ ea, const float* __restrict__ ca,
                            float* __restrict__ oea, float* __restrict__ oca) {
#pragma clang fp contract(off)
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nk + nd) return;
  const bool child = r >= nk;
  const int64_t i = child ? parent[r - nk] : kidx[r];
  for (int a = 0; a < 3; ++a) {
    float pv = in.p[3 * i + a];
    if (child) {
      const double t = (double)spread * (double)in.radius[i];
      pv = __double2float_rn((double)pv + t * (double)delta[3 * (r - nk) + a]);
    }
    out.p[3 * r + a] = pv;
    out.normal[3 * r + a] = in.normal[3 * i + a];
    out.rgb[3 * r + a] = in.rgb[3 * i + a];
  }
  out.power[r] = in.power[i];
  out.radius[r] = in.radius[i];
  out.occ_logit[r] = in.occ_logit[i];
  oea[r] = ea[i];
  oca[r] = ca[i];
}

// Texture rows, one thread per float.
__global__ void k_copy_tex(const float* __restrict__ tin, float* __restrict__ tout, const int32_t* __restrict__ kidx,
                           int64_t nk, const int32_t* __restrict__ parent, int64_t nd, int row) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (nk + nd) * row) return;
  const int64_t r = t / row, c = t - r * row;
  const int64_t i = r >= nk ? parent[r - nk] : kidx[r];
  tout[t] = tin[i * row + c];
}

}  // namespace

pf_status ema_impl(float* ema, const float* value, int64_t n, float beta, hipStream_t s) {
  k_ema<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ema, value, n, beta);
  PF_HIP_TRY(hipGetLastError());
  return PF_OK;
}

pf_status densify_impl(const pf_params& in, const float* err_ema, const float* contrib_ema, const float* u,
                       const float* delta, const pf_densify_opts& o, const pf_cell_arrays& out, float* out_err,
                       float* out_contrib, int32_t* out_parent, int64_t* n_kept, int64_t* n_drawn, hipStream_t s) {
  const int64_t n = in.n;
  const unsigned g = (unsigned)((n + 255) / 256);
  Tmp<uint32_t> keep(s), pos(s), kept_d(s);
  Tmp<int32_t> kidx(s), parent(s);
  Tmp<double> w(s), tsum(s);
  PF_HIP_TRY(keep.alloc(n));
  PF_HIP_TRY(pos.alloc(n));
  PF_HIP_TRY(kept_d.alloc(1));
  PF_HIP_TRY(kidx.alloc(n));
  PF_HIP_TRY(w.alloc(n));
  k_keep<<<g, 256, 0, s>>>(contrib_ema, n, o.prune_below, keep.p);
  PF_HIP_TRY(hipGetLastError());
  PF_HIP_TRY(exclusive_scan_u32(keep.p, pos.p, n, kept_d.p, s));
  k_kept_index<<<g, 256, 0, s>>>(keep.p, pos.p, n, err_ema, kidx.p, w.p);
  PF_HIP_TRY(hipGetLastError());
  uint32_t nk32 = 0;
  PF_HIP_TRY(hipMemcpyAsync(&nk32, kept_d.p, sizeof(nk32), hipMemcpyDeviceToHost, s));
  PF_HIP_TRY(hipStreamSynchronize(s));
  const int64_t nk = nk32;
  int64_t nd = nk > 0 ? o.n_new : 0;
  if (nd > 0) {
    const int64_t ntile = (nk + DTILE - 1) / DTILE;
    PF_HIP_TRY(tsum.alloc(ntile));
    k_dscan_tile<<<(unsigned)ntile, DT, 0, s>>>(w.p, nk, tsum.p);
    k_dscan_tiles<<<1, DT, 0, s>>>(tsum.p, ntile);
    k_dscan_add<<<(unsigned)((nk + 255) / 256), 256, 0, s>>>(w.p, nk, tsum.p);
    PF_HIP_TRY(hipGetLastError());
    double total = 0.0;
    PF_HIP_TRY(hipMemcpyAsync(&total, w.p + nk - 1, sizeof(total), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    if (!(total > 0.0)) nd = 0;
  }
  if (nd > 0) {
    PF_HIP_TRY(parent.alloc(nd));
    k_draw<<<(unsigned)((nd + 255) / 256), 256, 0, s>>>(w.p, nk, u, nd, kidx.p, parent.p);
    PF_HIP_TRY(hipGetLastError());
    if (out_parent)
      PF_HIP_TRY(hipMemcpyAsync(out_parent, parent.p, sizeof(int32_t) * nd, hipMemcpyDeviceToDevice, s));
  }
  const int64_t rows = nk + nd;
  if (rows > 0) {
    k_copy_rows<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(in, out, kidx.p, nk, parent.p, delta, nd, o.spread,
                                                               err_ema, contrib_ema, out_err, out_contrib);
    PF_HIP_TRY(hipGetLastError());
    const int row = in.k_detail * (3 + 6 * in.m_axes);
    const int64_t nt = rows * row;
    k_copy_tex<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(in.tex, out.tex, kidx.p, nk, parent.p, nd, row);
    PF_HIP_TRY(hipGetLastError());
  }
  *n_kept = nk;
  *n_drawn = nd;
  return PF_OK;
}

}  // namespace pf
