// Device-wide exclusive scan and stable LSD radix sort for wave64 (gfx950).
//
// Scan: reduce-then-scan over blocks of 256 threads x 8 items, recursive on
// the block sums.  Radix sort: 8-bit digits; per pass a block histogram, a
// digit-major scan of all block histograms, and a stable scatter that ranks
// equal digits inside a wave with ballot-based matching.
#include "pf_internal.hpp"

#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace pf {

// Device blocks come from the caller's allocator when one is set
// (pf_set_allocator), else from a cache of the library's own: a freed block
// is kept, with an event recorded on the stream that freed it, and handed
// out again to an allocation of at most twice its size on that stream
// (stream order makes it safe), or on another stream once the event has
// completed (no stream waits on another, so concurrent streams stay
// independent).  The runtime is asked for memory only on a miss; blocks go
// back to it when the cache exceeds its limit or an allocation fails.
// Either way the requested bytes of the blocks in use, and their high-water
// mark, are counted (pf_memory_stats).
namespace {
struct CachedBlock {
  void* p;
  size_t bytes;
  int dev;
  hipEvent_t ev;
  hipStream_t freed_on;
};
struct LiveBlock {
  size_t bytes;          // block size (the cache's rounding), or the request for a caller block
  size_t req;            // requested bytes
  int dev;
  bool caller;           // from the caller's allocator
  pf_allocator a;        // that allocator
};
std::mutex g_cache_mu;
std::multimap<size_t, CachedBlock> g_cache;                  // free blocks by size
std::unordered_map<void*, LiveBlock> g_live;                 // handed-out blocks
size_t g_cached_bytes = 0;
size_t g_cache_limit = size_t(48) << 30;
pf_allocator g_alloc{};                                      // caller's allocator (alloc == NULL: none)
int64_t g_live_req = 0, g_peak_req = 0;                      // requested bytes in use, high-water mark

void account(int64_t delta) {
  g_live_req += delta;
  if (g_live_req > g_peak_req) g_peak_req = g_live_req;
}

size_t round_bytes(size_t bytes) {
  // above 1 MiB in steps of 1/16 of the power of two (at most 6.25% more)
  if (bytes <= (1u << 20)) return bytes < 256 ? 256 : (bytes + 255) & ~size_t(255);
  size_t pw = 1;
  while (pw < bytes) pw <<= 1;
  const size_t step = pw >> 4;
  return (bytes + step - 1) / step * step;
}

void release_block(const CachedBlock& b) {
  (void)hipEventSynchronize(b.ev);
  (void)hipEventDestroy(b.ev);
  (void)hipFree(b.p);
}

// Returns the cached blocks of device dev to the runtime.
void flush_device(int dev) {
  std::vector<CachedBlock> out;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
      if (it->second.dev == dev) {
        out.push_back(it->second);
        g_cached_bytes -= it->second.bytes;
        it = g_cache.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (const CachedBlock& b : out) release_block(b);
}
}  // namespace

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  const size_t req = bytes;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  pf_allocator a{};
  {
    std::unique_lock<std::mutex> lk(g_cache_mu);
    a = g_alloc;
    if (!a.alloc) {
      bytes = round_bytes(bytes);
      for (auto it = g_cache.lower_bound(bytes); it != g_cache.end() && it->first <= 2 * bytes; ++it) {
        if (it->second.dev != dev) continue;
        if (it->second.freed_on != s && hipEventQuery(it->second.ev) != hipSuccess) {
          (void)hipGetLastError();   // "not ready" is not an error of the caller's
          continue;
        }
        const CachedBlock b = it->second;
        g_cache.erase(it);
        g_cached_bytes -= b.bytes;
        g_live[b.p] = LiveBlock{b.bytes, req, dev, false, {}};
        account((int64_t)req);
        lk.unlock();
        (void)hipEventDestroy(b.ev);
        *p = b.p;
        return hipSuccess;
      }
    }
  }
  if (a.alloc) {
    *p = a.alloc(a.ctx, req, (void*)s);
    if (!*p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_live[*p] = LiveBlock{req, req, dev, true, a};
    account((int64_t)req);
    return hipSuccess;
  }
  e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    flush_device(dev);
    e = hipMalloc(p, bytes);
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_live[*p] = LiveBlock{bytes, req, dev, false, {}};
    account((int64_t)req);
  }
  return e;
}

void pool_free(void* p, hipStream_t s) {
  if (!p) return;
  CachedBlock b{p, 0, 0, nullptr, s};
  LiveBlock lb{};
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;   // not from pool_alloc: nothing to do
    lb = it->second;
    b.bytes = lb.bytes;
    b.dev = lb.dev;
    g_live.erase(it);
    account(-(int64_t)lb.req);
  }
  if (lb.caller) {
    lb.a.free(lb.a.ctx, p, lb.req, (void*)s);
    return;
  }
  if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(b.ev, s) != hipSuccess) {
    if (b.ev) (void)hipEventDestroy(b.ev);
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    return;
  }
  std::vector<CachedBlock> out;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.insert({b.bytes, b});
    g_cached_bytes += b.bytes;
    while (g_cached_bytes > g_cache_limit && !g_cache.empty()) {
      auto last = std::prev(g_cache.end());
      out.push_back(last->second);
      g_cached_bytes -= last->second.bytes;
      g_cache.erase(last);
    }
  }
  for (const CachedBlock& v : out) release_block(v);
}

void set_allocator(const pf_allocator* a) {
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_alloc = a ? *a : pf_allocator{};
  }
  int dev = 0;
  if (a && hipGetDevice(&dev) == hipSuccess) flush_device(dev);   // the caller's allocator gets the memory
}

void set_cache_limit(size_t bytes) {
  std::vector<CachedBlock> out;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache_limit = bytes;
    while (g_cached_bytes > g_cache_limit && !g_cache.empty()) {
      auto last = std::prev(g_cache.end());
      out.push_back(last->second);
      g_cached_bytes -= last->second.bytes;
      g_cache.erase(last);
    }
  }
  for (const CachedBlock& v : out) release_block(v);
}

void memory_stats(int64_t* live, int64_t* peak, int64_t* cached, bool reset_peak) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (live) *live = g_live_req;
  if (peak) *peak = g_peak_req;
  if (cached) *cached = (int64_t)g_cached_bytes;
  if (reset_peak) g_peak_req = g_live_req;
}

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t v = __shfl_up(x, o, 64);
    if (lane >= o) x += v;
  }
  return x;
}

// Block-wide exclusive scan of one value per thread; returns the block total
// through *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_inclusive_scan(x);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / 64; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - x;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_block_sums(const uint32_t* __restrict__ in, int64_t n,
                                                             uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_block_apply(const uint32_t* in, int64_t n,
                                                              const uint32_t* __restrict__ offs,
                                                              uint32_t* out, uint32_t* total_dev) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) *total_dev = run;
}

}  // namespace

int64_t scan_scratch_bytes(int64_t n) {
  int64_t b = 0;
  while (n > 0) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) break;
    b += (int64_t)sizeof(uint32_t) * nb;
    n = nb;
  }
  return b;
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
                              hipStream_t s) {
  if (n <= 0) {
    if (total_dev) return hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s);
    return hipSuccess;
  }
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    k_block_apply<<<1, SCAN_THREADS, 0, s>>>(in, n, nullptr, out, total_dev);
    return hipGetLastError();
  }
  uint32_t* sums = nullptr;
  hipError_t e = pf::pool_alloc((void**)&sums, sizeof(uint32_t) * nb, s);
  if (e != hipSuccess) return e;
  k_block_sums<<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, sums);
  e = exclusive_scan_u32(sums, sums, nb, nullptr, s);
  if (e == hipSuccess) {
    k_block_apply<<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, sums, out, total_dev);
    e = hipGetLastError();
  }
  pf::pool_free(sums, s);
  return e;
}

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / 64;

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                        int shift, int64_t nblocks,
                                                        uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: within a round of 256 consecutive keys, a key's rank among
// equal digits is (earlier waves' counts) + (lower lanes of its own wave).
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin, int64_t n,
                                                           int shift, int64_t nblocks,
                                                           const uint32_t* __restrict__ hist_scan,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RS_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  run[threadIdx.x] = hist_scan[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) wcnt[q][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    const bool ok = i < n;
    uint32_t key = ok ? kin[i] : 0u, val = ok ? vin[i] : 0u;
    uint32_t dig = (key >> shift) & 255u;
    uint64_t match = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot(ok && ((dig >> b) & 1u));
      match &= ((dig >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(match & lt);
    if (ok && rank == 0) wcnt[w][dig] = (uint32_t)__popcll(match);
    __syncthreads();
    if (ok) {
      uint32_t off = run[dig] + rank;
      for (int q = 0; q < w; ++q) off += wcnt[q][dig];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) add += wcnt[q][threadIdx.x];
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  uint32_t *k2 = nullptr, *v2 = nullptr, *hist = nullptr;
  hipError_t e = pf::pool_alloc((void**)&k2, sizeof(uint32_t) * n, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&v2, sizeof(uint32_t) * n, s);
  if (e == hipSuccess) e = pf::pool_alloc((void**)&hist, sizeof(uint32_t) * 256 * nb, s);
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  int passes = 0;
  for (int shift = 0; e == hipSuccess && shift < bits; shift += 8, ++passes) {
    k_rs_hist<<<(unsigned)nb, RS_THREADS, 0, s>>>(ka, n, shift, nb, hist);
    e = exclusive_scan_u32(hist, hist, 256 * nb, nullptr, s);
    if (e != hipSuccess) break;
    k_rs_scatter<<<(unsigned)nb, RS_THREADS, 0, s>>>(ka, va, n, shift, nb, hist, kb, vb);
    e = hipGetLastError();
    uint32_t* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  if (e == hipSuccess && (passes & 1)) {
    e = hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
  }
  if (k2) pf::pool_free(k2, s);
  if (v2) pf::pool_free(v2, s);
  if (hist) pf::pool_free(hist, s);
  return e;
}

}  // namespace pf
