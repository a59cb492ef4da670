// Octree keys and stable radix sort on the GPU (plan time).
//
// Every interface-anchored point set gets 63-bit Morton keys: x, y and the
// height h above (side 1) or depth below (side 2) its anchoring interface are
// quantised to 21 bits each, q = min(floor((c - c0) * scale), 2^21 - 1), and
// interleaved with h in the top bit of each triple, then y, then x.  A stable
// LSD radix sort (8-bit digits, 8 passes) orders the points; ties keep their
// input order.  The quantisation uses separate IEEE operations (no FMA
// contraction) so the keys are reproducible bit for bit on any IEEE machine.
#include <hip/hip_runtime.h>

#include <string>

#include "fmm_internal.h"

namespace fmmlm {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;  // elements per thread per tile
constexpr int kTile = kSortThreads * kSortRounds;

__device__ inline uint64_t spread21(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ inline uint64_t quant21(double c, double c0, double scale) {
#pragma clang fp contract(off)
  const double t = c - c0;
  const double u = t * scale;
  double f = floor(u);
  if (f < 0.0) f = 0.0;
  if (f > 2097151.0) f = 2097151.0;
  return (uint64_t)f;
}

__global__ void morton_keys_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, const int32_t* __restrict__ idx,
                                   int64_t n, int side, double dref, double x0, double y0,
                                   double scale, uint64_t* __restrict__ keys) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t j = idx[i];
  const double zz = z[j];
  const double h = (side == 1) ? (zz - dref) : (dref - zz);
  const uint64_t qx = quant21(x[j], x0, scale);
  const uint64_t qy = quant21(y[j], y0, scale);
  const uint64_t qh = quant21(h, 0.0, scale);
  keys[i] = (spread21(qh) << 2) | (spread21(qy) << 1) | spread21(qx);
}

__device__ inline unsigned digit_of(uint64_t k, int shift) { return (unsigned)((k >> shift) & 0xffu); }

__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const uint64_t* __restrict__ keys, int64_t n, int shift, int nblk,
                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of hist[0..total) in one workgroup (plan-time sizes)
__global__ void __launch_bounds__(1024) scan_kernel(uint32_t* __restrict__ hist, int64_t total) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (total + 1023) / 1024;
  const int64_t b = t * chunk;
  const int64_t e = (b + chunk < total) ? b + chunk : total;
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const uint32_t v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  uint32_t acc = part[t];
  for (int64_t i = b; i < e; ++i) {
    const uint32_t v = hist[i];
    hist[i] = acc;
    acc += v;
  }
}

__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n,
                     int shift, int nblk, const uint32_t* __restrict__ offs,
                     uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  running[t] = offs[(int64_t)t * nblk + blockIdx.x];
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + t;
    const bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0ull;
    const unsigned dg = digit_of(key, shift);
    // lanes holding the same digit (valid lanes only)
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    if (valid && rank == 0) wcnt[wave][dg] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t o = running[dg] + rank;
      for (int w = 0; w < wave; ++w) o += wcnt[w][dg];
      kout[o] = key;
      vout[o] = vin[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kWaves; ++w) {
      add += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    running[t] += add;
    __syncthreads();
  }
}

}  // namespace

// Keys and stable sort of one anchored point set.  d{x,y,z} are the user
// coordinates on the device; the set's members are given by perm_out on
// entry (user indices, increasing) and replaced by the sorted order.
int gpu_sort_tree(const double* dx, const double* dy, const double* dz, int64_t n, int side,
                  double dref, double x0, double y0, double scale, uint64_t* keys_out,
                  int64_t* perm_out, hipStream_t st, std::string* err) {
  (void)err;
  if (n <= 0) return FMMLM_OK;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int32_t *v0 = nullptr, *v1 = nullptr;
  uint32_t* hist = nullptr;
  const int nblk = (int)((n + kTile - 1) / kTile);
  std::vector<int32_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)perm_out[i];
  int rc = FMMLM_OK;
  auto fail = [&](hipError_t e, const char* what) {
    set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  };
  hipError_t e;
  if ((e = hipMalloc(&k0, n * 8)) != hipSuccess) { fail(e, "hipMalloc keys"); goto done; }
  if ((e = hipMalloc(&k1, n * 8)) != hipSuccess) { fail(e, "hipMalloc keys"); goto done; }
  if ((e = hipMalloc(&v0, n * 4)) != hipSuccess) { fail(e, "hipMalloc vals"); goto done; }
  if ((e = hipMalloc(&v1, n * 4)) != hipSuccess) { fail(e, "hipMalloc vals"); goto done; }
  if ((e = hipMalloc(&hist, (size_t)256 * nblk * 4)) != hipSuccess) { fail(e, "hipMalloc hist"); goto done; }
  if ((e = hipMemcpyAsync(v0, idx.data(), n * 4, hipMemcpyHostToDevice, st)) != hipSuccess) {
    fail(e, "hipMemcpy idx");
    goto done;
  }
  morton_keys_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(dx, dy, dz, v0, n, side, dref, x0, y0,
                                                                   scale, k0);
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    radix_hist_kernel<<<nblk, kSortThreads, 0, st>>>(k0, n, shift, nblk, hist);
    scan_kernel<<<1, 1024, 0, st>>>(hist, (int64_t)256 * nblk);
    radix_scatter_kernel<<<nblk, kSortThreads, 0, st>>>(k0, v0, n, shift, nblk, hist, k1, v1);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  if ((e = hipGetLastError()) != hipSuccess) { fail(e, "radix sort launch"); goto done; }
  if ((e = hipMemcpyAsync(keys_out, k0, n * 8, hipMemcpyDeviceToHost, st)) != hipSuccess) {
    fail(e, "hipMemcpy keys");
    goto done;
  }
  if ((e = hipMemcpyAsync(idx.data(), v0, n * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) {
    fail(e, "hipMemcpy perm");
    goto done;
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) { fail(e, "sort sync"); goto done; }
  for (int64_t i = 0; i < n; ++i) perm_out[i] = idx[i];
done:
  hipFree(k0);
  hipFree(k1);
  hipFree(v0);
  hipFree(v1);
  hipFree(hist);
  return rc;
}

}  // namespace fmmlm
