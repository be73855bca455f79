// Device primitives: exclusive prefix sum and LSD radix sort (gfx950, wave64).
//
// Scan: reduce-then-scan over tiles of 4096 elements (256 threads x 16),
// recursive over the tile sums.
//
// Radix sort: 8-bit digits, three kernels per pass (tile histograms, scan of
// the digit-major histogram table, stable scatter).  The scatter ranks each
// 256-element sub-tile with 64-lane ballots (the lanes holding the same digit
// are found by eight ballots over the digit bits) and per-wave digit counts in
// LDS, so the sort is stable and deterministic.
#include "common.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *in, int64_t n, uint32_t *sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Each thread owns 16 consecutive items of the tile.
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const uint32_t *in, int64_t n, const uint32_t *offs,
                                                            uint32_t *out, uint32_t *total_out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? in[i] : 0;
    s += v[j];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, &total) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total_out = run;
}

// ------------------------------------------------------------ radix sort --

constexpr int kRsThreads = 256;
constexpr int kRsSub = 16;                       // sub-tiles per tile
constexpr int kRsTile = kRsThreads * kRsSub;     // 4096

__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                         uint32_t *hist, uint32_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int j = 0; j < kRsSub; ++j) {
    int64_t i = base + (int64_t)j * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint64_t *kin, const uint64_t *vin, int64_t n,
                                                            int shift, const uint32_t *offs, uint32_t nb,
                                                            uint64_t *kout, uint64_t *vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kRsThreads / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  run[threadIdx.x] = offs[(size_t)threadIdx.x * nb + blockIdx.x];
  for (int w = 0; w < kRsThreads / 64; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int j = 0; j < kRsSub; ++j) {
    const int64_t i = base + (int64_t)j * kRsThreads + threadIdx.x;
    const bool valid = i < n;
    uint64_t k = valid ? kin[i] : 0;
    uint64_t v = (valid && vin) ? vin[i] : 0;
    const uint32_t dgt = (uint32_t)(k >> shift) & 255u;
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long bb = __ballot((dgt >> b) & 1u);
      same &= ((dgt >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    if (valid && rank == 0) wcnt[wave][dgt] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dgt] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dgt];
      kout[pos] = k;
      if (vin) vout[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kRsThreads / 64; ++w) { add += wcnt[w][threadIdx.x]; wcnt[w][threadIdx.x] = 0; }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

namespace cld {

size_t scan_ws_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > 1) {
    m = (m + kScanTile - 1) / kScanTile;
    total += ((size_t)m * 4 + 255) & ~(size_t)255;
  }
  return total + 256;
}

// out[i] = sum of in[0..i); *d_total (device, optional) = sum of all.
int scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  if (n <= 0) {
    if (d_total) CLD_HIP(hipMemsetAsync(d_total, 0, 4, stream));
    return CLDIAM_OK;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_down<<<1, kScanThreads, 0, stream>>>(in, n, nullptr, out, d_total);
    CLD_LAUNCH_CHECK("k_scan_down");
    return CLDIAM_OK;
  }
  Arena a(ws, ws_bytes);
  uint32_t *sums = a.take<uint32_t>((size_t)nb);
  if (!sums) { set_error("scan: workspace too small"); return CLDIAM_ENOMEM; }
  k_scan_reduce<<<(unsigned)nb, kScanThreads, 0, stream>>>(in, n, sums);
  CLD_LAUNCH_CHECK("k_scan_reduce");
  // scan the tile sums in place (recursively, with the rest of the workspace)
  int rc = scan_exclusive_u32(sums, sums, nb, nullptr, a.base + a.used, a.cap - a.used, stream);
  if (rc) return rc;
  k_scan_down<<<(unsigned)nb, kScanThreads, 0, stream>>>(in, n, sums, out, d_total);
  CLD_LAUNCH_CHECK("k_scan_down");
  return CLDIAM_OK;
}

size_t radix_ws_bytes(int64_t n) {
  const int64_t nb = (n + kRsTile - 1) / kRsTile;
  const int64_t hn = nb * 256;
  return (((size_t)hn * 4 + 255) & ~(size_t)255) * 2 + scan_ws_bytes(hn);
}

// Sorts keys (and values) by bits [begin_bit, end_bit) of the key; stable.
// Ping-pongs with ktmp/vtmp; *in_tmp tells where the result ended.
int radix_sort_u64(uint64_t *keys, uint64_t *vals, int64_t n, int begin_bit, int end_bit, uint64_t *ktmp,
                   uint64_t *vtmp, bool *in_tmp, void *ws, size_t ws_bytes, hipStream_t stream) {
  *in_tmp = false;
  if (n <= 1 || begin_bit >= end_bit) return CLDIAM_OK;
  const int64_t nb64 = (n + kRsTile - 1) / kRsTile;
  if (nb64 > 0x7fffffff / 256) { set_error("radix sort: too many elements"); return CLDIAM_EINVAL; }
  const uint32_t nb = (uint32_t)nb64;
  Arena a(ws, ws_bytes);
  uint32_t *hist = a.take<uint32_t>((size_t)nb * 256);
  uint32_t *offs = a.take<uint32_t>((size_t)nb * 256);
  if (!hist || !offs) { set_error("radix sort: workspace too small"); return CLDIAM_ENOMEM; }
  uint64_t *ks = keys, *vs = vals, *kd = ktmp, *vd = vtmp;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    k_rs_hist<<<nb, kRsThreads, 0, stream>>>(ks, n, shift, hist, nb);
    CLD_LAUNCH_CHECK("k_rs_hist");
    int rc = scan_exclusive_u32(hist, offs, (int64_t)nb * 256, nullptr, a.base + a.used, a.cap - a.used, stream);
    if (rc) return rc;
    k_rs_scatter<<<nb, kRsThreads, 0, stream>>>(ks, vals ? vs : nullptr, n, shift, offs, nb, kd, vals ? vd : nullptr);
    CLD_LAUNCH_CHECK("k_rs_scatter");
    uint64_t *t = ks; ks = kd; kd = t;
    t = vs; vs = vd; vd = t;
    *in_tmp = !*in_tmp;
  }
  return CLDIAM_OK;
}

}  // namespace cld
