// Delta-stepping single-source shortest paths (Meyer and Sanders), the
// competitor of Section 5 of arXiv:1506.03265: twice the largest finite
// distance from one source is a 2-approximation of the diameter.
//
// Buckets of width delta: bucket i holds tentative distances in
// [i*delta, (i+1)*delta).  The current bucket is processed by light phases
// (arcs w <= delta, which are the prefix of each weight-sorted row) until it
// stops changing, then one heavy phase relaxes the arcs w > delta of every
// node settled in the bucket.  Improvements beyond the current bucket go to a
// deduplicated far list; when the bucket is done the far list yields the next
// non-empty bucket (minimum over its entries) and is split into that bucket's
// frontier and the remaining far entries.  Distances are exact (u32, with a
// u64 overflow check); the schedule only changes the work.
//
// The host drives the search: it enqueues sweep and control launches in
// batches and polls a done flag (a persistent kernel with grid barriers is
// slower on this device, where each workgroup's device-scope fence writes back
// and invalidates its L2).
#include <string.h>

#include "common.h"

namespace {

constexpr int kT = 256;

enum : uint32_t { S_LIGHT = 0, S_HEAVY = 1, S_MINB = 2, S_SPLIT = 3, S_DONE = 4 };

struct alignas(128) SPad {
  uint32_t v;
  uint32_t pad_[31];
};

struct SCtl {
  uint32_t phase;
  uint32_t sweep_id;
  uint32_t bucket;
  uint32_t far_epoch;
  uint32_t fcur, farcur;
  SPad cntF[2];
  SPad cntR;
  SPad cntFar[2];
  SPad minb;
  uint32_t total;
  uint32_t done;
  uint32_t overflow;
  uint32_t timeout;
  uint32_t sweeps;
  uint32_t pad;
  unsigned long long t_start, t_limit;
  CldBarrier bar;
};

struct SJob {
  const int64_t *rp;
  const uint64_t *arcs;
  int32_t n;
  uint32_t delta;
  uint32_t *dist;
  uint32_t *fstamp, *rstamp, *farstamp;
  int32_t *F[2];
  int32_t *R;
  int32_t *Far[2];
  SCtl *ctl;
};

__device__ void s_control(const SJob &j) {
  if (threadIdx.x != 0) return;
  SCtl *c = j.ctl;
  const uint32_t sweep_id = c->sweep_id + 1;
  if (c->overflow) c->phase = S_DONE;
  const unsigned long long now = wall_clock64();
  if (c->sweeps == 0 && c->t_start == 0) c->t_start = now;
  else if (now - c->t_start > c->t_limit) { c->timeout = 1; c->phase = S_DONE; }
  switch (c->phase) {
    case S_LIGHT:
      c->sweeps++;
      if (c->cntF[c->fcur ^ 1].v > 0) {
        c->cntF[c->fcur].v = 0;
        c->fcur ^= 1;
      } else {
        c->cntF[c->fcur].v = 0;
        c->phase = S_HEAVY;
      }
      break;
    case S_HEAVY:
      c->minb.v = CLD_INF32;
      c->phase = S_MINB;
      break;
    case S_MINB:
      if (c->minb.v == CLD_INF32) {
        c->phase = S_DONE;
      } else {
        c->bucket = c->minb.v;
        c->far_epoch = sweep_id;
        c->cntFar[c->farcur ^ 1].v = 0;
        c->cntF[c->fcur].v = 0;
        c->phase = S_SPLIT;
      }
      break;
    case S_SPLIT:
      c->cntFar[c->farcur].v = 0;
      c->farcur ^= 1;
      c->cntR.v = 0;
      c->phase = S_LIGHT;
      break;
    default:
      break;
  }
  uint32_t t = 0;
  switch (c->phase) {
    case S_LIGHT: t = c->cntF[c->fcur].v; break;
    case S_HEAVY: t = c->cntR.v; break;
    case S_MINB: case S_SPLIT: t = c->cntFar[c->farcur].v; break;
    default: t = 0;
  }
  c->total = t;
  c->done = c->phase == S_DONE;
  c->sweep_id = sweep_id;
}

__device__ __forceinline__ void relax(const SJob &j, SCtl *c, uint64_t nd, int32_t v, uint64_t bucket_end,
                                      uint32_t it, uint32_t far_epoch, uint32_t fnxt, uint32_t farcur) {
  bool tofront = false, tofar = false;
  if (nd >= CLD_INF32) {
    atomicOr(&c->overflow, 1u);
  } else if ((uint32_t)nd < j.dist[v]) {
    const uint32_t old = atomicMin(&j.dist[v], (uint32_t)nd);
    if ((uint32_t)nd < old) {
      if (nd < bucket_end) tofront = j.fstamp[v] != it && atomicExch(&j.fstamp[v], it) != it;
      else tofar = j.farstamp[v] != far_epoch && atomicExch(&j.farstamp[v], far_epoch) != far_epoch;
    }
  }
  uint32_t s1 = cld_wave_reserve(tofront, &c->cntF[fnxt].v);
  if (tofront) j.F[fnxt][s1] = v;
  uint32_t s2 = cld_wave_reserve(tofar, &c->cntFar[farcur].v);
  if (tofar) j.Far[farcur][s2] = v;
}

__device__ void s_item(const SJob &j, uint32_t i, uint32_t phase, uint32_t it) {
  SCtl *c = j.ctl;
  const uint32_t bucket = c->bucket, far_epoch = c->far_epoch, fcur = c->fcur, farcur = c->farcur;
  const uint64_t delta = j.delta;
  const uint64_t bucket_end = ((uint64_t)bucket + 1) * delta;
  switch (phase) {
    case S_LIGHT: {
      const int32_t u = j.F[fcur][i];
      const uint64_t du = j.dist[u];
      bool addr = j.rstamp[u] != bucket + 1 && atomicExch(&j.rstamp[u], bucket + 1) != bucket + 1;
      uint32_t s = cld_wave_reserve(addr, &c->cntR.v);
      if (addr) j.R[s] = u;
      for (int64_t a = j.rp[u]; a < j.rp[u + 1]; ++a) {
        const uint64_t arc = j.arcs[a];
        const uint64_t w = arc >> 32;
        if (w > delta) break;
        relax(j, c, du + w, (int32_t)(uint32_t)arc, bucket_end, it, far_epoch, fcur ^ 1, farcur);
      }
      break;
    }
    case S_HEAVY: {
      const int32_t u = j.R[i];
      const uint64_t du = j.dist[u];
      for (int64_t a = j.rp[u + 1] - 1; a >= j.rp[u]; --a) {
        const uint64_t arc = j.arcs[a];
        const uint64_t w = arc >> 32;
        if (w <= delta) break;
        relax(j, c, du + w, (int32_t)(uint32_t)arc, bucket_end, it, far_epoch, fcur ^ 1, farcur);
      }
      break;
    }
    case S_MINB: {
      const int32_t v = j.Far[farcur][i];
      const uint64_t d = j.dist[v];
      if (d >= bucket_end) {
        const uint32_t b = (uint32_t)(d / delta);
        if (b < c->minb.v) atomicMin(&c->minb.v, b);
      }
      break;
    }
    case S_SPLIT: {
      const int32_t v = j.Far[farcur][i];
      const uint64_t d = j.dist[v];
      const uint64_t b = d / delta;
      const bool tofront = b == bucket && j.fstamp[v] != it && atomicExch(&j.fstamp[v], it) != it;
      const bool tofar = b > bucket && j.farstamp[v] != far_epoch && atomicExch(&j.farstamp[v], far_epoch) != far_epoch;
      uint32_t s1 = cld_wave_reserve(tofront, &c->cntF[fcur].v);
      if (tofront) j.F[fcur][s1] = v;
      uint32_t s2 = cld_wave_reserve(tofar, &c->cntFar[farcur ^ 1].v);
      if (tofar) j.Far[farcur ^ 1][s2] = v;
      break;
    }
    default:
      break;
  }
}

__device__ void s_sweep(const SJob &j, uint32_t block, uint32_t nblocks) {
  const uint32_t total = j.ctl->total, phase = j.ctl->phase, it = j.ctl->sweep_id;
  const uint32_t stride = nblocks * blockDim.x;
  // whole waves stay in the loop so that wave-wide reservations see every lane
  for (uint32_t base = block * blockDim.x; base < total; base += stride) {
    const uint32_t i = base + threadIdx.x;
    if (i < total) s_item(j, i, phase, it);
  }
}

__global__ void __launch_bounds__(kT) k_sssp_init(SJob j, int32_t src, unsigned long long t_limit) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < j.n; v += (int64_t)gridDim.x * blockDim.x) {
    j.dist[v] = v == src ? 0u : CLD_INF32;
    j.fstamp[v] = 0; j.rstamp[v] = 0; j.farstamp[v] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SCtl *c = j.ctl;
    memset(c, 0, sizeof(SCtl));
    c->phase = S_LIGHT;
    c->far_epoch = 1;
    c->sweep_id = 1;
    c->cntF[0].v = 1;
    c->total = 1;
    c->t_limit = t_limit;
    j.F[0][0] = src;
  }
}

__global__ void __launch_bounds__(kT) k_sssp_sweep(SJob j) {
  if (j.ctl->done) return;
  s_sweep(j, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kT) k_sssp_control(SJob j) {
  if (j.ctl->done) return;
  s_control(j);
}

__global__ void __launch_bounds__(kT) k_sssp_max(const uint32_t *dist, int32_t n, unsigned long long *mx) {
  unsigned long long m = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (dist[v] != CLD_INF32 && dist[v] > m) m = dist[v];
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long x = __shfl_xor(m, o);
    m = x > m ? x : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax(mx, m);
}

// Sum of all arc weights (the high words of the packed arcs), for the default
// bucket width.
__global__ void __launch_bounds__(kT) k_sssp_weight_sum(const uint64_t *arcs, int64_t m, unsigned long long *sum) {
  unsigned long long s = 0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m; a += (int64_t)gridDim.x * blockDim.x)
    s += arcs[a] >> 32;
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(sum, s);
}

// Default bucket width: kDefaultWidth mean arc weights (at least 1, at most
// 2^31); 1 on a graph without arcs.
constexpr uint64_t kDefaultWidth = 16;

}  // namespace

extern "C" size_t cldiam_sssp_workspace_size(int32_t n, int64_t m) {
  (void)m;
  if (n < 1) return 0;
  cld::Sizer s;
  s.take<SCtl>(1);
  s.take<unsigned long long>(1);
  for (int i = 0; i < 3; ++i) s.take<uint32_t>((size_t)n);
  for (int i = 0; i < 5; ++i) s.take<int32_t>((size_t)n);
  return s.used;
}

extern "C" int cldiam_sssp_delta_stepping(int32_t n, int64_t m, const int64_t *d_row_ptr, const uint64_t *d_arcs,
                                          int32_t source, uint32_t bucket_delta, uint32_t *d_dist,
                                          uint64_t *h_max_dist, void *ws, size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (n < 1 || m < 0 || source < 0 || source >= n || !d_row_ptr || (m && !d_arcs) || !d_dist || !h_max_dist) {
    cld::set_error("sssp: invalid arguments");
    return CLDIAM_EINVAL;
  }
  cld::Arena a(ws, ws_bytes);
  SJob j;
  j.ctl = a.take<SCtl>(1);
  unsigned long long *mx = a.take<unsigned long long>(1);
  j.fstamp = a.take<uint32_t>((size_t)n);
  j.rstamp = a.take<uint32_t>((size_t)n);
  j.farstamp = a.take<uint32_t>((size_t)n);
  j.F[0] = a.take<int32_t>((size_t)n);
  j.F[1] = a.take<int32_t>((size_t)n);
  j.R = a.take<int32_t>((size_t)n);
  j.Far[0] = a.take<int32_t>((size_t)n);
  j.Far[1] = a.take<int32_t>((size_t)n);
  if (!j.Far[1]) {
    cld::set_error("sssp: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_sssp_workspace_size(n, m));
    return CLDIAM_ENOMEM;
  }
  if (bucket_delta == 0) {
    // default width from the mean arc weight (mx serves as the sum's slot)
    uint64_t wsum = 0;
    if (m > 0) {
      CLD_HIP(hipMemsetAsync(mx, 0, 8, stream));
      k_sssp_weight_sum<<<cld::blocks_for(m, kT, 4096), kT, 0, stream>>>(d_arcs, m, mx);
      CLD_LAUNCH_CHECK("k_sssp_weight_sum");
      unsigned long long hs = 0;
      CLD_HIP(hipMemcpyAsync(&hs, mx, 8, hipMemcpyDeviceToHost, stream));
      CLD_HIP(hipStreamSynchronize(stream));
      wsum = hs;
    }
    uint64_t b = m > 0 ? kDefaultWidth * (wsum / (uint64_t)m) : 1;
    if (b < 1) b = 1;
    if (b > CLD_DELTA_MAX) b = CLD_DELTA_MAX;
    bucket_delta = (uint32_t)b;
  }
  j.rp = d_row_ptr;
  j.arcs = d_arcs;
  j.n = n;
  j.delta = bucket_delta;
  j.dist = d_dist;
  int dev = 0, khz = 0, cus = 0;
  CLD_HIP(hipGetDevice(&dev));
  CLD_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  CLD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (khz <= 0) khz = 100000;
  const int blocks = 4 * cus;
  k_sssp_init<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(j, source, (unsigned long long)khz * 1000ull * 60ull);
  CLD_LAUNCH_CHECK("k_sssp_init");
  SCtl hc;
  int batch = 8;
  for (;;) {
    for (int i = 0; i < batch; ++i) {
      k_sssp_sweep<<<blocks, kT, 0, stream>>>(j);
      k_sssp_control<<<1, 64, 0, stream>>>(j);
    }
    CLD_LAUNCH_CHECK("k_sssp_sweep");
    CLD_HIP(hipMemcpyAsync(&hc, j.ctl, sizeof hc, hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (hc.done || hc.timeout) break;
    if (batch < 128) batch *= 2;
  }
  CLD_HIP(hipMemsetAsync(mx, 0, 8, stream));
  k_sssp_max<<<cld::blocks_for(n, kT, 4096), kT, 0, stream>>>(d_dist, n, mx);
  CLD_LAUNCH_CHECK("k_sssp_max");
  unsigned long long hm = 0;
  CLD_HIP(hipMemcpyAsync(&hm, mx, 8, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  if (hc.timeout) { cld::set_error("sssp: grid barrier timed out"); return CLDIAM_ETIMEOUT; }
  if (hc.overflow) { cld::set_error("sssp: a distance does not fit in 32 bits"); return CLDIAM_EOVERFLOW; }
  if (!hc.done) { cld::set_error("sssp: persistent kernel ended early"); return CLDIAM_EHIP; }
  *h_max_dist = hm;
  return CLDIAM_OK;
}
