// Diameter estimate (Section 4 of arXiv:1506.03265):
//   Phi_approx = Phi(G_C) + 2 * radius,
// where Phi(G_C) is the largest finite shortest-path distance between two
// nodes of the quotient graph.  G_C is small (the number of clusters), so it
// is solved exactly: every workgroup runs single-source shortest paths from
// one quotient node at a time (label-correcting relaxation with a
// deduplicated queue; all distances exact at the fixpoint), keeping distances
// and queues in LDS when they fit, in a per-workgroup workspace slice
// otherwise.
#include <mutex>
#include <vector>

#include "common.h"

namespace {

constexpr int kT = 256;
constexpr int kLdsMaxK = 3072;  // 20 bytes per node -> 60 KB

struct ECtl {
  unsigned long long phi;
  uint32_t bad;   // the quotient CSR is malformed: nothing is indexed with it
  uint32_t pad;
};

// The quotient CSR must have row offsets from 0 to qm, non-decreasing, and
// columns in [0, k); anything else fails the call before the APSP reads it.
__global__ void k_check_quotient(int32_t k, int64_t qm, const int64_t *rp, const int32_t *col, uint32_t *bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
    bool ok = rp[i] <= rp[i + 1];
    if (i == 0) ok = ok && rp[0] == 0;
    if (i == k - 1) ok = ok && rp[k] == qm;
    if (!ok) *bad = 1u;
  }
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < qm; a += stride)
    if ((uint32_t)col[a] >= (uint32_t)k) *bad = 1u;
}

__device__ void sssp_block(int32_t k, const int64_t *rp, const int32_t *col, const uint64_t *w, int32_t s,
                           uint64_t *dist, uint32_t *stamp, int32_t *q0, int32_t *q1, uint64_t *phi) {
  __shared__ uint32_t qn_next;
  __shared__ unsigned long long bmax;
  for (int32_t v = threadIdx.x; v < k; v += blockDim.x) { dist[v] = CLD_INF64; stamp[v] = 0; }
  if (threadIdx.x == 0) { qn_next = 0; bmax = 0; }
  __syncthreads();
  if (threadIdx.x == 0) { dist[s] = 0; q0[0] = s; }
  __syncthreads();
  uint32_t qn = 1, iter = 1;
  int32_t *qc = q0, *qx = q1;
  while (qn > 0) {
    for (uint32_t i = threadIdx.x; i < qn; i += blockDim.x) {
      const int32_t u = qc[i];
      const uint64_t du = dist[u];
      for (int64_t a = rp[u]; a < rp[u + 1]; ++a) {
        const int32_t v = col[a];
        const uint64_t nd = du + w[a];
        if (nd < dist[v]) {
          const uint64_t old = atomicMin((unsigned long long *)&dist[v], (unsigned long long)nd);
          if (nd < old && atomicExch(&stamp[v], iter) != iter) qx[atomicAdd(&qn_next, 1u)] = v;
        }
      }
    }
    __syncthreads();
    qn = qn_next;
    __syncthreads();
    if (threadIdx.x == 0) qn_next = 0;
    int32_t *t = qc; qc = qx; qx = t;
    ++iter;
    __syncthreads();
  }
  unsigned long long m = 0;
  for (int32_t v = threadIdx.x; v < k; v += blockDim.x)
    if (dist[v] != CLD_INF64 && dist[v] > m) m = dist[v];
  atomicMax(&bmax, m);
  __syncthreads();
  if (threadIdx.x == 0 && bmax) atomicMax((unsigned long long *)phi, bmax);
  __syncthreads();
}

__global__ void __launch_bounds__(kT) k_apsp_lds(int32_t k, const int64_t *rp, const int32_t *col,
                                                 const uint64_t *w, uint64_t *phi, const uint32_t *bad) {
  if (*bad) return;
  extern __shared__ uint64_t lds[];
  uint64_t *dist = lds;
  uint32_t *stamp = (uint32_t *)(dist + k);
  int32_t *q0 = (int32_t *)(stamp + k);
  int32_t *q1 = q0 + k;
  for (int32_t s = blockIdx.x; s < k; s += gridDim.x) sssp_block(k, rp, col, w, s, dist, stamp, q0, q1, phi);
}

__global__ void __launch_bounds__(kT) k_apsp_global(int32_t k, const int64_t *rp, const int32_t *col,
                                                    const uint64_t *w, uint64_t *phi, char *slices,
                                                    const uint32_t *bad) {
  if (*bad) return;
  const size_t per = (size_t)k * 20;
  char *base = slices + per * blockIdx.x;
  uint64_t *dist = (uint64_t *)base;
  uint32_t *stamp = (uint32_t *)(dist + k);
  int32_t *q0 = (int32_t *)(stamp + k);
  int32_t *q1 = q0 + k;
  for (int32_t s = blockIdx.x; s < k; s += gridDim.x) sssp_block(k, rp, col, w, s, dist, stamp, q0, q1, phi);
}

int grid_for(int32_t k) { return k < 1024 ? k : 1024; }

// Fresh control block (a kernel rather than a memset node, so that a caller
// may capture the call in a graph).
__global__ void k_zero_ctl(ECtl *ctl) {
  if (threadIdx.x == 0) { ctl->phi = 0; ctl->bad = 0; ctl->pad = 0; }
}

// Checks, APSP and readback, with the control block and the per-workgroup
// slices already placed; `grid` workgroups take the sources in turn.
int estimate_run(int32_t k, int64_t qm, const int64_t *rp, const int32_t *col, const uint64_t *w, uint64_t radius,
                 uint64_t *h_phi_gc, uint64_t *h_phi_approx, ECtl *ctl, char *slices, int grid, hipStream_t stream) {
  k_zero_ctl<<<1, 64, 0, stream>>>(ctl);
  CLD_LAUNCH_CHECK("k_zero_ctl");
  k_check_quotient<<<cld::blocks_for(k > qm ? (int64_t)k : qm, kT, 1024), kT, 0, stream>>>(k, qm, rp, col,
                                                                                           &ctl->bad);
  CLD_LAUNCH_CHECK("k_check_quotient");
  if (k <= kLdsMaxK) {
    k_apsp_lds<<<grid_for(k), kT, (size_t)k * 20, stream>>>(k, rp, col, w, (uint64_t *)&ctl->phi, &ctl->bad);
  } else {
    k_apsp_global<<<grid, kT, 0, stream>>>(k, rp, col, w, (uint64_t *)&ctl->phi, slices, &ctl->bad);
  }
  CLD_LAUNCH_CHECK("k_apsp");
  ECtl h;
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  if (h.bad) {
    cld::set_error("estimate_diameter: malformed quotient CSR (row offsets or a column out of range)");
    return CLDIAM_EINVAL;
  }
  *h_phi_gc = h.phi;
  *h_phi_approx = h.phi + 2 * radius;
  return CLDIAM_OK;
}

// ----------------------------------------------- no-allocation variant --
// Scratch of cldiam_estimate_diameter_noalloc: the control block at offset 0,
// then the per-workgroup APSP slices of quotients above kLdsMaxK nodes.  Each
// device holds its own copy from the library's load until the process ends.
constexpr size_t kStaticBytes = (size_t)32 << 20;
constexpr size_t kStaticCtl = 256;
static_assert(sizeof(ECtl) <= kStaticCtl, "control block fits its slot");
static __device__ __align__(256) char scratch[kStaticBytes];

// Device address of `scratch` on each device, resolved once per device with
// that device current (the host-side name is not a device address).
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;

int scratch_on_current_device(char **out) {
  int dev = 0, count = 0;
  CLD_HIP(hipGetDevice(&dev));
  CLD_HIP(hipGetDeviceCount(&count));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() < count) g_scratch_ptr.resize(count, nullptr);
  if (dev < 0 || dev >= count) { cld::set_error("estimate_diameter_noalloc: no current device"); return CLDIAM_EHIP; }
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    CLD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return CLDIAM_OK;
}

}  // namespace

extern "C" size_t cldiam_estimate_workspace_size(int32_t k, int64_t qm) {
  (void)qm;
  if (k < 1) return 0;
  size_t s = 256;
  if (k > kLdsMaxK) s += (size_t)k * 20 * grid_for(k) + 256;
  return s;
}

extern "C" int cldiam_estimate_diameter(int32_t k, int64_t qm, const int64_t *d_qrow_ptr, const int32_t *d_qcol,
                                        const uint64_t *d_qw, uint64_t radius, uint64_t *h_phi_gc,
                                        uint64_t *h_phi_approx, void *ws, size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (k < 1 || qm < 0 || !d_qrow_ptr || (qm && (!d_qcol || !d_qw)) || !h_phi_gc || !h_phi_approx) {
    cld::set_error("estimate_diameter: invalid arguments");
    return CLDIAM_EINVAL;
  }
  cld::Arena a(ws, ws_bytes);
  ECtl *ctl = a.take<ECtl>(1);
  char *slices = nullptr;
  if (k > kLdsMaxK) slices = a.take<char>((size_t)k * 20 * grid_for(k));
  if (!ctl || (k > kLdsMaxK && !slices)) {
    cld::set_error("estimate_diameter: workspace of %zu bytes, %zu needed", ws_bytes,
                   cldiam_estimate_workspace_size(k, qm));
    return CLDIAM_ENOMEM;
  }
  return estimate_run(k, qm, d_qrow_ptr, d_qcol, d_qw, radius, h_phi_gc, h_phi_approx, ctl, slices, grid_for(k),
                      stream);
}

extern "C" int cldiam_estimate_diameter_noalloc(int32_t k, int64_t qm, const int64_t *d_qrow_ptr,
                                                const int32_t *d_qcol, const uint64_t *d_qw, uint64_t radius,
                                                uint64_t *h_phi_gc, uint64_t *h_phi_approx, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (k < 1 || qm < 0 || !d_qrow_ptr || (qm && (!d_qcol || !d_qw)) || !h_phi_gc || !h_phi_approx) {
    cld::set_error("estimate_diameter_noalloc: invalid arguments");
    return CLDIAM_EINVAL;
  }
  if (k > CLDIAM_NOALLOC_MAX_K) {
    cld::set_error("estimate_diameter_noalloc: k = %d above the maximum %d of the static scratch", k,
                   CLDIAM_NOALLOC_MAX_K);
    return CLDIAM_EINVAL;
  }
  char *base = nullptr;
  int rc = scratch_on_current_device(&base);
  if (rc) return rc;
  // as many workgroups as the slices that fit (at least 1 for every k up to the maximum)
  int grid = grid_for(k);
  if (k > kLdsMaxK) {
    const size_t fit = (kStaticBytes - kStaticCtl) / ((size_t)k * 20);
    if ((size_t)grid > fit) grid = (int)fit;
  }
  return estimate_run(k, qm, d_qrow_ptr, d_qcol, d_qw, radius, h_phi_gc, h_phi_approx, (ECtl *)base,
                      base + kStaticCtl, grid, stream);
}
