// Weighted quotient graph G_C (Section 4 of arXiv:1506.03265).
//
// Clusters are numbered densely by ascending center id (a scan over the
// center flags).  Every arc u->v of G whose endpoints lie in different
// clusters emits the pair key (a, b) = (cluster index of u, of v), packed as
// a << kb | b with kb = bits of k-1, and the weight w(u,v) + D_u + D_v.  A
// radix sort over the 2*kb key bits groups equal pairs; the first element of
// each run marks a quotient arc and an atomic minimum over the run keeps the
// lightest parallel edge.  Because both arcs of every edge are emitted, the
// sorted unique pairs are directly the symmetric CSR of G_C with rows sorted
// by column.
#include <vector>

#include "common.h"

namespace cld {
size_t scan_ws_bytes(int64_t n);
size_t radix_ws_bytes(int64_t n);
int scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total, void *ws, size_t ws_bytes,
                       hipStream_t stream);
int radix_sort_u64(uint64_t *keys, uint64_t *vals, int64_t n, int begin_bit, int end_bit, uint64_t *ktmp,
                   uint64_t *vtmp, bool *in_tmp, void *ws, size_t ws_bytes, hipStream_t stream);
}  // namespace cld

namespace {

constexpr int kT = 256;

struct QCtl {
  uint32_t k;
  uint32_t pairs;   // emitted arcs
  uint32_t uniq;    // quotient arcs
  uint32_t pad;
};

__global__ void k_center_flags(const int32_t *cluster, int32_t n, uint32_t *flag) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    flag[v] = cluster[v] == (int32_t)v ? 1u : 0u;
}

__global__ void k_center_list(const int32_t *cluster, int32_t n, const uint32_t *dense, int32_t *qcenter) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (cluster[v] == (int32_t)v) qcenter[dense[v]] = (int32_t)v;
}

// One thread per row; every inter-cluster arc appends (key, weight) through
// a wave-aggregated reservation.
__global__ void __launch_bounds__(kT) k_emit(const int32_t *rp, const uint64_t *arcs, int32_t n,
                                             const int32_t *cluster, const uint64_t *D, const uint32_t *dense,
                                             int kb, uint64_t *keys, uint64_t *vals, QCtl *ctl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole waves iterate together so that the reservation sees every lane
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t u = base + threadIdx.x;
    int32_t a = 0, a1 = 0, cu = -1;
    uint64_t du = 0, ka = 0;
    if (u < n) {
      a = rp[u];
      a1 = rp[u + 1];
      cu = cluster[u];
      du = D[u];
      ka = (uint64_t)dense[cu] << kb;
    }
    for (;;) {
      const bool live = a < a1;
      if (!__any(live)) break;
      bool emit = false;
      uint64_t key = 0, val = 0;
      if (live) {
        const uint64_t arc = arcs[a];
        const int32_t v = (int32_t)(uint32_t)arc;
        const int32_t cv = cluster[v];
        if (cv != cu) {
          emit = true;
          key = ka | (uint64_t)dense[cv];
          val = (arc >> 32) + du + D[v];
        }
        ++a;
      }
      const uint32_t slot = cld_wave_reserve(emit, &ctl->pairs);
      if (emit) { keys[slot] = key; vals[slot] = val; }
    }
  }
}

__global__ void k_heads(const uint64_t *keys, int64_t P, uint32_t *head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_fill_inf(uint64_t *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = CLD_INF64;
}

// Run minimum into the unique slot; heads also write the column and fill the
// row offsets of every row in (previous row, this row].
__global__ void k_reduce_runs(const uint64_t *keys, const uint64_t *vals, int64_t P, const uint32_t *head,
                              const uint32_t *idx, int kb, int32_t *qcol, uint64_t *qw, int64_t *qrp) {
  const uint64_t bmask = (kb >= 64) ? ~0ull : ((1ull << kb) - 1ull);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = idx[i] + head[i] - 1;  // unique slot of this run
    atomicMin((unsigned long long *)&qw[j], (unsigned long long)vals[i]);
    if (head[i]) {
      qcol[j] = (int32_t)(keys[i] & bmask);
      const int64_t row = (int64_t)(keys[i] >> kb);
      const int64_t prev = (i == 0) ? -1 : (int64_t)(keys[i - 1] >> kb);
      for (int64_t r = prev + 1; r <= row; ++r) qrp[r] = j;
    }
  }
}

__global__ void k_tail_rows(const uint64_t *keys, int64_t P, int kb, int32_t k, uint32_t uniq, int64_t *qrp) {
  const int64_t last = P > 0 ? (int64_t)(keys[P - 1] >> kb) : -1;
  for (int64_t r = last + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= k;
       r += (int64_t)gridDim.x * blockDim.x)
    qrp[r] = uniq;
}

int bits_for(uint32_t x) {  // bits needed for values 0..x
  int b = 1;
  while (b < 32 && (x >> b) != 0) ++b;
  return b;
}

template <class A>
void carve(A &a, int32_t n, int64_t m, uint32_t **flag, uint32_t **dense, QCtl **ctl, uint64_t **keys,
           uint64_t **vals, uint64_t **ktmp, uint64_t **vtmp, uint32_t **head, uint32_t **idx) {
  *ctl = a.template take<QCtl>(1);
  *flag = a.template take<uint32_t>((size_t)n);
  *dense = a.template take<uint32_t>((size_t)n);
  *keys = a.template take<uint64_t>((size_t)m + 1);
  *vals = a.template take<uint64_t>((size_t)m + 1);
  *ktmp = a.template take<uint64_t>((size_t)m + 1);
  *vtmp = a.template take<uint64_t>((size_t)m + 1);
  *head = a.template take<uint32_t>((size_t)m + 1);
  *idx = a.template take<uint32_t>((size_t)m + 1);
}

struct SizeA {
  cld::Sizer s;
  template <class T>
  T *take(size_t n) { s.take<T>(n); return nullptr; }
};

}  // namespace

extern "C" size_t cldiam_quotient_workspace_size(int32_t n, int64_t m) {
  if (n < 1 || m < 0) return 0;
  SizeA s;
  uint32_t *f, *d, *h, *x;
  QCtl *c;
  uint64_t *k, *v, *kt, *vt;
  carve(s, n, m, &f, &d, &c, &k, &v, &kt, &vt, &h, &x);
  size_t extra = cld::radix_ws_bytes(m + 1);
  size_t sc = cld::scan_ws_bytes((int64_t)n > m + 1 ? (int64_t)n : m + 1);
  return s.s.used + (extra > sc ? extra : sc);
}

extern "C" int cldiam_build_quotient(int32_t n, int64_t m, const int32_t *d_row_ptr, const uint64_t *d_arcs,
                                     const int32_t *d_cluster, const uint64_t *d_D, int32_t *d_qcenter,
                                     int64_t *d_qrow_ptr, int32_t *d_qcol, uint64_t *d_qw, int32_t *h_k,
                                     int64_t *h_qm, void *ws, size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (n < 1 || m < 0 || m >= ((int64_t)1 << 31) || !d_row_ptr || (m && !d_arcs) || !d_cluster || !d_D ||
      !d_qcenter || !d_qrow_ptr || !h_k || !h_qm) {
    cld::set_error("build_quotient: invalid arguments");
    return CLDIAM_EINVAL;
  }
  cld::Arena a(ws, ws_bytes);
  uint32_t *flag, *dense, *head, *idx;
  QCtl *ctl;
  uint64_t *keys, *vals, *ktmp, *vtmp;
  carve(a, n, m, &flag, &dense, &ctl, &keys, &vals, &ktmp, &vtmp, &head, &idx);
  if (!idx || a.used > ws_bytes) {
    cld::set_error("build_quotient: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_quotient_workspace_size(n, m));
    return CLDIAM_ENOMEM;
  }
  void *rest = a.base + a.used;
  const size_t rest_bytes = a.cap - a.used;
  CLD_HIP(hipMemsetAsync(ctl, 0, sizeof(QCtl), stream));
  k_center_flags<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(d_cluster, n, flag);
  CLD_LAUNCH_CHECK("k_center_flags");
  int rc = cld::scan_exclusive_u32(flag, dense, n, &ctl->k, rest, rest_bytes, stream);
  if (rc) return rc;
  k_center_list<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(d_cluster, n, dense, d_qcenter);
  CLD_LAUNCH_CHECK("k_center_list");
  QCtl h;
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  const int32_t k = (int32_t)h.k;
  const int kb = bits_for(k > 0 ? (uint32_t)(k - 1) : 0u);
  if (m > 0) {
    k_emit<<<cld::blocks_for(n, kT, 16384), kT, 0, stream>>>(d_row_ptr, d_arcs, n, d_cluster, d_D,
                                                                          dense, kb, keys, vals, ctl);
    CLD_LAUNCH_CHECK("k_emit");
  }
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  const int64_t P = h.pairs;
  bool in_tmp = false;
  rc = cld::radix_sort_u64(keys, vals, P, 0, 2 * kb, ktmp, vtmp, &in_tmp, rest, rest_bytes, stream);
  if (rc) return rc;
  const uint64_t *sk = in_tmp ? ktmp : keys;
  const uint64_t *sv = in_tmp ? vtmp : vals;
  uint32_t uniq = 0;
  if (P > 0) {
    k_heads<<<cld::blocks_for(P, kT, 8192), kT, 0, stream>>>(sk, P, head);
    CLD_LAUNCH_CHECK("k_heads");
    rc = cld::scan_exclusive_u32(head, idx, P, &ctl->uniq, rest, rest_bytes, stream);
    if (rc) return rc;
    CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    uniq = h.uniq;
    k_fill_inf<<<cld::blocks_for(uniq, kT, 8192), kT, 0, stream>>>(d_qw, uniq);
    CLD_LAUNCH_CHECK("k_fill_inf");
    k_reduce_runs<<<cld::blocks_for(P, kT, 8192), kT, 0, stream>>>(sk, sv, P, head, idx, kb, d_qcol, d_qw,
                                                                    d_qrow_ptr);
    CLD_LAUNCH_CHECK("k_reduce_runs");
  }
  k_tail_rows<<<cld::blocks_for((int64_t)k + 1, kT, 4096), kT, 0, stream>>>(sk, P, kb, k, uniq, d_qrow_ptr);
  CLD_LAUNCH_CHECK("k_tail_rows");
  CLD_HIP(hipStreamSynchronize(stream));
  *h_k = k;
  *h_qm = uniq;
  return CLDIAM_OK;
}
