// Graph ingest: CSR validation and packing of weight-sorted arcs.
//
// The graph model of Section 2 is an undirected graph with positive integer
// weights.  A symmetric CSR is validated (columns in range, rows strictly
// increasing, no self loops, weights >= 1, every arc matched by its reverse
// with the same weight) and each arc is packed as (w << 32) | col.  Rows are
// then re-sorted by (w, col) so that the light arcs of a node (w <= Delta,
// Section 3) are a prefix of its row, and the heavy ones a suffix.
#include <string.h>

#include <vector>

#include "common.h"

namespace cld {
size_t scan_ws_bytes(int64_t n);
size_t radix_ws_bytes(int64_t n);
int radix_sort_u64(uint64_t *keys, uint64_t *vals, int64_t n, int begin_bit, int end_bit, uint64_t *ktmp,
                   uint64_t *vtmp, bool *in_tmp, void *ws, size_t ws_bytes, hipStream_t stream);
}  // namespace cld

namespace {

constexpr int kT = 256;
constexpr int kSmallRow = 32;     // thread-per-row insertion sort
constexpr int kLdsRow = 8192;     // block-per-row bitonic sort in LDS
constexpr int64_t kBatchArcs = (int64_t)1 << 26;   // hub-row arcs sorted together (at least n)

enum : uint32_t {
  BAD_ROWPTR = 1, BAD_COL = 2, BAD_SELF = 4, BAD_ORDER = 8, BAD_WEIGHT = 16, BAD_ASYM = 32,
};

struct IngestCtl {
  uint32_t bad;
  uint32_t nmid, nbig;
  uint32_t pad;
  unsigned long long wsum;
};

__global__ void k_check_rows(const int64_t *rp, int32_t n, int64_t m, IngestCtl *ctl) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    bool ok = rp[i] <= rp[i + 1] && rp[i] >= 0 && rp[i + 1] <= m;
    if (i == 0) ok = ok && rp[0] == 0;
    if (i == n - 1) ok = ok && rp[n] == m;
    if (!ok) atomicOr(&ctl->bad, BAD_ROWPTR);
  }
}

// One wave per row: validates every arc of the row and packs it.
__global__ void __launch_bounds__(kT) k_validate_pack(const int64_t *rp, const int32_t *col, const uint32_t *w,
                                                      int32_t n, uint64_t *arcs, IngestCtl *ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t bad = 0;
  unsigned long long wsum = 0;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int64_t a0 = rp[u], a1 = rp[u + 1];
    for (int64_t a = a0 + lane; a < a1; a += 64) {
      const int32_t v = col[a];
      const uint32_t wt = w[a];
      wsum += wt;
      if (v < 0 || v >= n) { bad |= BAD_COL; continue; }
      if (v == u) bad |= BAD_SELF;
      if (a > a0 && col[a - 1] >= v) bad |= BAD_ORDER;
      if (wt == 0) bad |= BAD_WEIGHT;
      // reverse arc v -> u by binary search in row v (sorted by column)
      int64_t lo = rp[v], hi = rp[v + 1] - 1;
      bool found = false;
      while (lo <= hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const int32_t c = col[mid];
        if (c == (int32_t)u) { found = (w[mid] == wt); break; }
        if (c < (int32_t)u) lo = mid + 1; else hi = mid - 1;
      }
      if (!found) bad |= BAD_ASYM;
      arcs[a] = ((uint64_t)wt << 32) | (uint32_t)v;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    bad |= __shfl_xor(bad, o);
    wsum += __shfl_xor(wsum, o);
  }
  if (lane == 0) {
    if (bad) atomicOr(&ctl->bad, bad);
    if (wsum) atomicAdd(&ctl->wsum, wsum);
  }
}

// Small rows sorted in place by one thread; larger rows queued by size class.
__global__ void k_small_sort(const int64_t *rp, int32_t n, uint64_t *arcs, int32_t *mid, int32_t *big,
                             IngestCtl *ctl) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = rp[u], a1 = rp[u + 1], deg = a1 - a0;
    if (deg <= kSmallRow) {
      for (int64_t i = a0 + 1; i < a1; ++i) {
        const uint64_t x = arcs[i];
        int64_t j = i - 1;
        while (j >= a0 && arcs[j] > x) { arcs[j + 1] = arcs[j]; --j; }
        arcs[j + 1] = x;
      }
    } else if (deg <= kLdsRow) {
      mid[atomicAdd(&ctl->nmid, 1u)] = (int32_t)u;
    } else {
      big[atomicAdd(&ctl->nbig, 1u)] = (int32_t)u;
    }
  }
}

// One block per mid-size row: bitonic sort of the row in LDS.
__global__ void __launch_bounds__(1024) k_mid_sort(const int64_t *rp, const int32_t *rows, const IngestCtl *ctl,
                                                   uint64_t *arcs) {
  __shared__ uint64_t s[kLdsRow];
  for (uint32_t r = blockIdx.x; r < ctl->nmid; r += gridDim.x) {
    const int32_t u = rows[r];
    const int64_t a0 = rp[u];
    const int32_t deg = (int32_t)(rp[u + 1] - a0);
    int size = 1;
    while (size < deg) size <<= 1;
    for (int i = threadIdx.x; i < size; i += blockDim.x) s[i] = i < deg ? arcs[a0 + i] : ~(uint64_t)0;
    __syncthreads();
    for (int k = 2; k <= size; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < size; i += blockDim.x) {
          const int p = i ^ j;
          if (p > i) {
            const bool up = (i & k) == 0;
            const uint64_t x = s[i], y = s[p];
            if ((x > y) == up) { s[i] = y; s[p] = x; }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < deg; i += blockDim.x) arcs[a0 + i] = s[i];
    __syncthreads();
  }
}

// Rows longer than kLdsRow arcs are sorted in batches: their arcs are copied
// side by side (with the row's ordinal in the batch as value), radix-sorted by
// arc, then stably by ordinal, which regroups every row in place with its
// arcs in order; a batch holds up to the batch capacity of arcs.
struct BigRow {
  int64_t a0;      // first arc of the row
  uint32_t start;  // its first slot in the batch
  uint32_t deg;
};

__global__ void k_big_rows(const int64_t *rp, const int32_t *big, uint32_t nbig, int64_t *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nbig; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = big[i];
    out[2 * i] = rp[u];
    out[2 * i + 1] = rp[u + 1] - rp[u];
  }
}

__global__ void k_batch_gather(const uint64_t *arcs, const BigRow *rows, uint32_t nrows, uint64_t *key,
                               uint64_t *ord) {
  for (uint32_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const BigRow b = rows[r];
    for (uint32_t j = threadIdx.x; j < b.deg; j += blockDim.x) {
      key[b.start + j] = arcs[b.a0 + j];
      ord[b.start + j] = r;
    }
  }
}

__global__ void k_batch_scatter(uint64_t *arcs, const BigRow *rows, uint32_t nrows, const uint64_t *key) {
  for (uint32_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const BigRow b = rows[r];
    for (uint32_t j = threadIdx.x; j < b.deg; j += blockDim.x) arcs[b.a0 + j] = key[b.start + j];
  }
}

int64_t batch_cap(int32_t n, int64_t m) {
  const int64_t want = kBatchArcs > (int64_t)n ? kBatchArcs : (int64_t)n;   // every row fits one batch
  return m + 1 < want ? m + 1 : want;
}

int64_t big_rows_cap(int64_t m) { return m / (kLdsRow + 1) + 1; }

}  // namespace

extern "C" size_t cldiam_load_csr_workspace_size(int32_t n, int64_t m) {
  if (n < 1 || m < 0) return 0;
  cld::Sizer s;
  s.take<IngestCtl>(1);
  s.take<int32_t>((size_t)n);  // mid rows
  s.take<int32_t>((size_t)n);  // big rows
  const int64_t nb = big_rows_cap(m), B = batch_cap(n, m);
  s.take<int64_t>(2 * (size_t)nb);   // (offset, degree) of every big row
  s.take<BigRow>((size_t)nb);
  for (int i = 0; i < 4; ++i) s.take<uint64_t>((size_t)B);   // batch keys, ordinals and their radix buffers
  s.used += cld::radix_ws_bytes(B);
  return s.used;
}

extern "C" int cldiam_load_csr(const cldiam_csr *g, uint64_t *d_arcs, uint64_t *h_weight_sum, void *ws,
                               size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!g || g->n < 1 || g->m < 0 || g->m >= ((int64_t)1 << 40) || !g->d_row_ptr || (g->m && (!g->d_col || !g->d_w || !d_arcs))) {
    cld::set_error("load_csr: invalid arguments");
    return CLDIAM_EINVAL;
  }
  const int32_t n = g->n;
  const int64_t m = g->m;
  cld::Arena a(ws, ws_bytes);
  IngestCtl *ctl = a.take<IngestCtl>(1);
  int32_t *mid = a.take<int32_t>((size_t)n);
  int32_t *big = a.take<int32_t>((size_t)n);
  const int64_t nbcap = big_rows_cap(m), B = batch_cap(n, m);
  int64_t *binfo = a.take<int64_t>(2 * (size_t)nbcap);
  BigRow *brows = a.take<BigRow>((size_t)nbcap);
  uint64_t *bk = a.take<uint64_t>((size_t)B), *bo = a.take<uint64_t>((size_t)B);
  uint64_t *bkt = a.take<uint64_t>((size_t)B), *bot = a.take<uint64_t>((size_t)B);
  if (!ctl || !mid || !big || !binfo || !brows || !bk || !bo || !bkt || !bot) {
    cld::set_error("load_csr: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_load_csr_workspace_size(n, m));
    return CLDIAM_ENOMEM;
  }
  CLD_HIP(hipMemsetAsync(ctl, 0, sizeof(IngestCtl), stream));
  k_check_rows<<<cld::blocks_for(n, kT, 4096), kT, 0, stream>>>(g->d_row_ptr, n, m, ctl);
  CLD_LAUNCH_CHECK("k_check_rows");
  IngestCtl h;
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  if (h.bad) { cld::set_error("load_csr: malformed row offsets"); return CLDIAM_EINVAL; }
  if (m > 0) {
    k_validate_pack<<<cld::blocks_for((int64_t)n * 64, kT, 16384), kT, 0, stream>>>(g->d_row_ptr, g->d_col, g->d_w,
                                                                                     n, d_arcs, ctl);
    CLD_LAUNCH_CHECK("k_validate_pack");
    CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (h.bad) {
      cld::set_error("load_csr: malformed CSR (flags 0x%x: 1 row offsets, 2 column range, 4 self loop, "
                     "8 row order, 16 zero weight, 32 not symmetric)", h.bad);
      return CLDIAM_EINVAL;
    }
    k_small_sort<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(g->d_row_ptr, n, d_arcs, mid, big, ctl);
    CLD_LAUNCH_CHECK("k_small_sort");
    CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (h.nmid) {
      k_mid_sort<<<h.nmid < 4096 ? h.nmid : 4096, 1024, 0, stream>>>(g->d_row_ptr, mid, ctl, d_arcs);
      CLD_LAUNCH_CHECK("k_mid_sort");
    }
    if (h.nbig) {
      if ((int64_t)h.nbig > nbcap) { cld::set_error("load_csr: hub row count out of range"); return CLDIAM_EHIP; }
      k_big_rows<<<cld::blocks_for(h.nbig, kT, 1024), kT, 0, stream>>>(g->d_row_ptr, big, h.nbig, binfo);
      CLD_LAUNCH_CHECK("k_big_rows");
      std::vector<int64_t> info(2 * (size_t)h.nbig);
      CLD_HIP(hipMemcpyAsync(info.data(), binfo, 16 * (size_t)h.nbig, hipMemcpyDeviceToHost, stream));
      CLD_HIP(hipStreamSynchronize(stream));
      // batches of whole rows, at most B arcs each (every row has at most n - 1 < B arcs)
      std::vector<BigRow> desc(h.nbig);
      std::vector<std::pair<uint32_t, uint32_t>> batches;   // (first row, row count)
      int64_t fill = 0;
      uint32_t first = 0;
      for (uint32_t i = 0; i < h.nbig; ++i) {
        const int64_t deg = info[2 * i + 1];
        if (fill + deg > B) {
          batches.push_back({first, i - first});
          first = i;
          fill = 0;
        }
        desc[i] = {info[2 * i], (uint32_t)fill, (uint32_t)deg};
        fill += deg;
      }
      batches.push_back({first, h.nbig - first});
      CLD_HIP(hipMemcpyAsync(brows, desc.data(), sizeof(BigRow) * desc.size(), hipMemcpyHostToDevice, stream));
      for (const auto &bt : batches) {
        const BigRow &last = desc[bt.first + bt.second - 1];
        const int64_t total = (int64_t)last.start + last.deg;
        int ob = 1;
        while (ob < 64 && (bt.second - 1) >> ob) ++ob;
        k_batch_gather<<<bt.second < 4096 ? bt.second : 4096, 1024, 0, stream>>>(d_arcs, brows + bt.first,
                                                                                bt.second, bk, bo);
        CLD_LAUNCH_CHECK("k_batch_gather");
        bool t1 = false, t2 = false;
        int rc = cld::radix_sort_u64(bk, bo, total, 0, 64, bkt, bot, &t1, a.base + a.used, a.cap - a.used, stream);
        if (rc) return rc;
        uint64_t *k1 = t1 ? bkt : bk, *o1 = t1 ? bot : bo, *k1t = t1 ? bk : bkt, *o1t = t1 ? bo : bot;
        // stable by ordinal: the ordinals are the keys now, the arcs ride along
        rc = cld::radix_sort_u64(o1, k1, total, 0, ob, o1t, k1t, &t2, a.base + a.used, a.cap - a.used, stream);
        if (rc) return rc;
        k_batch_scatter<<<bt.second < 4096 ? bt.second : 4096, 1024, 0, stream>>>(d_arcs, brows + bt.first,
                                                                                 bt.second, t2 ? k1t : k1);
        CLD_LAUNCH_CHECK("k_batch_scatter");
      }
      CLD_HIP(hipStreamSynchronize(stream));   // desc is read by the copies above
    }
  }
  CLD_HIP(hipStreamSynchronize(stream));
  if (h_weight_sum) *h_weight_sum = h.wsum;
  return CLDIAM_OK;
}
