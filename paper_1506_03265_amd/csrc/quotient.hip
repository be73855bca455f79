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
  unsigned long long pairs;   // emitted arcs
  uint32_t k;
  uint32_t uniq;    // quotient arcs
  uint32_t wide;    // some D does not fit the packed node word
  uint32_t bad;     // some label is out of range or not a center
};

// Center flags; a label that is out of range or names a node that is not its
// own center is reported (the caller then gets CLDIAM_EINVAL, no kernel
// indexes with it).
__global__ void k_center_flags(const int32_t *cluster, int32_t n, uint32_t *flag, QCtl *ctl) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = cluster[v];
    flag[v] = c == (int32_t)v ? 1u : 0u;
    if ((uint32_t)c >= (uint32_t)n || cluster[c] != c) ctl->bad = 1u;
  }
}

__device__ __forceinline__ int bits_for_dev(uint32_t x) {  // bits needed for values 0..x, at least 1
  return x ? 32 - __clz(x) : 1;
}

// Node word of the packed emission: the dense cluster index in the top kb
// bits (kb = bits of k-1, k counted by the scan), D in the low 64 - kb bits,
// so that an arc's far end costs one 8-byte gather instead of three.  A D
// that does not fit sets ctl->wide, and the emission then reads the plain
// arrays instead.
__global__ void k_pack_nodes(const int32_t *cluster, const uint64_t *D, const uint32_t *dense, int32_t n,
                             QCtl *ctl, uint64_t *pk) {
  const uint32_t k = ctl->k;
  const int lb = 64 - bits_for_dev(k > 0 ? k - 1 : 0u);
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = D[v];
    const int32_t c = cluster[v];
    if (d >> lb) ctl->wide = 1u;
    pk[v] = (uint32_t)c < (uint32_t)n ? ((uint64_t)dense[c] << lb) | d : 0ull;   // bad labels fail the call
  }
}

__global__ void k_center_list(const int32_t *cluster, int32_t n, const uint32_t *dense, int32_t *qcenter) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (cluster[v] == (int32_t)v) qcenter[dense[v]] = (int32_t)v;
}

// Emission of inter-cluster arcs.  Each workgroup takes a contiguous range of
// rows; rows of up to kEmitThreadDeg arcs are walked by one thread, longer rows
// are deferred to LDS and walked by one wave (64 arcs per step) or, above
// kEmitBlockDeg, by the whole workgroup.  Every pair (key, weight) first goes
// into an LDS hash table of the workgroup that keeps the minimum weight per key
// (the same minimum the quotient keeps), so only distinct pairs reach global
// memory: the table is written out, with one global reservation, whenever it
// is half full after a round and at the end.  A pair that finds no slot after
// a few probes goes straight to global memory.
constexpr int kEmitThreads = 1024;
constexpr int kEmitThreadDeg = 16;
constexpr int kEmitBlockDeg = 4096;
constexpr int kEmitDefer = 512;     // deferred rows per round
constexpr int kHashCap = 4096;      // LDS hash slots (power of two)
constexpr int kHashProbes = 16;

struct EmitState {
  unsigned long long hkey[kHashCap];
  unsigned long long hval[kHashCap];
  int32_t mid[kEmitDefer];
  int32_t big[kEmitDefer];
  unsigned long long base;
  uint32_t nmid, nbig, used, cursor;
};

__device__ __forceinline__ uint32_t hash_slot(uint64_t key) {
  uint64_t x = key * 0x9E3779B97F4A7C15ull;
  return (uint32_t)(x >> 40) & (kHashCap - 1);
}

__device__ __forceinline__ void emit_pair(EmitState &E, uint64_t key, uint64_t val, uint64_t *keys, uint64_t *vals,
                                          QCtl *ctl) {
  uint32_t h = hash_slot(key);
  for (int p = 0; p < kHashProbes; ++p) {
    const unsigned long long k = atomicCAS(&E.hkey[h], ~0ull, (unsigned long long)key);
    if (k == ~0ull) atomicAdd(&E.used, 1u);
    if (k == ~0ull || k == key) {
      atomicMin(&E.hval[h], (unsigned long long)val);
      return;
    }
    h = (h + 1) & (kHashCap - 1);
  }
  const unsigned long long at = atomicAdd(&ctl->pairs, 1ull);
  keys[at] = key;
  vals[at] = val;
}

__device__ void hash_flush(EmitState &E, uint64_t *keys, uint64_t *vals, QCtl *ctl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    E.base = E.used ? atomicAdd(&ctl->pairs, (unsigned long long)E.used) : 0ull;
    E.cursor = 0;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHashCap; i += blockDim.x) {
    if (E.hkey[i] != ~0ull) {
      const unsigned long long at = E.base + atomicAdd(&E.cursor, 1u);
      keys[at] = E.hkey[i];
      vals[at] = E.hval[i];
      E.hkey[i] = ~0ull;
      E.hval[i] = ~0ull;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) E.used = 0;
  __syncthreads();
}

// One pending pair per thread, in registers.  A stage has few clusters, so
// consecutive arcs of a row mostly lead to the same cluster: their pairs fold
// here and only a change of key touches the LDS table (whose random slots
// cost bank conflicts).  Flushed at the end of each row part.
struct PairCache {
  uint64_t key = ~0ull, val = ~0ull;
};

__device__ __forceinline__ void cache_pair(PairCache &pc, uint64_t key, uint64_t val, EmitState &E, uint64_t *keys,
                                           uint64_t *vals, QCtl *ctl) {
  if (key == pc.key) {
    if (val < pc.val) pc.val = val;
    return;
  }
  if (pc.key != ~0ull) emit_pair(E, pc.key, pc.val, keys, vals, ctl);
  pc.key = key;
  pc.val = val;
}

__device__ __forceinline__ void cache_flush(PairCache &pc, EmitState &E, uint64_t *keys, uint64_t *vals, QCtl *ctl) {
  if (pc.key != ~0ull) emit_pair(E, pc.key, pc.val, keys, vals, ctl);
  pc.key = ~0ull;
}

// Node-side inputs of the emission: either cluster ids, D and the dense
// numbering, or the packed words of k_pack_nodes.
struct NodeIn {
  const int32_t *cluster;
  const uint64_t *D;
  const uint32_t *dense;
  const uint64_t *pk;
  int lb;
};

// Cluster tag (cluster id, or dense index when packed), D and the key's
// high part of node u.
template <bool kPacked>
__device__ __forceinline__ void node_of(const NodeIn &in, int32_t u, int kb, uint32_t *cu, uint64_t *du,
                                        uint64_t *ka) {
  if (kPacked) {
    const uint64_t x = in.pk[u];
    *cu = (uint32_t)(x >> in.lb);
    *du = x & ((1ull << in.lb) - 1ull);
    *ka = (uint64_t)*cu << kb;
  } else {
    *cu = (uint32_t)in.cluster[u];
    *du = in.D[u];
    *ka = (uint64_t)in.dense[*cu] << kb;
  }
}

// The graph is symmetric with equal weights both ways and w + D_u + D_v is
// symmetric, so each edge is taken once, from its smaller end (u < v), and
// gives both directed pairs: half the far-end gathers of walking every arc.
// pc folds the pairs out of u's cluster, rc those into it.
template <bool kPacked>
__device__ __forceinline__ void emit_arc(uint64_t arc, int32_t u, uint32_t cu, uint64_t du, uint64_t ka, int kb,
                                         const NodeIn &in, PairCache &pc, PairCache &rc, EmitState &E,
                                         uint64_t *keys, uint64_t *vals, QCtl *ctl) {
  const int32_t v = (int32_t)(uint32_t)arc;
  if (v < u) return;
  const uint64_t da = ka >> kb;   // dense index of u's cluster
  uint64_t db, val;
  if (kPacked) {
    const uint64_t x = in.pk[v];
    const uint32_t cv = (uint32_t)(x >> in.lb);
    if (cv == cu) return;
    db = cv;
    val = (arc >> 32) + du + (x & ((1ull << in.lb) - 1ull));
  } else {
    const int32_t cv = in.cluster[v];
    if ((uint32_t)cv == cu) return;
    db = in.dense[cv];
    val = (arc >> 32) + du + in.D[v];
  }
  cache_pair(pc, ka | db, val, E, keys, vals, ctl);
  cache_pair(rc, (db << kb) | da, val, E, keys, vals, ctl);
}

template <bool kPacked>
__global__ void __launch_bounds__(kEmitThreads) k_emit(const int64_t *rp, const uint64_t *arcs, int32_t n, NodeIn in,
                                                       int kb, uint64_t *keys, uint64_t *vals, QCtl *ctl) {
  __shared__ EmitState E;
  for (uint32_t i = threadIdx.x; i < kHashCap; i += blockDim.x) { E.hkey[i] = ~0ull; E.hval[i] = ~0ull; }
  if (threadIdx.x == 0) { E.nmid = 0; E.nbig = 0; E.used = 0; }
  __syncthreads();
  const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int64_t r = lo; r < hi; r += blockDim.x) {
    const int64_t u = r + threadIdx.x;
    if (u < hi) {
      const int64_t a0 = rp[u];
      const int32_t deg = (int32_t)(rp[u + 1] - a0);
      bool done = false;
      if (deg > kEmitThreadDeg) {
        uint32_t *cnt = deg > kEmitBlockDeg ? &E.nbig : &E.nmid;
        int32_t *lst = deg > kEmitBlockDeg ? E.big : E.mid;
        const uint32_t slot = atomicAdd(cnt, 1u);
        if (slot < kEmitDefer) { lst[slot] = (int32_t)u; done = true; }
      }
      if (!done) {
        uint32_t cu;
        uint64_t du, ka;
        node_of<kPacked>(in, (int32_t)u, kb, &cu, &du, &ka);
        const uint64_t *row = arcs + a0;
        PairCache pc, rc;
        for (int32_t a = 0; a < deg; ++a)
          emit_arc<kPacked>(row[a], (int32_t)u, cu, du, ka, kb, in, pc, rc, E, keys, vals, ctl);
        cache_flush(pc, E, keys, vals, ctl);
        cache_flush(rc, E, keys, vals, ctl);
      }
    }
    __syncthreads();
    const uint32_t nm = E.nmid < kEmitDefer ? E.nmid : kEmitDefer;
    for (uint32_t i = wave; i < nm; i += nwaves) {
      const int32_t u = E.mid[i];
      const int64_t a0 = rp[u];
      const int32_t deg = (int32_t)(rp[u + 1] - a0);
      const uint64_t *row = arcs + a0;
      uint32_t cu;
      uint64_t du, ka;
      node_of<kPacked>(in, u, kb, &cu, &du, &ka);
      PairCache pc, rc;
      for (int32_t a = (int32_t)lane; a < deg; a += 64)
        emit_arc<kPacked>(row[a], u, cu, du, ka, kb, in, pc, rc, E, keys, vals, ctl);
      cache_flush(pc, E, keys, vals, ctl);
      cache_flush(rc, E, keys, vals, ctl);
    }
    const uint32_t nbg = E.nbig < kEmitDefer ? E.nbig : kEmitDefer;
    for (uint32_t i = 0; i < nbg; ++i) {
      const int32_t u = E.big[i];
      const int64_t a0 = rp[u];
      const int32_t deg = (int32_t)(rp[u + 1] - a0);
      const uint64_t *row = arcs + a0;
      uint32_t cu;
      uint64_t du, ka;
      node_of<kPacked>(in, u, kb, &cu, &du, &ka);
      PairCache pc, rc;
      for (int32_t a = (int32_t)threadIdx.x; a < deg; a += (int32_t)blockDim.x)
        emit_arc<kPacked>(row[a], u, cu, du, ka, kb, in, pc, rc, E, keys, vals, ctl);
      cache_flush(pc, E, keys, vals, ctl);
      cache_flush(rc, E, keys, vals, ctl);
      __syncthreads();
      if (E.used > kHashCap / 2) hash_flush(E, keys, vals, ctl);
    }
    __syncthreads();
    if (threadIdx.x == 0) { E.nmid = 0; E.nbig = 0; }
    __syncthreads();
    if (E.used > kHashCap / 2) hash_flush(E, keys, vals, ctl);
  }
  hash_flush(E, keys, vals, ctl);
}

__global__ void k_heads(const uint64_t *keys, int64_t P, uint32_t *head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_fill_inf(uint64_t *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = CLD_INF64;
}

// Run minimum into the unique slot, one chunk of kRunChunk consecutive
// elements per thread: one atomic per (run, chunk) piece.  Heads also write the
// column and fill the row offsets of every row in (previous row, this row].
constexpr int kRunChunk = 64;

__global__ void k_reduce_runs(const uint64_t *keys, const uint64_t *vals, int64_t P, const uint32_t *head,
                              const uint32_t *idx, int kb, int32_t *qcol, uint64_t *qw, int64_t *qrp) {
  const uint64_t bmask = (kb >= 64) ? ~0ull : ((1ull << kb) - 1ull);
  const int64_t chunks = (P + kRunChunk - 1) / kRunChunk;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < chunks; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = c * kRunChunk, e = b + kRunChunk < P ? b + kRunChunk : P;
    uint32_t slot = idx[b] + head[b] - 1;
    uint64_t best = vals[b];
    for (int64_t i = b; i < e; ++i) {
      if (head[i]) {
        if (i > b) atomicMin((unsigned long long *)&qw[slot], (unsigned long long)best);
        slot = idx[i];
        best = vals[i];
        qcol[slot] = (int32_t)(keys[i] & bmask);
        const int64_t row = (int64_t)(keys[i] >> kb);
        const int64_t prev = (i == 0) ? -1 : (int64_t)(keys[i - 1] >> kb);
        for (int64_t r = prev + 1; r <= row; ++r) qrp[r] = slot;
      } else if (vals[i] < best) {
        best = vals[i];
      }
    }
    atomicMin((unsigned long long *)&qw[slot], (unsigned long long)best);
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

constexpr int kEmitBlocks = 2048;

template <class A>
void carve(A &a, int32_t n, int64_t m, uint32_t **flag, uint32_t **dense, QCtl **ctl, uint64_t **keys,
           uint64_t **vals, uint64_t **ktmp, uint64_t **vtmp, uint32_t **head, uint32_t **idx, uint64_t **pk) {
  *ctl = a.template take<QCtl>(1);
  *pk = a.template take<uint64_t>((size_t)n);
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
  uint64_t *pk;
  carve(s, n, m, &f, &d, &c, &k, &v, &kt, &vt, &h, &x, &pk);
  size_t extra = cld::radix_ws_bytes(m + 1);
  size_t sc = cld::scan_ws_bytes((int64_t)n > m + 1 ? (int64_t)n : m + 1);
  return s.s.used + (extra > sc ? extra : sc);
}

extern "C" int cldiam_build_quotient(int32_t n, int64_t m, const int64_t *d_row_ptr, const uint64_t *d_arcs,
                                     const int32_t *d_cluster, const uint64_t *d_D, int32_t *d_qcenter,
                                     int64_t *d_qrow_ptr, int32_t *d_qcol, uint64_t *d_qw, int32_t *h_k,
                                     int64_t *h_qm, void *ws, size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (n < 1 || m < 0 || m >= ((int64_t)1 << 40) || !d_row_ptr || (m && !d_arcs) || !d_cluster || !d_D ||
      !d_qcenter || !d_qrow_ptr || !h_k || !h_qm) {
    cld::set_error("build_quotient: invalid arguments");
    return CLDIAM_EINVAL;
  }
  cld::Arena a(ws, ws_bytes);
  uint32_t *flag, *dense, *head, *idx;
  QCtl *ctl;
  uint64_t *keys, *vals, *ktmp, *vtmp;
  uint64_t *pk;
  carve(a, n, m, &flag, &dense, &ctl, &keys, &vals, &ktmp, &vtmp, &head, &idx, &pk);
  if (!idx || a.used > ws_bytes) {
    cld::set_error("build_quotient: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_quotient_workspace_size(n, m));
    return CLDIAM_ENOMEM;
  }
  void *rest = a.base + a.used;
  const size_t rest_bytes = a.cap - a.used;
  CLD_HIP(hipMemsetAsync(ctl, 0, sizeof(QCtl), stream));
  k_center_flags<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(d_cluster, n, flag, ctl);
  CLD_LAUNCH_CHECK("k_center_flags");
  int rc = cld::scan_exclusive_u32(flag, dense, n, &ctl->k, rest, rest_bytes, stream);
  if (rc) return rc;
  k_center_list<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(d_cluster, n, dense, d_qcenter);
  CLD_LAUNCH_CHECK("k_center_list");
  if (m > 0) {
    k_pack_nodes<<<cld::blocks_for(n, kT, 8192), kT, 0, stream>>>(d_cluster, d_D, dense, n, ctl, pk);
    CLD_LAUNCH_CHECK("k_pack_nodes");
  }
  QCtl h;
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  if (h.bad) {
    cld::set_error("build_quotient: a cluster label is out of range or not a center (cluster[c] != c)");
    return CLDIAM_EINVAL;
  }
  const int32_t k = (int32_t)h.k;
  const int kb = bits_for(k > 0 ? (uint32_t)(k - 1) : 0u);
  if (m > 0) {
    const unsigned eb = (unsigned)(n < kEmitBlocks * 64 ? (n + 63) / 64 : kEmitBlocks);
    NodeIn in{d_cluster, d_D, dense, pk, 64 - kb};
    if (!h.wide) {   // every D fits beside the cluster index
      k_emit<true><<<eb, kEmitThreads, 0, stream>>>(d_row_ptr, d_arcs, n, in, kb, keys, vals, ctl);
    } else {
      k_emit<false><<<eb, kEmitThreads, 0, stream>>>(d_row_ptr, d_arcs, n, in, kb, keys, vals, ctl);
    }
    CLD_LAUNCH_CHECK("k_emit");
  }
  CLD_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  const int64_t P = (int64_t)h.pairs;
  if (P >= (int64_t)0xffffffff) {
    cld::set_error("build_quotient: %lld distinct cluster pairs exceed the 2^32 - 1 the run numbering holds",
                   (long long)P);
    return CLDIAM_EOVERFLOW;
  }
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
    k_reduce_runs<<<cld::blocks_for((P + kRunChunk - 1) / kRunChunk, kT, 8192), kT, 0, stream>>>(sk, sv, P, head, idx, kb, d_qcol, d_qw,
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
